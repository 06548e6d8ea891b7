// Variable-size batched FP64 GEMM on the CDNA4 matrix cores.
//
// Every small contraction of the left-looking TLR step (Section 4.1-4.3 of
// the paper: the four-product sampling of Eq. (2), its transpose for the
// projection, the dense diagonal update, the block Gram-Schmidt projections
// and the trailing updates of the tile factorizations) is a batch of GEMMs
// whose sizes differ from tile to tile, because the tile ranks are adaptive.
// The paper runs these through a non-uniform batched GEMM; this is the
// gfx950 one.
//
// Design: one 256-thread workgroup (4 wave64) per BM x BN output tile of one
// problem.  Operand tiles are staged through LDS in the natural column-major
// direction (so global loads coalesce whatever the transposition) and fed to
// v_mfma_f64_16x16x4f64.  A host-built block map assigns workgroups to
// (problem, tile) pairs, so problems of any shape share one launch.
#include <algorithm>

#include "mfma_tiles.h"
#include "tlr_internal.h"

namespace tlr {

namespace {

constexpr int BM = 64;
constexpr int PAD = 2;

// MFMA f64 16x16x4 operand layout (measured on gfx950): lane l supplies
// A(l % 16, l / 16) and B(l / 16, l % 16); accumulator register r of lane l
// holds D(l / 16 + 4 r, l % 16).
//
// BK is the depth of one K slice.  A slice's loads are in flight while the
// previous slice's MFMAs run, and with few workgroups (a long product over
// m = 1024 with only ~160 output tiles) every slice costs about one memory
// latency: long contractions take BK = 64, short ones (K <= 32) BK = 16.
template <bool TA, bool TB, int BN, int BK>
__global__ __launch_bounds__(256) void k_gemm(const GemmDesc* __restrict__ descs,
                                              const BlockMap* __restrict__ map) {
  static_assert(BK == 16 || BK == 32 || BK == 64, "slice depth");
  constexpr int WAVES_N = (BN == 64) ? 2 : 1;
  constexpr int WAVES_M = 4 / WAVES_N;
  constexpr int WM = BM / WAVES_M;   // rows per wave: 32 or 16
  constexpr int WN = BN / WAVES_N;   // cols per wave: 32 or 16
  constexpr int FM = WM / 16;
  constexpr int FN = WN / 16;

  __shared__ double sA[BK][BM + PAD];
  __shared__ double sB[BK][BN + PAD];

  const BlockMap bm = map[blockIdx.x];
  const GemmDesc d = descs[bm.desc];
  const int tiles_m = (d.M + BM - 1) / BM;
  const int row0 = (bm.tile % tiles_m) * BM;
  const int col0 = (bm.tile / tiles_m) * BN;
  if ((d.flags & GEMM_LOWER_C) && col0 >= row0 + BM) return;
  int kbeg = 0, kend = d.K;
  if (d.flags & GEMM_TRIL_A) kend = min(kend, row0 + BM - d.koff);
  if (d.flags & GEMM_TRIU_A) kbeg = (row0 / BK) * BK;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr0 = (wave % WAVES_M) * WM;
  const int wc0 = (wave / WAVES_M) * WN;
  const int li = lane & 15;
  const int lk = lane >> 4;

  d4 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  // Software pipeline: the global loads of slice k0 + BK are issued into
  // registers before the MFMAs of slice k0 run from LDS, so one memory
  // latency per slice is hidden behind the compute and the barriers.
  // op(A)(row0 + r, k0 + kk) is staged as 64 x 16, op(B)(k0 + kk, col0 + c)
  // as 16 x BN; every thread owns fixed (r, kk) / (kk, c) positions.
  // (the loads of a wave run down the stored columns: 64 rows of op(A) for
  // A, BK consecutive k for A^T and B, BN consecutive columns for B^T)
  constexpr int NAL = BM * BK / 256;
  constexpr int NBL = BK * BN / 256;
  int ar[NAL], ak[NAL], bc[NBL], bk[NBL];
#pragma unroll
  for (int j = 0; j < NAL; ++j) {
    if (!TA) { ar[j] = tid & 63; ak[j] = (tid >> 6) + 4 * j; }
    else     { ak[j] = tid % BK; ar[j] = tid / BK + (256 / BK) * j; }
  }
#pragma unroll
  for (int j = 0; j < NBL; ++j) {
    if (!TB) { bk[j] = tid % BK; bc[j] = tid / BK + (256 / BK) * j; }
    else     { bc[j] = tid % BN; bk[j] = tid / BN + (256 / BN) * j; }
  }
  double ra[NAL], rb[NBL];
  auto load = [&](int k0) {
#pragma unroll
    for (int j = 0; j < NAL; ++j) {
      const int gr = row0 + ar[j], gk = k0 + ak[j];
      double v = 0.0;
      if (gr < d.M && gk < d.K)
        v = TA ? gmem(d.A)[gk + (size_t)gr * d.lda] : gmem(d.A)[gr + (size_t)gk * d.lda];
      ra[j] = v;
    }
#pragma unroll
    for (int j = 0; j < NBL; ++j) {
      const int gc = col0 + bc[j], gk = k0 + bk[j];
      double v = 0.0;
      if (gc < d.N && gk < d.K)
        v = TB ? gmem(d.B)[gc + (size_t)gk * d.ldb] : gmem(d.B)[gk + (size_t)gc * d.ldb];
      rb[j] = v;
    }
  };
  if (kbeg < kend) load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int j = 0; j < NAL; ++j) sA[ak[j]][ar[j]] = ra[j];
#pragma unroll
    for (int j = 0; j < NBL; ++j) sB[bk[j]][bc[j]] = rb[j];
    __syncthreads();
    if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double av[FM], bv[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) av[a] = sA[ks + lk][wr0 + a * 16 + li];
#pragma unroll
      for (int b = 0; b < FN; ++b) bv[b] = sB[ks + lk][wc0 + b * 16 + li];
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }

  // ---- epilogue: C = alpha * acc + beta * C
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      const int gc = col0 + wc0 + b * 16 + li;
      if (gc >= d.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wr0 + a * 16 + lk + 4 * r;
        if (gr >= d.M) continue;
        gdouble* cp = gmem(d.C) + gr + (size_t)gc * d.ldc;
        double v = d.alpha * acc[a][b][r];
        if (d.beta != 0.0) v += d.beta * *cp;
        *cp = v;
      }
    }
}

// C = alpha A^T B + beta C with A stored K x M and B stored K x N (both
// column-major, the contraction runs down their columns): the projections
// U^T Omega, Q^T Y, V^T V, U^T Q of the method, where K is the tile height.
// A 512-thread workgroup owns a (16 FM) x (16 FN) tile of C (tn_tile).
template <int FM, int FN>
__global__ __launch_bounds__(512) void k_gemm_tn(const GemmDesc* __restrict__ descs,
                                                 const BlockMap* __restrict__ map) {
  constexpr int TM = 16 * FM, TN = 16 * FN, NW = 8;
  __shared__ double red[NW][FM * FN * 4][64];
  const BlockMap bm = map[blockIdx.x];
  const GemmDesc d = descs[bm.desc];
  const int tiles_m = (d.M + TM - 1) / TM;
  const int row0 = (bm.tile % tiles_m) * TM;
  const int col0 = (bm.tile / tiles_m) * TN;
  int kbeg = 0;
  if (d.flags & GEMM_TRIU_A) kbeg = (row0 / 16) * 16;
  tn_tile<FM, FN, NW>(d.A, d.lda, d.B, d.ldb, d.C, d.ldc, d.M, d.N, kbeg, d.K, d.alpha, d.beta, row0,
                      col0, red);
}

// The same product streamed through LDS with coalesced loads (tn_lds_tile):
// a BM x BN tile per 256-thread workgroup, 64-row chunks.  For problems
// with K >= 1 and no flags but GEMM_STORE_T.
template <int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm_tn_lds(const GemmDesc* __restrict__ descs,
                                                     const BlockMap* __restrict__ map) {
  constexpr int KC = 64;
  __shared__ double smem[tn_lds_smem<BM, BN, KC>()];
  const BlockMap bm = map[blockIdx.x];
  const GemmDesc d = descs[bm.desc];
  const int tiles_m = (d.M + BM - 1) / BM;
  const int row0 = (bm.tile % tiles_m) * BM;
  const int col0 = (bm.tile / tiles_m) * BN;
  tn_lds_tile<BM, BN, KC>(d.A, d.lda, d.B, d.ldb, d.C, d.ldc, d.M, d.N, d.K, d.alpha, d.beta, row0,
                          col0, (d.flags & GEMM_STORE_T) != 0, smem);
}

template <bool TA, bool TB>
hipError_t launch_tt(const GemmDesc* d, const BlockMap* map, int nblocks, int bn, int bk,
                     hipStream_t s) {
  if (bn == 64 && bk == 64)
    hipLaunchKernelGGL((k_gemm<TA, TB, 64, 64>), dim3(nblocks), dim3(256), 0, s, d, map);
  else if (bn == 64)
    hipLaunchKernelGGL((k_gemm<TA, TB, 64, 16>), dim3(nblocks), dim3(256), 0, s, d, map);
  else if (bk == 64)
    hipLaunchKernelGGL((k_gemm<TA, TB, 16, 64>), dim3(nblocks), dim3(256), 0, s, d, map);
  else
    hipLaunchKernelGGL((k_gemm<TA, TB, 16, 16>), dim3(nblocks), dim3(256), 0, s, d, map);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_splitk_sum(double* C, int ldc, int M, int N,
                                                    const double* __restrict__ part, int S,
                                                    double alpha, double beta) {
  const size_t mn = (size_t)M * N;
  for (size_t e = blockIdx.x * 256ull + threadIdx.x; e < mn; e += (size_t)gridDim.x * 256) {
    const int r = (int)(e % M), c = (int)(e / M);
    double v = 0.0;
    for (int s = 0; s < S; ++s) v += gmem(part)[e + (size_t)s * mn];
    gdouble* cp = gmem(C) + r + (size_t)c * ldc;
    v *= alpha;
    if (beta != 0.0) v += beta * *cp;
    *cp = v;
  }
}

}  // namespace

hipError_t launch_splitk_sum(double* C, int ldc, int M, int N, const double* part, int S,
                             double alpha, double beta, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const long long mn = (long long)M * N;
  const unsigned blocks = (unsigned)std::min<long long>((mn + 255) / 256, 4096);
  hipLaunchKernelGGL(k_splitk_sum, dim3(blocks), dim3(256), 0, s, C, ldc, M, N, part, S, alpha,
                     beta);
  return hipGetLastError();
}

int gemm_tile_n(int N) { return N <= 16 ? 16 : 64; }

void gemm_tile_shape(bool trans_a, bool trans_b, int maxn, int* tm, int* tn) {
  if (trans_a && !trans_b) {
    *tm = 32;
    *tn = maxn <= 16 ? 16 : 32;
  } else {
    *tm = 64;
    *tn = gemm_tile_n(maxn);
  }
}

hipError_t launch_gemm_tn_lds(const GemmDesc* d_descs, const BlockMap* d_map, int nblocks, int bm,
                              int bn, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (bm == 16 && bn == 16)
    hipLaunchKernelGGL((k_gemm_tn_lds<16, 16>), dim3(nblocks), dim3(256), 0, s, d_descs, d_map);
  else if (bm == 64 && bn == 16)
    hipLaunchKernelGGL((k_gemm_tn_lds<64, 16>), dim3(nblocks), dim3(256), 0, s, d_descs, d_map);
  else if (bm == 64 && bn == 32)
    hipLaunchKernelGGL((k_gemm_tn_lds<64, 32>), dim3(nblocks), dim3(256), 0, s, d_descs, d_map);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

bool gemm_tn_lds_ok(const GemmDesc& d) { return (d.flags & ~GEMM_STORE_T) == 0 && d.K >= 1; }

hipError_t launch_gemm_batched(const GemmDesc* d_descs, const BlockMap* d_map, int nblocks,
                               bool trans_a, bool trans_b, int bn, int max_k, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  const int bk = max_k > 32 ? 64 : 16;
  if (!trans_a && !trans_b) return launch_tt<false, false>(d_descs, d_map, nblocks, bn, bk, s);
  if (trans_a && !trans_b) {
    if (bn == 0)
      hipLaunchKernelGGL((k_gemm_tn<1, 1>), dim3(nblocks), dim3(512), 0, s, d_descs, d_map);
    else if (bn <= 16)
      hipLaunchKernelGGL((k_gemm_tn<2, 1>), dim3(nblocks), dim3(512), 0, s, d_descs, d_map);
    else
      hipLaunchKernelGGL((k_gemm_tn<2, 2>), dim3(nblocks), dim3(512), 0, s, d_descs, d_map);
    return hipGetLastError();
  }
  if (!trans_a && trans_b) return launch_tt<false, true>(d_descs, d_map, nblocks, bn, bk, s);
  return launch_tt<true, true>(d_descs, d_map, nblocks, bn, bk, s);
}

}  // namespace tlr
