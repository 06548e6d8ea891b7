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
#include "tlr_internal.h"

namespace tlr {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 64;
constexpr int BK = 16;
constexpr int PAD = 2;

// MFMA f64 16x16x4 operand layout (measured on gfx950): lane l supplies
// A(l % 16, l / 16) and B(l / 16, l % 16); accumulator register r of lane l
// holds D(l / 16 + 4 r, l % 16).
template <bool TA, bool TB, int BN>
__global__ __launch_bounds__(256) void k_gemm(const GemmDesc* __restrict__ descs,
                                              const BlockMap* __restrict__ map) {
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

  for (int k0 = 0; k0 < d.K; k0 += BK) {
    // ---- stage op(A)(row0 + r, k0 + kk), 64 x 16
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int r, kk;
      if (!TA) { r = tid & 63; kk = (tid >> 6) + 4 * j; }
      else     { kk = tid & 15; r = (tid >> 4) + 16 * j; }
      const int gr = row0 + r, gk = k0 + kk;
      double v = 0.0;
      if (gr < d.M && gk < d.K)
        v = TA ? d.A[gk + (size_t)gr * d.lda] : d.A[gr + (size_t)gk * d.lda];
      sA[kk][r] = v;
    }
    // ---- stage op(B)(k0 + kk, col0 + c), 16 x BN
#pragma unroll
    for (int j = 0; j < BN / 16; ++j) {
      int c, kk;
      if (!TB) { kk = tid & 15; c = (tid >> 4) + 16 * j; }
      else     { c = tid % BN; kk = tid / BN + (256 / BN) * j; }
      const int gc = col0 + c, gk = k0 + kk;
      double v = 0.0;
      if (gc < d.N && gk < d.K)
        v = TB ? d.B[gc + (size_t)gk * d.ldb] : d.B[gk + (size_t)gc * d.ldb];
      sB[kk][c] = v;
    }
    __syncthreads();
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
        double* cp = d.C + gr + (size_t)gc * d.ldc;
        double v = d.alpha * acc[a][b][r];
        if (d.beta != 0.0) v += d.beta * *cp;
        *cp = v;
      }
    }
}

template <bool TA, bool TB>
hipError_t launch_tt(const GemmDesc* d, const BlockMap* map, int nblocks, int bn, hipStream_t s) {
  if (bn == 64)
    hipLaunchKernelGGL((k_gemm<TA, TB, 64>), dim3(nblocks), dim3(256), 0, s, d, map);
  else
    hipLaunchKernelGGL((k_gemm<TA, TB, 16>), dim3(nblocks), dim3(256), 0, s, d, map);
  return hipGetLastError();
}

}  // namespace

int gemm_tile_n(int N) { return N <= 16 ? 16 : 64; }

hipError_t launch_gemm_batched(const GemmDesc* d_descs, const BlockMap* d_map, int nblocks,
                               bool trans_a, bool trans_b, int bn, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (!trans_a && !trans_b) return launch_tt<false, false>(d_descs, d_map, nblocks, bn, s);
  if (trans_a && !trans_b) return launch_tt<true, false>(d_descs, d_map, nblocks, bn, s);
  if (!trans_a && trans_b) return launch_tt<false, true>(d_descs, d_map, nblocks, bn, s);
  return launch_tt<true, true>(d_descs, d_map, nblocks, bn, s);
}

}  // namespace tlr
