// Streaming product of the Schur-complement sampling (Eq. (2), Section 4.1):
//
//   C = beta C + A0 B0 + A1 B1,   A_s m x K_s column-major, B_s K_s x N,
//
// with N = the ARA block size (16 or 32).  For one tile of column k the two
// segments are (U^A_ik, V^A_ik^T Omega) and (U_i*, -[G_ij P_j]_j), i.e. the
// sampled input tile and the row panel of the factor against the reduced
// test matrix; the same kernel performs the Gram-Schmidt update Y - Q C.
// Every element of A is used once, so the kernel is bound by HBM: a
// workgroup owns 16 rows of one problem and its four waves take interleaved
// 16-wide slices of the K range of both segments (many loads in flight even
// when few tiles are active), reduced through LDS in a fixed order.  Lane (i, g) reads row i of A for the four columns
// k0 + 4 g + t (128-byte runs per column over the 16 lanes of a group) and
// rows k0 + 4 g + t of column i of B (32-byte runs); MFMA t consumes k0 +
// 4 g + t on both operands.
#include "tlr_internal.h"

namespace tlr {

typedef double d4s __attribute__((ext_vector_type(4)));

namespace {

// Segment 1's A is read as float when A1F32 is set (the FP32 copy of the
// factor's row panels used by the mixed-precision sampling); the products
// are still formed and accumulated in FP64.
template <int NF, bool A1F32>
__global__ __launch_bounds__(256) void k_sample_nn(const SegDesc* __restrict__ descs,
                                                   const BlockMap* __restrict__ map) {
  __shared__ double red[4][NF * 4][64];
  const BlockMap bm = map[blockIdx.x];
  const SegDesc d = descs[bm.desc];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int r0 = bm.tile * 16;
  const int row = r0 + li;
  const bool rok = row < d.M;

  d4s acc[NF];
#pragma unroll
  for (int b = 0; b < NF; ++b) acc[b] = d4s{0.0, 0.0, 0.0, 0.0};

  // U 16-wide k steps per pass, all loads of a pass in flight together;
  // loads past K read a clamped in-range address and are zeroed
  constexpr int U = 4;
#pragma unroll
  for (int sg = 0; sg < 2; ++sg) {
    const int K = d.K[sg];
    if (K <= 0) continue;
    const bool f32 = A1F32 && sg == 1;
    const double* __restrict__ A = (const double*)d.A[sg] + (rok ? row : 0);
    const float* __restrict__ Af = (const float*)d.A[sg] + (rok ? row : 0);
    const double* __restrict__ B = d.B[sg];
    const size_t lda = d.lda[sg], ldb = d.ldb[sg];
    const double* bcol[NF];
    bool bok[NF];
#pragma unroll
    for (int b = 0; b < NF; ++b) {
      const int c = b * 16 + li;
      bok[b] = c < d.N;
      bcol[b] = B + (size_t)(bok[b] ? c : 0) * ldb;
    }
    // wave w takes the 16-wide k steps w, w + 4, w + 8, ...
    for (int k0 = wave * 16; k0 < K; k0 += 64 * U) {
      double av[U][4], bv[U][NF][4];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int kr = k0 + 64 * u + 4 * g;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const bool kin = kr + t < K;
          const int kk = kin ? kr + t : K - 1;
          const double a = f32 ? (double)Af[(size_t)kk * lda] : A[(size_t)kk * lda];
          av[u][t] = (rok && kin) ? a : 0.0;
#pragma unroll
          for (int b = 0; b < NF; ++b) {
            const double v = bcol[b][kk];
            bv[u][b][t] = (bok[b] && kin) ? v : 0.0;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int b = 0; b < NF; ++b)
            acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][t], bv[u][b][t], acc[b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int b = 0; b < NF; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) red[wave][b * 4 + r][lane] = acc[b][r];
  __syncthreads();
  // accumulator register r of lane l holds row r0 + l/16 + 4 r, column l%16
  for (int e = threadIdx.x; e < NF * 4 * 64; e += 256) {
    const int slot = e >> 6, l = e & 63;
    const int b = slot >> 2, r = slot & 3;
    const int rr = r0 + (l >> 4) + 4 * r;
    const int c = b * 16 + (l & 15);
    if (rr >= d.M || c >= d.N) continue;
    double v = ((red[0][slot][l] + red[1][slot][l]) + red[2][slot][l]) + red[3][slot][l];
    double* cp = d.C + rr + (size_t)c * d.ldc;
    if (d.beta != 0.0) v += d.beta * *cp;
    *cp = v;
  }
}

}  // namespace

hipError_t launch_sample_nn(const SegDesc* d, const BlockMap* map, int nblocks, int maxn,
                            bool a1_f32, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (maxn > 32) return hipErrorInvalidValue;
  if (maxn <= 16) {
    if (a1_f32)
      hipLaunchKernelGGL((k_sample_nn<1, true>), dim3(nblocks), dim3(256), 0, s, d, map);
    else
      hipLaunchKernelGGL((k_sample_nn<1, false>), dim3(nblocks), dim3(256), 0, s, d, map);
  } else {
    if (a1_f32)
      hipLaunchKernelGGL((k_sample_nn<2, true>), dim3(nblocks), dim3(256), 0, s, d, map);
    else
      hipLaunchKernelGGL((k_sample_nn<2, false>), dim3(nblocks), dim3(256), 0, s, d, map);
  }
  return hipGetLastError();
}

}  // namespace tlr
