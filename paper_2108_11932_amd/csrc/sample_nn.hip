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
#include "mfma_tiles.h"
#include "tlr_internal.h"

namespace tlr {

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
  seg_strip<NF, A1F32>((const double*)d.A[0], d.lda[0], d.B[0], d.ldb[0], d.K[0], d.A[1], d.lda[1],
                       d.B[1], d.ldb[1], d.K[1], d.C, d.ldc, d.M, d.N, d.beta, bm.tile * 16, red,
                       nullptr);
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
