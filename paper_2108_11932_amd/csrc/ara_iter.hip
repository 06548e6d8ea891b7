// Products of one device-driven ARA iteration (Algorithm "Left Looking
// Cholesky TLR ARA Update", Section 4.2, with the sampling of Eq. (2)
// reassociated): every block finds its slot through the device-side active
// list, so one launch serves whatever subset of tiles is still active, and
// blocks past the active count or the slot's sizes return at once.
//
//   k_ara_tn   P = U_k*^T Omega and W^A_i = V^A_ik^T Omega      (mode 0)
//              C_i = -Q_i^T Y_i  /  C_i = -Q_i^T X_i             (modes 1, 2)
//   k_ara_z    Z_i = -[G_ij P_j]_j                 (block diagonal in j)
//   k_ara_seg  Y_i = U^A_ik W^A_i + U_i* Z_i                     (mode 0)
//              Y_i += Q_i C_i  /  X_i += Q_i C_i                 (modes 1, 2)
//              and the double-double Gram partials of the result per
//              16-row strip (input of the Cholesky QR step)
#include "dd.h"
#include "mfma_tiles.h"
#include "tlr_internal.h"

// the Gram partials use error-free transformations
#pragma clang fp contract(off)

namespace tlr {

namespace {

constexpr int TN_NW = 8;

template <int FN>
__global__ __launch_bounds__(512) void k_ara_tn(AraDev D, int mode, const double* omega,
                                                const double* uk, int rk, double* P, int p_blocks,
                                                int bps) {
  constexpr int FM = 2;
  __shared__ double red[TN_NW][FM * FN * 4][64];
  const int m = D.m, bs = D.bs;
  int b = blockIdx.x;
  if (mode == 0 && b < p_blocks) {
    tn_tile<FM, FN, TN_NW>(uk, m, omega, m, P, rk, rk, bs, 0, m, 1.0, 0.0, b * 16 * FM, 0, red);
    return;
  }
  if (mode == 0) b -= p_blocks;
  const int ai = b / bps, tile = b % bps;
  if (ai >= D.counts[0]) return;
  const int slot = D.act[ai];
  const AraSlotDesc& d = D.slots[slot];
  const int row0 = tile * 16 * FM;
  if (mode == 0) {
    if (row0 >= d.a) return;
    tn_tile<FM, FN, TN_NW>(d.va, m, omega, m, d.wa, d.a, d.a, bs, 0, m, 1.0, 0.0, row0, 0, red);
  } else {
    const int q = D.q[slot];
    if (row0 >= q) return;
    const double* B = mode == 1 ? d.y : d.q + (size_t)q * m;
    tn_tile<FM, FN, TN_NW>(d.q, m, B, m, d.c, m, q, bs, 0, m, -1.0, 0.0, row0, 0, red);
  }
}

// 64 rows of Z per block; each output row lies in exactly one segment
// (the rows of tile (i, j) in the panel).  The slot's segment table is
// staged in LDS and searched there; the contraction over the segment's
// columns loads ZCH G and P values ahead of the sums.
constexpr int ZROWS = 64;
constexpr int ZSEG_MAX = 1024;   // segments staged in LDS (j < k <= nb)
constexpr int ZCH = 8;

__global__ __launch_bounds__(256) void k_ara_z(AraDev D, const ZSeg* __restrict__ segs,
                                               const double* __restrict__ P, int ldp, int bps) {
  __shared__ int zrow[ZSEG_MAX];
  const int ai = blockIdx.x / bps, tile = blockIdx.x % bps;
  if (ai >= D.counts[0]) return;
  const int slot = D.act[ai];
  const AraSlotDesc& d = D.slots[slot];
  const int r0 = tile * ZROWS;
  if (r0 >= d.R) return;
  const int bs = D.bs, nz = d.nz;
  const ZSeg* sg = segs + d.zseg;
  for (int e = threadIdx.x; e < nz && e < ZSEG_MAX; e += 256) zrow[e] = sg[e].zrow;
  __syncthreads();
  const int nzl = min(nz, ZSEG_MAX);
  for (int e = threadIdx.x; e < ZROWS * bs; e += 256) {
    const int row = r0 + (e % ZROWS), col = e / ZROWS;
    if (row >= d.R) continue;
    int lo = 0, hi = nzl - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (zrow[mid] <= row) lo = mid; else hi = mid - 1;
    }
    // a panel of more than ZSEG_MAX segments continues linearly
    while (lo + 1 < nz && sg[lo + 1].zrow <= row) ++lo;
    const ZSeg z = sg[lo];
    const double* gr = z.g + (row - z.zrow);
    const double* pc = P + z.prow + (size_t)col * ldp;
    double v = 0.0;
    for (int t0 = 0; t0 < z.cols; t0 += ZCH) {
      double gv[ZCH], pv[ZCH];
#pragma unroll
      for (int u = 0; u < ZCH; ++u) {
        const int t = min(t0 + u, z.cols - 1);
        gv[u] = gr[(size_t)t * z.rows];
        pv[u] = pc[t];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < ZCH; ++u)
        if (t0 + u < z.cols) v += gv[u] * pv[u];
    }
    d.z[row + (size_t)col * d.R] = -v;
  }
}

template <int NF>
__global__ __launch_bounds__(256) void k_ara_seg(AraDev D, int mode) {
  __shared__ double red[4][NF * 4][64];
  __shared__ double ys[16][16 * NF + 1];
  const int ns = D.nstrip;
  const int ai = blockIdx.x / ns, strip = blockIdx.x % ns;
  if (ai >= D.counts[0]) return;
  const int slot = D.act[ai];
  const AraSlotDesc& d = D.slots[slot];
  const int m = D.m, bs = D.bs;
  const int r0 = strip * 16;
  double* part;
  if (mode == 0) {
    if (d.a1_f32)
      seg_strip<NF, true>(d.a0, d.lda0, d.b0, d.ldb0, d.k0, d.a1, d.lda1, d.b1, d.ldb1, d.k1, d.y, m,
                          m, bs, 0.0, r0, red, ys);
    else
      seg_strip<NF, false>(d.a0, d.lda0, d.b0, d.ldb0, d.k0, d.a1, d.lda1, d.b1, d.ldb1, d.k1, d.y,
                           m, m, bs, 0.0, r0, red, ys);
    part = d.part1;
  } else {
    const int q = D.q[slot];
    if (q == 0) return;
    double* dst = mode == 1 ? d.y : d.q + (size_t)q * m;
    seg_strip<NF, false>(d.q, m, d.c, m, q, nullptr, 1, nullptr, 1, 0, dst, m, m, bs, 1.0, r0, red,
                         ys);
    part = mode == 1 ? d.part1 : d.part2;
  }
  // Gram partials of the strip (Dot2 over its 16 rows), pairs a <= b
  const int npairs = bs * (bs + 1) / 2;
  double* out = part + (size_t)strip * bs * bs * 2;
  for (int pr = threadIdx.x; pr < npairs; pr += 256) {
    int b = (int)((sqrt(8.0 * pr + 1.0) - 1.0) * 0.5);
    while (b * (b + 1) / 2 > pr) --b;
    while ((b + 1) * (b + 2) / 2 <= pr) ++b;
    const int a = pr - b * (b + 1) / 2;
    double sh = 0.0, sl = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) dot2_step(ys[r][a], ys[r][b], sh, sl);
    const dd v = fast_two_sum(sh, sl);
    out[(a + b * bs) * 2 + 0] = v.hi;
    out[(a + b * bs) * 2 + 1] = v.lo;
  }
}

}  // namespace

hipError_t launch_ara_tn(const AraDev& D, int mode, const double* omega, const double* uk, int rk,
                         double* P, int p_blocks, int count_bound, int bps, hipStream_t s) {
  if (D.bs > 32) return hipErrorInvalidValue;
  const int pb = mode == 0 ? p_blocks : 0;
  const long long n = pb + (long long)std::max(count_bound, 0) * std::max(bps, 0);
  if (n <= 0) return hipSuccess;
  if (D.bs <= 16)
    hipLaunchKernelGGL((k_ara_tn<1>), dim3((unsigned)n), dim3(512), 0, s, D, mode, omega, uk, rk, P,
                       pb, std::max(bps, 1));
  else
    hipLaunchKernelGGL((k_ara_tn<2>), dim3((unsigned)n), dim3(512), 0, s, D, mode, omega, uk, rk, P,
                       pb, std::max(bps, 1));
  return hipGetLastError();
}

hipError_t launch_ara_z(const AraDev& D, const ZSeg* segs, const double* P, int ldp,
                        int count_bound, int bps, hipStream_t s) {
  const long long n = (long long)std::max(count_bound, 0) * std::max(bps, 0);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ara_z, dim3((unsigned)n), dim3(256), 0, s, D, segs, P, ldp, bps);
  return hipGetLastError();
}

hipError_t launch_ara_seg(const AraDev& D, int mode, int count_bound, hipStream_t s) {
  if (D.bs > 32) return hipErrorInvalidValue;
  const long long n = (long long)std::max(count_bound, 0) * D.nstrip;
  if (n <= 0) return hipSuccess;
  if (D.bs <= 16)
    hipLaunchKernelGGL((k_ara_seg<1>), dim3((unsigned)n), dim3(256), 0, s, D, mode);
  else
    hipLaunchKernelGGL((k_ara_seg<2>), dim3((unsigned)n), dim3(256), 0, s, D, mode);
  return hipGetLastError();
}

}  // namespace tlr
