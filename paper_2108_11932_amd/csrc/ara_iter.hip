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
#include <hip/hip_ext.h>

#include "dd.h"
#include "mfma_tiles.h"
#include "tlr_internal.h"

// the Gram partials use error-free transformations
#pragma clang fp contract(off)

namespace tlr {

namespace {

constexpr int TN_NW = 4;
constexpr int TN_KC = 16 * TN_NW;   // rows of K per workgroup: one 16-row slice per wave
constexpr int TN_TM = 32;

// Output tile `tid` of a TN launch: operands, destination and bounds.
struct TnTile {
  const double* A;
  const double* B;
  double* C;
  int M, ldc, row0, gtile;
  double alpha;
};
__device__ inline bool tn_resolve(const AraDev& D, int mode, int tid, const double* omega,
                                  const PTile* ptiles, int p_tiles, int ldp, int tps, TnTile* o) {
  const int m = D.m;
  if (mode == 0 && tid < p_tiles) {
    const PTile& pt = ptiles[tid];
    *o = TnTile{pt.A, omega, pt.C, pt.M, ldp, pt.row0, tid, 1.0};
    return true;
  }
  const int t = mode == 0 ? tid - p_tiles : tid;
  const int ai = t / tps, tile = t % tps;
  if (ai >= D.counts[0]) return false;
  const int slot = D.act[ai];
  if (D.skip && D.skip[slot]) return false;
  const AraSlotDesc& d = D.slots[slot];
  const int row0 = tile * TN_TM;
  if (mode == 0) {
    if (row0 >= d.a) return false;
    *o = TnTile{d.va, omega, d.wa, d.a, d.a, row0, tid, 1.0};
  } else {
    const int q = D.q[slot];
    if (row0 >= q) return false;
    const double* B = mode == 1 ? d.y + D.yoff : d.q + (size_t)q * m;
    *o = TnTile{d.q, B, d.c, q, m, row0, tid, -1.0};
  }
  return true;
}

// The products of these kernels have few output tiles (a handful of active
// tiles late in a column) and K = m, while one CU streams only a few tens of
// GB/s: the K range is split over ceil(m / TN_KC) workgroups per output
// tile, each storing its partial tile in scratch; k_ara_tn_sum then adds the
// partials in a fixed order (a second launch rather than a cross-workgroup
// handshake, whose device-scope fences are costly across the XCDs).  One
// workgroup per output tile over the whole K range (one launch, partials
// summed in LDS) measured twice as slow: a CU alone streams too little.
template <int FN>
__global__ __launch_bounds__(64 * TN_NW) void k_ara_tn(AraDev D, int mode, const double* omega,
                                                        const PTile* ptiles, int p_tiles, int ldp,
                                                        int tps, double* scratch) {
  constexpr int FM = 2, TSZ = TN_TM * 16 * FN;
  __shared__ double red[TN_NW][FM * FN * 4][64];
  const int m = D.m, bs = D.bs;
  const int ks_n = (m + TN_KC - 1) / TN_KC;
  const int ks = blockIdx.x % ks_n, tid = blockIdx.x / ks_n;
  TnTile o;
  if (!tn_resolve(D, mode, tid, omega, ptiles, p_tiles, ldp, tps, &o)) return;
  const int k0 = ks * TN_KC, k1 = min(m, k0 + TN_KC);
  tn_tile<FM, FN, TN_NW, 1, true>(o.A, m, o.B, m, scratch + ((size_t)tid * ks_n + ks) * TSZ, TN_TM,
                                  o.M, bs, k0, k1, 1.0, 0.0, o.row0, 0, red);
}

template <int FN>
__global__ __launch_bounds__(256) void k_ara_tn_sum(AraDev D, int mode, const double* omega,
                                                    const PTile* ptiles, int p_tiles, int ldp,
                                                    int tps, const double* scratch) {
  constexpr int TSZ = TN_TM * 16 * FN;
  const int m = D.m, bs = D.bs;
  const int ks_n = (m + TN_KC - 1) / TN_KC;
  TnTile o;
  if (!tn_resolve(D, mode, blockIdx.x, omega, ptiles, p_tiles, ldp, tps, &o)) return;
  const double* part = scratch + (size_t)blockIdx.x * ks_n * TSZ;
  for (int e = threadIdx.x; e < TSZ; e += 256) {
    const int lr = e % TN_TM, lc = e / TN_TM;
    if (o.row0 + lr >= o.M || lc >= bs) continue;
    constexpr int CH = 16;
    double v = 0.0;
    for (int s0 = 0; s0 < ks_n; s0 += CH) {
      double pv[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) pv[u] = gmem(part)[(size_t)min(s0 + u, ks_n - 1) * TSZ + e];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (s0 + u < ks_n) v += pv[u];
    }
    gmem(o.C)[o.row0 + lr + (size_t)lc * o.ldc] = o.alpha * v;
  }
}

// Z on the matrix cores: one wave per piece (16 rows of one block G_ij P_j),
// four pieces per workgroup.  Lane l supplies G(l % 16, t) and P(t, l % 16)
// for t = t0 + l / 16; the k loop loads ZCH MFMA steps ahead.
constexpr int ZCH = 4;

__global__ __launch_bounds__(256) void k_ara_z(AraDev D, const ZSeg* __restrict__ segs,
                                               const double* __restrict__ P, int ldp, int bps) {
  const int ai = blockIdx.x / bps, tb = blockIdx.x % bps;
  if (ai >= D.counts[0]) return;
  const int slot = D.act[ai];
  if (D.skip && D.skip[slot]) return;
  const AraSlotDesc& d = D.slots[slot];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int pi = tb * 4 + wave;
  if (pi >= d.nz) return;
  const ZSeg z = segs[d.zseg + pi];
  const int bs = D.bs;
  const int li = lane & 15, kq = lane >> 4;
  const gdouble* grow = gmem(z.g) + min(li, z.rows - 1);
  for (int n0 = 0; n0 < bs; n0 += 16) {
    const gdouble* pcol = gmem(P) + z.prow + (size_t)min(n0 + li, bs - 1) * ldp;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    for (int t0 = 0; t0 < z.cols; t0 += 4 * ZCH) {
      double av[ZCH], bv[ZCH];
#pragma unroll
      for (int u = 0; u < ZCH; ++u) {
        const int t = min(t0 + 4 * u + kq, z.cols - 1);
        av[u] = grow[(size_t)t * z.ldg];
        bv[u] = pcol[t];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < ZCH; ++u) {
        if (t0 + 4 * u + kq >= z.cols) av[u] = 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
      }
    }
    // accumulator register r of lane l holds row l / 16 + 4 r, column l % 16
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = kq + 4 * r, col = n0 + li;
      if (row < z.rows && col < bs) gmem(d.z)[z.zrow + row + (size_t)col * d.R] = -acc[r];
    }
  }
}

// MODE 0 (the sampling product) and modes 1, 2 are separate instantiations
// so that profiles tell them apart.  A workgroup computes FM 16-row strips
// of one tile: FM = 4 (64-row strips) reads 512 contiguous bytes of every
// panel column and each test-matrix row once for four row blocks, where
// enough tiles are active to keep the CUs busy; FM = 1 spreads few tiles over
// four times more workgroups.  Both give the same Y bit for bit.  In mode 0
// the panel segment U_i* Z_i of a slot runs in the precision its descriptor
// names (a1_prec: FP64, or the packed FP32 / BF16 panel copy with FP32
// accumulation).
template <int NF, int MODE, int FM>
__global__ __launch_bounds__(256) void k_ara_seg(AraDev D) {
  constexpr int mode = MODE;
  constexpr int R32 = MODE == 0 ? 4 : 1;
  __shared__ double red[4][FM * NF * 4][64];
  __shared__ float red32[R32][FM * NF * 4][64];
  __shared__ double ys[16 * FM][16 * NF + 1];
  const int ns = D.nstrip;
  const int nblk = (ns + FM - 1) / FM;
  const int ai = blockIdx.x / nblk, blk = blockIdx.x % nblk;
  if (ai >= D.counts[0]) return;
  const int slot = D.act[ai];
  if (D.skip && D.skip[slot]) return;
  const AraSlotDesc& d = D.slots[slot];
  const int m = D.m, bs = D.bs;
  const int r0 = blk * 16 * FM;
  double* part;
  if (mode == 0) {
    float (*r32)[FM * NF * 4][64] = (float (*)[FM * NF * 4][64])red32;
    if (d.a1_prec == 1)
      seg_strip<NF, 1, FM>(d.a0, d.lda0, d.b0, d.ldb0, d.k0, d.a1, d.lda1, d.b1, d.ldb1, d.k1,
                           d.y + D.yoff, m, m, bs, 0.0, r0, red, r32, ys);
    else if (d.a1_prec == 2)
      seg_strip<NF, 2, FM>(d.a0, d.lda0, d.b0, d.ldb0, d.k0, d.a1, d.lda1, d.b1, d.ldb1, d.k1,
                           d.y + D.yoff, m, m, bs, 0.0, r0, red, r32, ys);
    else
      seg_strip<NF, 0, FM>(d.a0, d.lda0, d.b0, d.ldb0, d.k0, d.a1, d.lda1, d.b1, d.ldb1, d.k1,
                           d.y + D.yoff, m, m, bs, 0.0, r0, red, r32, ys);
    part = d.part1 + D.poff;
  } else {
    const int q = D.q[slot];
    if (q == 0) return;
    double* dst = mode == 1 ? d.y + D.yoff : d.q + (size_t)q * m;
    seg_strip<NF, 0, FM>(d.q, m, d.c, m, q, nullptr, 1, nullptr, 1, 0, dst, m, m, bs, 1.0, r0,
                         red, nullptr, ys);
    part = mode == 1 ? d.part1 + D.poff : d.part2;
  }
  // Gram partials of each 16-row strip (Dot2 over its rows), pairs a <= b
  const int npairs = bs * (bs + 1) / 2;
  const int s0 = blk * FM, nsub = min(FM, ns - s0);
  for (int e = threadIdx.x; e < nsub * npairs; e += 256) {
    const int sub = e / npairs, pr = e % npairs;
    int b = (int)((sqrt(8.0 * pr + 1.0) - 1.0) * 0.5);
    while (b * (b + 1) / 2 > pr) --b;
    while ((b + 1) * (b + 2) / 2 <= pr) ++b;
    const int a = pr - b * (b + 1) / 2;
    double sh = 0.0, sl = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) dot2_step(ys[16 * sub + r][a], ys[16 * sub + r][b], sh, sl);
    const dd v = fast_two_sum(sh, sl);
    gdouble* out = gmem(part) + (size_t)(s0 + sub) * bs * bs * 2;
    out[(a + b * bs) * 2 + 0] = v.hi;
    out[(a + b * bs) * 2 + 1] = v.lo;
  }
}

}  // namespace

int ara_tn_scratch(int m, int bs, long long tiles, size_t* doubles) {
  const int ks_n = (m + TN_KC - 1) / TN_KC;
  *doubles = (size_t)tiles * ks_n * TN_TM * (bs <= 16 ? 16 : 32);
  return TN_TM;
}

hipError_t launch_ara_tn(const AraDev& D, int mode, const double* omega, const PTile* ptiles,
                         int p_tiles, int ldp, int count_bound, int tps, double* scratch,
                         hipStream_t s) {
  if (D.bs > 32) return hipErrorInvalidValue;
  const int pt = mode == 0 ? p_tiles : 0;
  const int ks_n = (D.m + TN_KC - 1) / TN_KC;
  const long long tiles = pt + (long long)std::max(count_bound, 0) * std::max(tps, 0);
  if (tiles <= 0) return hipSuccess;
  const int tp = std::max(tps, 1);
  if (D.bs <= 16) {
    hipLaunchKernelGGL((k_ara_tn<1>), dim3((unsigned)(tiles * ks_n)), dim3(64 * TN_NW), 0, s, D,
                       mode, omega, ptiles, pt, ldp, tp, scratch);
    hipLaunchKernelGGL((k_ara_tn_sum<1>), dim3((unsigned)tiles), dim3(256), 0, s, D, mode, omega,
                       ptiles, pt, ldp, tp, scratch);
  } else {
    hipLaunchKernelGGL((k_ara_tn<2>), dim3((unsigned)(tiles * ks_n)), dim3(64 * TN_NW), 0, s, D,
                       mode, omega, ptiles, pt, ldp, tp, scratch);
    hipLaunchKernelGGL((k_ara_tn_sum<2>), dim3((unsigned)tiles), dim3(256), 0, s, D, mode, omega,
                       ptiles, pt, ldp, tp, scratch);
  }
  return hipGetLastError();
}

hipError_t launch_ara_z(const AraDev& D, const ZSeg* segs, const double* P, int ldp,
                        int count_bound, int bps, hipStream_t s) {
  const long long n = (long long)std::max(count_bound, 0) * std::max(bps, 0);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ara_z, dim3((unsigned)n), dim3(256), 0, s, D, segs, P, ldp, bps);
  return hipGetLastError();
}

namespace {
// the sampling product runs on 64-row strips once this many workgroups of
// them fill the launch
constexpr long long kTallWgs = 512;

template <int NF, int FM>
hipError_t seg_launch(const AraDev& D, int mode, int count_bound, hipStream_t s, hipEvent_t start,
                      hipEvent_t stop) {
  const long long n = (long long)count_bound * ((D.nstrip + FM - 1) / FM);
  const dim3 g((unsigned)n), b(256);
  if (start || stop) {
    // the events take the dispatch's own begin and end timestamps
    hipExtLaunchKernelGGL((k_ara_seg<NF, 0, FM>), g, b, 0, s, start, stop, 0, D);
    return mode == 0 ? hipGetLastError() : hipErrorInvalidValue;
  }
  if (mode == 0) hipLaunchKernelGGL((k_ara_seg<NF, 0, FM>), g, b, 0, s, D);
  if (mode == 1) hipLaunchKernelGGL((k_ara_seg<NF, 1, 1>), g, b, 0, s, D);
  if (mode == 2) hipLaunchKernelGGL((k_ara_seg<NF, 2, 1>), g, b, 0, s, D);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_ara_seg(const AraDev& D, int mode, int count_bound, hipStream_t s, int strip,
                          hipEvent_t start, hipEvent_t stop) {
  if (D.bs > 32 || mode < 0 || mode > 2) return hipErrorInvalidValue;
  if ((long long)std::max(count_bound, 0) * D.nstrip <= 0) return hipSuccess;
  const bool tall = mode == 0 && (strip == 64 || (strip == 0 && (long long)count_bound *
                                                                       ((D.nstrip + 3) / 4) >=
                                                                   kTallWgs));
  if (D.bs <= 16)
    return tall ? seg_launch<1, 4>(D, mode, count_bound, s, start, stop)
                : seg_launch<1, 1>(D, mode, count_bound, s, start, stop);
  return tall ? seg_launch<2, 4>(D, mode, count_bound, s, start, stop)
              : seg_launch<2, 1>(D, mode, count_bound, s, start, stop);
}

}  // namespace tlr
