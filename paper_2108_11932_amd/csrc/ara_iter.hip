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

#include "ara_compact.h"
#include "ara_orth.h"

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
  // the slot and the active count are read together: act has an entry for
  // every block of the launch
  const int slot = D.act[ai];
  if (ai >= D.counts[0]) return false;
  if (D.skip && D.skip[slot]) return false;
  const AraSlotDesc& d = D.slots[slot];
  const int row0 = tile * TN_TM;
  if (mode == 0) {
    if (row0 >= d.a) return false;
    *o = TnTile{d.va, omega, d.wa, d.a, d.a, row0, tid, 1.0};
  } else {
    const int q = D.qin[slot];
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
__device__ inline void tn_body(const AraDev& D, int mode, const double* omega, const PTile* ptiles,
                               int p_tiles, int ldp, int tps, double* scratch, int bid) {
  constexpr int FM = 2, TSZ = TN_TM * 16 * FN;
  __shared__ double red[TN_NW][FM * FN * 4][64];
  const int m = D.m, bs = D.bs;
  const int ks_n = (m + TN_KC - 1) / TN_KC;
  const int ks = bid % ks_n, tid = bid / ks_n;
  TnTile o;
  if (!tn_resolve(D, mode, tid, omega, ptiles, p_tiles, ldp, tps, &o)) return;
  const int k0 = ks * TN_KC, k1 = min(m, k0 + TN_KC);
  tn_tile<FM, FN, TN_NW, 1, true>(o.A, m, o.B, m, scratch + ((size_t)tid * ks_n + ks) * TSZ, TN_TM,
                                  o.M, bs, k0, k1, 1.0, 0.0, o.row0, 0, red);
}

template <int FN>
__global__ __launch_bounds__(64 * TN_NW) void k_ara_tn(AraDev D, int mode, const double* omega,
                                                        const PTile* ptiles, int p_tiles, int ldp,
                                                        int tps, double* scratch) {
  tn_body<FN>(D, mode, omega, ptiles, p_tiles, ldp, tps, scratch, blockIdx.x);
}

template <int FN>
__device__ inline void tn_sum_body(const AraDev& D, int mode, const double* omega,
                                   const PTile* ptiles, int p_tiles, int ldp, int tps,
                                   const double* scratch, int bid) {
  constexpr int TSZ = TN_TM * 16 * FN;
  const int m = D.m, bs = D.bs;
  const int ks_n = (m + TN_KC - 1) / TN_KC;
  TnTile o;
  if (!tn_resolve(D, mode, bid, omega, ptiles, p_tiles, ldp, tps, &o)) return;
  const double* part = scratch + (size_t)bid * ks_n * TSZ;
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

template <int FN>
__global__ __launch_bounds__(256) void k_ara_tn_sum(AraDev D, int mode, const double* omega,
                                                    const PTile* ptiles, int p_tiles, int ldp,
                                                    int tps, const double* scratch) {
  tn_sum_body<FN>(D, mode, omega, ptiles, p_tiles, ldp, tps, scratch, blockIdx.x);
}

// Z on the matrix cores: one wave per piece (16 rows of one block G_ij P_j),
// four pieces per workgroup.  Lane l supplies G(l % 16, t) and P(t, l % 16)
// for t = t0 + l / 16; the k loop loads ZCH MFMA steps ahead.
constexpr int ZCH = 4;

__device__ inline void z_body(const AraDev& D, const ZSeg* __restrict__ segs,
                              const double* __restrict__ P, int ldp, int bps, int bid) {
  const int ai = bid / bps, tb = bid % bps;
  const int slot = D.act[ai];   // read with the active count, as in tn_resolve
  if (ai >= D.counts[0]) return;
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

__global__ __launch_bounds__(256) void k_ara_z(AraDev D, const ZSeg* __restrict__ segs,
                                               const double* __restrict__ P, int ldp, int bps) {
  z_body(D, segs, P, ldp, bps, blockIdx.x);
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
__device__ inline void seg_body(const AraDev& D, int bid) {
  constexpr int mode = MODE;
  constexpr int R32 = MODE == 0 ? 4 : 1;
  __shared__ double red[4][FM * NF * 4][64];
  __shared__ float red32[R32][FM * NF * 4][64];
  __shared__ double ys[16 * FM][16 * NF + 1];
  const int ns = D.nstrip;
  const int nblk = (ns + FM - 1) / FM;
  const int ai = bid / nblk, blk = bid % nblk;
  const int slot = D.act[ai];   // read with the active count, as in tn_resolve
  if (ai >= D.counts[0]) return;
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
    const int q = D.qin[slot];
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

template <int NF, int MODE, int FM>
__global__ __launch_bounds__(256) void k_ara_seg(AraDev D) {
  seg_body<NF, MODE, FM>(D, blockIdx.x);
}


// ---------------------------------------------------- fused launches
// The sampling of ARA iteration t + 1 needs only the convergence flags of
// iteration t (it skips the tiles they name), so it is computed in the same
// launches as the second Gram-Schmidt pass of iteration t: the first blocks
// of each launch do the one, the others the other.  Both halves run
// concurrently without a second stream, and the host issues one launch for
// two.
//   tn     : P, W^A of t + 1 (mode 0)   |  C = -Q^T X of t (mode 2), split K
//            and, in one more workgroup, the compaction of t's active list
//            into t + 1's (the flags are set by pass 1; the list t + 1 reads
//            is a second copy, and the widths need no commit)
//   tn_sum : their partial sums
//   z_seg  : Z of t + 1                 |  X += Q C of t (mode 2)
//   seg_orth: Y of t + 1 (mode 0)       |  pass-2 Cholesky QR of t
struct CompactArgs {
  const int* waiting;
  int nwaiting, s_max;
  const int* info;
  int* host_out;
  int* host_res;
  int res_ints;
};

template <int FN>
__global__ __launch_bounds__(64 * TN_NW) void k_fuse_tn(AraDev Da, const double* omega,
                                                         const PTile* ptiles, int p_tiles, int ldp,
                                                         int tpsa, double* scra, int na, AraDev Db,
                                                         int tpsb, double* scrb, int nab,
                                                         CompactArgs ca) {
  static_assert(64 * TN_NW == 256, "the compaction runs on 256 threads");
  if ((int)blockIdx.x < na)
    tn_body<FN>(Da, 0, omega, ptiles, p_tiles, ldp, tpsa, scra, blockIdx.x);
  else if ((int)blockIdx.x < nab)
    tn_body<FN>(Db, 2, nullptr, nullptr, 0, 0, tpsb, scrb, blockIdx.x - na);
  else
    ara_compact_body(Db, ca.waiting, ca.nwaiting, ca.s_max, ca.info, ca.host_out, ca.host_res,
                     ca.res_ints);
}

template <int FN>
__global__ __launch_bounds__(256) void k_fuse_tn_sum(AraDev Da, const double* omega,
                                                     const PTile* ptiles, int p_tiles, int ldp,
                                                     int tpsa, const double* scra, int na,
                                                     AraDev Db, int tpsb, const double* scrb) {
  if ((int)blockIdx.x < na)
    tn_sum_body<FN>(Da, 0, omega, ptiles, p_tiles, ldp, tpsa, scra, blockIdx.x);
  else
    tn_sum_body<FN>(Db, 2, nullptr, nullptr, 0, 0, tpsb, scrb, blockIdx.x - na);
}

template <int NF>
__global__ __launch_bounds__(256) void k_fuse_z_seg(AraDev Dz, const ZSeg* __restrict__ segs,
                                                    const double* __restrict__ P, int ldp, int bps,
                                                    int nz, AraDev Ds) {
  if ((int)blockIdx.x < nz)
    z_body(Dz, segs, P, ldp, bps, blockIdx.x);
  else
    seg_body<NF, 2, 1>(Ds, blockIdx.x - nz);
}

template <int NF, int FM, int BS>
__global__ __launch_bounds__(256) void k_fuse_seg_orth(AraDev D0, int n0, AraDev D2, int r_min,
                                                       int gx) {
  if ((int)blockIdx.x < n0) {
    seg_body<NF, 0, FM>(D0, blockIdx.x);
  } else {
    const int b = blockIdx.x - n0;
    orth_body<BS, false>(D2, r_min, b % gx, b / gx);
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

bool fused_block_supported(int bs) { return bs == 16 || bs == 32; }

hipError_t launch_fused_tn(const AraDev& Da, const double* omega, const PTile* ptiles, int p_tiles,
                           int ldp, int cba, int tpsa, double* scra, const AraDev& Db, int cbb,
                           int tpsb, double* scrb, const int* waiting, int nwaiting, int s_max,
                           const int* info, int* host_out, int* host_res, int res_ints,
                           hipStream_t s) {
  if (Da.bs != Db.bs || !fused_block_supported(Da.bs)) return hipErrorInvalidValue;
  const int ks_n = (Da.m + TN_KC - 1) / TN_KC;
  const long long ta = p_tiles + (long long)std::max(cba, 0) * std::max(tpsa, 0);
  const long long tb = (long long)std::max(cbb, 0) * std::max(tpsb, 0);
  const int pa = std::max(tpsa, 1), pb = std::max(tpsb, 1);
  // the products' blocks, then the compaction's
  const unsigned na = (unsigned)(ta * ks_n), nab = (unsigned)((ta + tb) * ks_n);
  const unsigned ma = (unsigned)ta, ms = (unsigned)(ta + tb);
  const CompactArgs ca{waiting, nwaiting, s_max, info, host_out, host_res, res_ints};
  if (Da.bs <= 16)
    hipLaunchKernelGGL((k_fuse_tn<1>), dim3(nab + 1), dim3(64 * TN_NW), 0, s, Da, omega, ptiles,
                       p_tiles, ldp, pa, scra, (int)na, Db, pb, scrb, (int)nab, ca);
  else
    hipLaunchKernelGGL((k_fuse_tn<2>), dim3(nab + 1), dim3(64 * TN_NW), 0, s, Da, omega, ptiles,
                       p_tiles, ldp, pa, scra, (int)na, Db, pb, scrb, (int)nab, ca);
  if (ms > 0) {
    if (Da.bs <= 16)
      hipLaunchKernelGGL((k_fuse_tn_sum<1>), dim3(ms), dim3(256), 0, s, Da, omega, ptiles, p_tiles,
                         ldp, pa, scra, (int)ma, Db, pb, scrb);
    else
      hipLaunchKernelGGL((k_fuse_tn_sum<2>), dim3(ms), dim3(256), 0, s, Da, omega, ptiles, p_tiles,
                         ldp, pa, scra, (int)ma, Db, pb, scrb);
  }
  return hipGetLastError();
}

hipError_t launch_fused_z_seg(const AraDev& Dz, const ZSeg* segs, const double* P, int ldp, int cbz,
                              int bps, const AraDev& Ds, int cbs, hipStream_t s) {
  if (Dz.bs != Ds.bs || !fused_block_supported(Ds.bs)) return hipErrorInvalidValue;
  const long long nz = (long long)std::max(cbz, 0) * std::max(bps, 0);
  const long long ns = (long long)std::max(cbs, 0) * Ds.nstrip;
  if (nz + ns <= 0) return hipSuccess;
  const dim3 g((unsigned)(nz + ns)), b(256);
  if (Ds.bs <= 16)
    hipLaunchKernelGGL((k_fuse_z_seg<1>), g, b, 0, s, Dz, segs, P, ldp, std::max(bps, 1), (int)nz,
                       Ds);
  else
    hipLaunchKernelGGL((k_fuse_z_seg<2>), g, b, 0, s, Dz, segs, P, ldp, std::max(bps, 1), (int)nz,
                       Ds);
  return hipGetLastError();
}

hipError_t launch_fused_seg_orth(const AraDev& D0, int cb0, int strip, const AraDev& D2, int cb2,
                                 int r_min, hipStream_t s) {
  if (D0.bs != D2.bs || !fused_block_supported(D2.bs)) return hipErrorInvalidValue;
  const bool tall = strip == 64 || (strip == 0 && (long long)std::max(cb0, 0) *
                                                         ((D0.nstrip + 3) / 4) >= kTallWgs);
  const int fm = tall ? 4 : 1;
  const long long n0 = (long long)std::max(cb0, 0) * ((D0.nstrip + fm - 1) / fm);
  const int gx = (D2.m + APPLY_ROWS - 1) / APPLY_ROWS;
  const long long n2 = (long long)gx * std::max(cb2, 0);
  if (n0 + n2 <= 0) return hipSuccess;
  const dim3 g((unsigned)(n0 + n2)), b(256);
  static_assert(APPLY_ROWS == 256, "the fused launch runs 256 threads per block");
  if (D2.bs == 16) {
    if (tall)
      hipLaunchKernelGGL((k_fuse_seg_orth<1, 4, 16>), g, b, 0, s, D0, (int)n0, D2, r_min, gx);
    else
      hipLaunchKernelGGL((k_fuse_seg_orth<1, 1, 16>), g, b, 0, s, D0, (int)n0, D2, r_min, gx);
  } else {
    if (tall)
      hipLaunchKernelGGL((k_fuse_seg_orth<2, 4, 32>), g, b, 0, s, D0, (int)n0, D2, r_min, gx);
    else
      hipLaunchKernelGGL((k_fuse_seg_orth<2, 1, 32>), g, b, 0, s, D0, (int)n0, D2, r_min, gx);
  }
  return hipGetLastError();
}

}  // namespace tlr
