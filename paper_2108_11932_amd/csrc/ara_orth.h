// Cholesky QR step of the batched ARA (batchOrthog, Section 3.1): the
// device body shared by the kernel that runs it alone and the fused launches
// of the ARA iteration.  Included by the ARA kernel files, which compile
// without floating-point contraction (the double-double arithmetic needs
// every product and sum rounded separately).
#pragma once

#include "dd.h"
#include "mfma_tiles.h"
#include "tlr_internal.h"

namespace tlr {
namespace {

// Value of a double in lane `lane` (wave-uniform) of the wave.
__device__ inline double lane_value(double v, int lane) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Largest unsigned key over each row of 16 lanes (rotations within the row).
__device__ inline unsigned row_max16(unsigned k) {
  k = max(k, (unsigned)__builtin_amdgcn_update_dpp(0, (int)k, 0x128, 0xf, 0xf, false));  // row_ror:8
  k = max(k, (unsigned)__builtin_amdgcn_update_dpp(0, (int)k, 0x124, 0xf, 0xf, false));  // row_ror:4
  k = max(k, (unsigned)__builtin_amdgcn_update_dpp(0, (int)k, 0x122, 0xf, 0xf, false));  // row_ror:2
  k = max(k, (unsigned)__builtin_amdgcn_update_dpp(0, (int)k, 0x121, 0xf, 0xf, false));  // row_ror:1
  return k;
}

// Gram partials of a block of rows, one 16-row strip at a time: X (ld ldx)
// holds rows [0, 16 nstrips) of the block in LDS, part receives, for strip
// s, the Dot2 sums of X(16 s : 16 s + 16, a) . X(.., b) for a <= b < nc as
// (hi, lo) at part + s * bs * bs * 2 + (a + b * bs) * 2.
__device__ inline void strip_grams(const double* X, int ldx, int nstrips, int nc, int bs,
                                   double* part) {
  const int npairs = nc * (nc + 1) / 2;
  for (int e = threadIdx.x; e < nstrips * npairs; e += blockDim.x) {
    const int st = e / npairs, pr = e % npairs;
    int b = (int)((sqrt(8.0 * pr + 1.0) - 1.0) * 0.5);
    while (b * (b + 1) / 2 > pr) --b;
    while ((b + 1) * (b + 2) / 2 <= pr) ++b;
    const int a = pr - b * (b + 1) / 2;
    double sh = 0.0, sl = 0.0;
    for (int r = 0; r < 16; ++r) dot2_step(X[16 * st + r + a * ldx], X[16 * st + r + b * ldx], sh, sl);
    const dd v = fast_two_sum(sh, sl);
    gdouble* o = gmem(part) + (size_t)st * bs * bs * 2 + (a + b * bs) * 2;
    o[0] = v.hi;
    o[1] = v.lo;
  }
}

// ------------------------------------- Cholesky QR step: factor + apply
// One kernel per pass.  Every workgroup of a tile sums the partial Gram
// matrices, factors the BS x BS Gram, then turns its own block of APPLY_ROWS
// rows into new basis rows by a triangular solve with R.  The factorization
// is repeated by the workgroups of a tile (it is tiny and deterministic, so
// all of them reach the same R); only the first writes the pivot record.
//
// Pass 1 (PIV): diagonally pivoted Cholesky with the threshold tau^2 on the
// Schur-complement diagonal.  Column j is accepted while the largest
// remaining diagonal (the squared norm of a sample column after removing
// the accepted directions) exceeds tau^2; p accepted pivots give
// Y_P = Q_new R, R p x p upper triangular in pivot order.  The tile has
// converged when at least r_min samples were left below tau, or the basis
// has reached its capacity.
// Pass 2: unpivoted Cholesky of the Gram of the p new columns (already
// orthogonal to about u * cond, so the Gram is close to the identity);
// the columns are replaced in place.
//
// The dd Gram is spread over the workgroup: thread t = x + BS g holds row x,
// columns g CPG .. g CPG + CPG - 1, in registers, and mirrors them to one
// of two LDS copies (read one, write the other: one barrier per step).  At
// each step every wave finds the pivot on its own (a lane per column and a
// reduction across lanes) and every thread reads the pivot row from LDS;
// symmetry is exact because the partial sums are shared and the dd product
// is commutative.
constexpr int APPLY_ROWS = 256;

template <int BS, bool PIV>
__device__ inline void orth_body(const AraDev& D, int r_min, int bx, int by) {
  constexpr int NG = APPLY_ROWS / BS;
  constexpr int CPG = (BS + NG - 1) / NG;
  constexpr int XR = 64;   // rows of X staged at a time for the pass-1 strip Grams
  constexpr int GSZ = BS * (BS + 1);
  constexpr int SMEM = (4 * GSZ > BS * (XR + 1)) ? 4 * GSZ : BS * (XR + 1);
  // two dd copies of the Gram (read one, write the other: one barrier per
  // step), reused for the X staging once the factor is done
  __shared__ double smem[SMEM];
  __shared__ double Lm[BS][BS + 1];   // Lm[j][b]: Schur-complement row of the pivot of step j
  __shared__ double dpiv[BS];         // its diagonal (pass 1)
  __shared__ double Rs[BS][BS + 1];   // R(a, c), a <= c
  __shared__ int perm[BS];
  // copy s of the Gram: (dd (*)[BS + 1])(smem + 2 * GSZ * s)
  double (*Xs)[XR + 1] = (double (*)[XR + 1])smem;
  // the slot and the active count are read together (act has an entry
  // for every block row of the launch), and then every per-slot value, so
  // that two memory latencies precede the Gram partials; pass 2 takes the
  // accepted count from the basis widths (qnew = q + accepted) rather than
  // from the pivot record, one dependent load fewer
  const int slot = D.act[by];
  if ((int)by >= D.counts[0]) return;
  const AraSlotDesc& d = D.slots[slot];
  const int m = D.m, qcap = D.qcap, nrb = D.nstrip;
  const int qold = D.qin[slot];
  const int qnew = PIV ? 0 : D.qnew[slot];
  const double tau2 = d.tau2;
  const double* part = PIV ? d.part1 + D.poff : d.part2;
  const int t = threadIdx.x, lane = t & 63;
  const int x = t % BS, g = t / BS;
  const int nc = PIV ? BS : qnew - qold;
  if (nc == 0) return;
  // ---- sum of the partial Gram matrices (stored for a <= b).  Thread t
  // sums the pairs p = t, t + APPLY_ROWS, ... of the upper triangle (b
  // major: entry e = a + b BS, a <= b; at most three per thread when
  // BS = 32) over the strips with one 16-byte (hi, lo) load per strip,
  // nearby threads reading nearby entries of a strip, in chunks of PCH
  // strips all in flight before the sums (one round for m <= 1024 in pass
  // 1; pass 2 runs inside the fused sampling launch, whose occupancy the
  // registers of a larger chunk would halve); the sums go to copy 0 of the
  // Gram in LDS, both triangles (entries beyond nc are zero).
  constexpr int PCH = PIV ? 64 : 32;
  dd (*G0)[BS + 1] = (dd (*)[BS + 1])smem;
  constexpr int NPAIR = BS * (BS + 1) / 2;
  for (int p = t; p < NPAIR; p += APPLY_ROWS) {
    int b = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
    while (b * (b + 1) / 2 > p) --b;
    while ((b + 1) * (b + 2) / 2 <= p) ++b;
    const int a = p - b * (b + 1) / 2;
    const int e = a + b * BS;
    dd acc{0.0, 0.0};
    if (b < nc) {
      // compensated summation (Sum2 of Ogita, Rump and Oishi): the running
      // sum is the only dependency chain, the rounding errors and the low
      // parts are gathered beside it
      const gdv2* pp = (const gdv2*)(gmem(part) + (size_t)e * 2);
      double sh = 0.0, sc = 0.0;
      for (int rb0 = 0; rb0 < nrb; rb0 += PCH) {
        dv2 pv[PCH];
#pragma unroll
        for (int u = 0; u < PCH; ++u) pv[u] = pp[(size_t)min(rb0 + u, nrb - 1) * BS * BS];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < PCH; ++u)
          if (rb0 + u < nrb) {
            const dd t2 = two_sum(sh, pv[u].x);
            sh = t2.hi;
            sc += t2.lo + pv[u].y;
          }
      }
      acc = fast_two_sum(sh, sc);
    }
    G0[a][b] = acc;
    G0[b][a] = acc;
  }
  __syncthreads();
  dd gv[CPG];
#pragma unroll
  for (int i = 0; i < CPG; ++i) {
    const int b = g * CPG + i;
    gv[i] = (g < NG && b < BS) ? G0[x][b] : dd{0.0, 0.0};
  }
  for (int e = t; e < BS * (BS + 1); e += APPLY_ROWS) {
    (&Lm[0][0])[e] = 0.0;
    (&Rs[0][0])[e] = 0.0;
  }
  __syncthreads();
  int np = 0;
  if (PIV) {
    const int room = max(0, qcap - qold);
    unsigned taken = 0u;
    for (int j = 0; j < BS && j < room; ++j) {
      dd (*Gr)[BS + 1] = (dd (*)[BS + 1])(smem + 2 * GSZ * (j & 1));
      dd (*Gw)[BS + 1] = (dd (*)[BS + 1])(smem + 2 * GSZ * ((j & 1) ^ 1));
      // pivot.  Lane c of a row of 16 lanes (lane c of the first two rows
      // when BS > 16) holds column c's key: the upper word of its remaining
      // diagonal (positive, so the bits order like the values) with the
      // low five bits replaced by 31 - c; taken columns and non-positive
      // diagonals have key 0.  The largest key names a column whose
      // diagonal is within a relative 2^-15 of the largest, ties to the
      // lowest column.  Every lane forms the reciprocal of its diagonal
      // beside the reduction; the pivot's comes from the pivot's lane.
      const int cl = (BS > 16) ? (lane & 31) : (lane & 15);
      dd dc{1.0, 0.0};
      unsigned key = 0u;
      if (cl < BS) {
        dc = Gr[cl][cl];
        if (!((taken >> cl) & 1u) && dc.hi > 0.0)
          key = ((unsigned)((unsigned long long)__double_as_longlong(dc.hi) >> 32) & ~31u) |
                (31u - (unsigned)cl);
      }
      dd ic = dd_recip(dc);
      key = row_max16(key);
      unsigned kmax = __builtin_amdgcn_readlane(key, 0);
      if (BS > 16) kmax = max(kmax, (unsigned)__builtin_amdgcn_readlane(key, 16));
      // keep the reciprocal ahead of the exit test (the compiler would sink
      // it past the branch, onto the dependency chain of the update)
      asm volatile("" : "+v"(ic.hi), "+v"(ic.lo));
      if (kmax == 0u) break;
      const int pv = 31 - (int)(kmax & 31u);
      const dd dpp{lane_value(dc.hi, pv), lane_value(dc.lo, pv)};
      if (!(dpp.hi > tau2)) break;
      const dd invd{lane_value(ic.hi, pv), lane_value(ic.lo, pv)};
      // Schur update G(x, b) -= G(x, pv) G(pv, b) / d, d = G(pv, pv).  The
      // row of R is G(pv, b) / sqrt(d); its unscaled values and d are kept
      // and scaled after the loop, off the dependency chain.
      const dd gx = ((taken >> x) & 1u) ? dd{0.0, 0.0} : Gr[x][pv];
#pragma unroll
      for (int i = 0; i < CPG; ++i) {
        const int b = g * CPG + i;
        if (g < NG && b < BS) {
          const bool tb = (taken >> b) & 1u;
          const dd gpb = tb ? dd{0.0, 0.0} : Gr[pv][b];
          const dd pr = dd_mul(gx, gpb);
          gv[i] = dd_sub_sloppy(gv[i], dd_mul(pr, invd));
          Gw[x][b] = gv[i];
          if (x == 0) Lm[j][b] = gpb.hi + gpb.lo;
        }
      }
      if (t == 0) dpiv[j] = dpp.hi + dpp.lo;
      if (t == 0) perm[j] = pv;
      taken |= 1u << pv;
      np = j + 1;
      __syncthreads();
    }
    if (t == 0) {
      int nxt = np;
      for (int c = 0; c < BS; ++c)
        if (!((taken >> c) & 1u)) perm[nxt++] = c;
    }
    __syncthreads();
    // R in pivot order: R(jj, i) = Lm[jj][perm[i]] / sqrt(d_jj) for i >= jj
    for (int e = t; e < BS * BS; e += APPLY_ROWS) {
      const int jj = e % BS, i = e / BS;
      if (jj < np && i < np && i >= jj) Rs[jj][i] = Lm[jj][perm[i]] / sqrt(dpiv[jj]);
    }
    if (bx == 0) {
      if (t < BS) d.piv[t] = perm[t];
      if (t == 0) {
        d.piv[BS] = np;
        D.qnew[slot] = qold + np;
        D.qout[slot] = qold + np;
        D.q[slot] = qold + np;
        D.flag[slot] = ((np <= BS - r_min) || (qold + np >= qcap)) ? 1 : 0;
        D.iters[slot] += 1;
        D.qsum[slot] += qold * BS;
        D.ncol[slot] += BS;
      }
    }
  } else {
    // pass 2: the Gram of the new columns is within u * cond of the
    // identity, so its Cholesky factor is taken in FP64 (the Gram itself
    // was summed with compensation)
    np = nc;
    double gd[CPG];
#pragma unroll
    for (int i = 0; i < CPG; ++i) gd[i] = gv[i].hi + gv[i].lo;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
      const int b = g * CPG + i;
      if (g < NG && b < BS) ((double (*)[BS + 1])smem)[x][b] = gd[i];
    }
    __syncthreads();
    for (int j = 0; j < nc; ++j) {
      double (*Gr)[BS + 1] = (double (*)[BS + 1])(smem + GSZ * (j & 1));
      double (*Gw)[BS + 1] = (double (*)[BS + 1])(smem + GSZ * ((j & 1) ^ 1));
      const double gjj = Gr[j][j];
      double gj = 1.0, rinv = 1.0;
      if (gjj > 0.0) {
        gj = sqrt(gjj);
        rinv = 1.0 / gj;
      }
      const double lx = (x > j && x < nc) ? Gr[x][j] * rinv : 0.0;
#pragma unroll
      for (int i = 0; i < CPG; ++i) {
        const int b = g * CPG + i;
        const double lb = (b > j && b < nc) ? Gr[j][b] * rinv : (b == j ? gj : 0.0);
        if (g < NG && b < BS) {
          if (x > j && b > j) {
            gd[i] = fma(-lx, lb, gd[i]);
            Gw[x][b] = gd[i];
          }
          if (x == 0 && b >= j) Rs[j][b] = lb;
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // ---- apply: rows of Q_new from Y_P = Q_new R (pass 1) or X = Q_new R
  // (pass 2, in place), by forward substitution along the row
  const int r = bx * APPLY_ROWS + t;
  if (np == 0) return;
  gdouble* dst = gmem(d.q) + (size_t)qold * m;
  const gdouble* ysrc = gmem(d.y + D.yoff);
  double xv[BS], rd[BS];
#pragma unroll
  for (int a = 0; a < BS; ++a) {
    xv[a] = 0.0;
    rd[a] = (a < np) ? 1.0 / Rs[a][a] : 0.0;   // off the substitution's dependency chain
  }
  if (r < m) {
#pragma unroll
    for (int a = 0; a < BS; ++a)
      if (a < np) xv[a] = PIV ? ysrc[r + (size_t)perm[a] * m] : dst[r + (size_t)a * m];
#pragma unroll
    for (int c = 0; c < BS; ++c) {
      if (c < np) {
        double v = xv[c];
#pragma unroll
        for (int a = 0; a < c; ++a) v = fma(-xv[a], Rs[a][c], v);
        v *= rd[c];
        xv[c] = v;
        dst[r + (size_t)c * m] = v;
      }
    }
  }
  // pass 1 on an empty basis: no block Gram-Schmidt step follows, so the
  // Gram partials of the new columns for pass 2 are formed here
  if (PIV && qold == 0) {
    for (int h = 0; h < APPLY_ROWS / XR; ++h) {
      if (t / XR == h) {
#pragma unroll
        for (int a = 0; a < BS; ++a) Xs[a][t % XR] = xv[a];
      }
      __syncthreads();
      const int strip0 = (bx * APPLY_ROWS + h * XR) / 16;
      const int ns = min(XR / 16, nrb - strip0);
      if (ns > 0)
        strip_grams(&Xs[0][0], XR + 1, ns, np, BS, d.part2 + (size_t)strip0 * BS * BS * 2);
      __syncthreads();
    }
  }
}


}  // namespace
}  // namespace tlr
