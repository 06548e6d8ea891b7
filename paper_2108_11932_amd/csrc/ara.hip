// Kernels of the batched adaptive randomized approximation (Section 3.1 and
// Algorithm "Left Looking Cholesky TLR ARA Update", Section 4.2):
//
//  * batchRandn      -- Philox4x32-10 + Box-Muller Gaussian test matrices
//  * batchOrthog     -- block Gram-Schmidt, the QR of each block done by a
//                       Cholesky QR whose Gram matrix and Cholesky factor are
//                       carried in double-double (the paper's mixed-precision
//                       Cholesky QR), with diagonal pivoting and a threshold
//                       so that the rank is found column by column
//  * getConvergedTiles / updateSubset -- convergence flags and the stable
//                       compaction + refill of the active subset
//  * sortRanks       -- order of the tiles of a column by input rank
#include "tlr_internal.h"

// The double-double arithmetic below relies on error-free transformations
// that must see every product and sum rounded separately: no contraction of
// a*b + c into fused multiply-adds in this file (explicit fma() calls stay).
#pragma clang fp contract(off)

namespace tlr {

namespace {

// ------------------------------------------------------------------ Philox
constexpr unsigned PH_M0 = 0xD2511F53u, PH_M1 = 0xCD9E8D57u;
constexpr unsigned PH_W0 = 0x9E3779B9u, PH_W1 = 0xBB67AE85u;

__device__ inline uint4 philox10(uint4 c, unsigned k0, unsigned k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += PH_W0; k1 += PH_W1; }
    const unsigned hi0 = __umulhi(PH_M0, c.x), lo0 = PH_M0 * c.x;
    const unsigned hi1 = __umulhi(PH_M1, c.z), lo1 = PH_M1 * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

__device__ inline double u53(unsigned hi, unsigned lo) {
  return ((double)(hi >> 5) * 67108864.0 + (double)(lo >> 6)) * (1.0 / 9007199254740992.0);
}

__global__ void k_randn(double* out, int rows, int cols, int ld, unsigned k0, unsigned k1,
                        unsigned k, unsigned t, unsigned strm) {
  const long long n = (long long)rows * cols;
  const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (2 * c >= n) return;
  const uint4 w = philox10(make_uint4((unsigned)c, t, k, strm), k0, k1);
  const double u1 = 1.0 - u53(w.x, w.y);
  const double u2 = u53(w.z, w.w);
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos(6.283185307179586476925286766559 * u2, &sn, &cs);
  long long e = 2 * c;
  out[(e % rows) + (e / rows) * (long long)ld] = rad * cs;
  if (e + 1 < n) {
    e += 1;
    out[(e % rows) + (e / rows) * (long long)ld] = rad * sn;
  }
}

__global__ void k_philox_raw(unsigned* out, int n, unsigned k0, unsigned k1, unsigned c1,
                             unsigned c2, unsigned c3) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const uint4 w = philox10(make_uint4((unsigned)c, c1, c2, c3), k0, k1);
  out[4 * c + 0] = w.x;
  out[4 * c + 1] = w.y;
  out[4 * c + 2] = w.z;
  out[4 * c + 3] = w.w;
}

// ------------------------------------------------------------ double-double
// Error-free transformations (Knuth TwoSum, FMA-based TwoProduct) and the
// double-double operations built on them (Dekker; Bailey's QD library).
struct dd {
  double hi, lo;
};
__device__ inline dd two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ inline dd fast_two_sum(double a, double b) {
  const double s = a + b;
  return {s, b - (s - a)};
}
__device__ inline dd two_prod(double a, double b) {
  const double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ inline dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  const dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
__device__ inline dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
__device__ inline dd dd_mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p.hi, p.lo);
}
__device__ inline dd dd_div(dd a, dd b) {
  const double q1 = a.hi / b.hi;
  dd r = dd_sub(a, dd_mul(b, dd{q1, 0.0}));
  const double q2 = r.hi / b.hi;
  r = dd_sub(r, dd_mul(b, dd{q2, 0.0}));
  const double q3 = r.hi / b.hi;
  const dd q = fast_two_sum(q1, q2);
  return dd_add(q, dd{q3, 0.0});
}
__device__ inline dd dd_sqrt(dd a) {
  if (!(a.hi > 0.0)) return {0.0, 0.0};
  const double x = 1.0 / sqrt(a.hi);
  const double ax = a.hi * x;
  const dd diff = dd_sub(a, two_prod(ax, ax));
  return fast_two_sum(ax, diff.hi * (x * 0.5));
}

// ------------------------------------------------------------ Gram matrices
// Partial Gram sums X^T X over a block of rows, accumulated with the
// compensated dot product of Ogita, Rump and Oishi (Dot2) and stored as
// unevaluated (hi, lo) pairs.  X is the first `nc` columns of the block;
// nc comes from the tile's pivot record when ncols_from_piv is set.
constexpr int GRAM_ROWS = 64;
constexpr int BS_MAX = 32;

__global__ __launch_bounds__(256) void k_gram_dd(const OrthDesc* __restrict__ descs, int m, int bs,
                                                 int pass, int nrb) {
  __shared__ double X[BS_MAX][GRAM_ROWS + 1];
  const OrthDesc d = descs[blockIdx.y];
  const int rb = blockIdx.x;
  const int r0 = rb * GRAM_ROWS;
  const int rows = min(GRAM_ROWS, m - r0);
  const double* src;
  int nc;
  if (pass == 1) {
    src = d.Y;
    nc = bs;
  } else {
    nc = d.piv[bs];
    src = d.Q + (size_t)d.qold * m;
  }
  const int tid = threadIdx.x;
  for (int e = tid; e < nc * GRAM_ROWS; e += blockDim.x) {
    const int r = e % GRAM_ROWS, c = e / GRAM_ROWS;
    X[c][r] = (r < rows) ? src[(r0 + r) + (size_t)c * m] : 0.0;
  }
  __syncthreads();
  const int npairs = nc * (nc + 1) / 2;
  double* out = d.part + (size_t)rb * bs * bs * 2;
  for (int pr = tid; pr < npairs; pr += blockDim.x) {
    // pair index -> (a, b), a <= b, column-by-column upper triangle
    int b = (int)((sqrt(8.0 * pr + 1.0) - 1.0) * 0.5);
    while (b * (b + 1) / 2 > pr) --b;
    while ((b + 1) * (b + 2) / 2 <= pr) ++b;
    const int a = pr - b * (b + 1) / 2;
    double s = 0.0, c = 0.0;
    for (int r = 0; r < rows; ++r) {
      const double x = X[a][r], y = X[b][r];
      const double p = x * y;
      const double e = fma(x, y, -p);
      const double t = s + p;
      const double z = t - s;
      const double q = (s - (t - z)) + (p - z);
      s = t;
      c += q + e;
    }
    const dd v = fast_two_sum(s, c);
    out[(a + b * bs) * 2 + 0] = v.hi;
    out[(a + b * bs) * 2 + 1] = v.lo;
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
// columns g CPG .. g CPG + CPG - 1, in registers, and mirrors them to LDS,
// from which every thread reads the pivot column at each step (one LDS
// exchange and two barriers per step; symmetry is exact because the
// partial sums are shared and the dd product is commutative).
constexpr int APPLY_ROWS = 256;

template <int BS, bool PIV>
__global__ __launch_bounds__(APPLY_ROWS) void k_orth_step(const OrthDesc* __restrict__ descs, int m,
                                                          int nrb, double tau2, int r_min,
                                                          int qcap) {
  constexpr int NG = APPLY_ROWS / BS;
  constexpr int CPG = (BS + NG - 1) / NG;
  __shared__ dd Gs[BS][BS + 1];
  __shared__ double Lm[BS][BS + 1];   // Lm[j][b]: multiplier of column b at step j
  __shared__ double Rs[BS][BS + 1];   // R(a, c), a <= c
  __shared__ int perm[BS];
  const OrthDesc d = descs[blockIdx.y];
  const int t = threadIdx.x;
  const int x = t % BS, g = t / BS;
  const int nc = PIV ? BS : d.piv[BS];
  if (nc == 0) return;
  // ---- sum of the partial Gram matrices (stored for a <= b)
  dd gv[CPG];
#pragma unroll
  for (int i = 0; i < CPG; ++i) {
    const int b = g * CPG + i;
    dd acc{0.0, 0.0};
    if (g < NG && b < nc && x < nc) {
      const int lo = min(x, b), hi = max(x, b);
      const double* pp = d.part + (size_t)(lo + hi * BS) * 2;
      for (int rb = 0; rb < nrb; ++rb) {
        const double* q2 = pp + (size_t)rb * BS * BS * 2;
        acc = dd_add(acc, dd{q2[0], q2[1]});
      }
    }
    gv[i] = acc;
    if (g < NG && b < BS) Gs[x][b] = acc;
  }
  for (int e = t; e < BS * (BS + 1); e += APPLY_ROWS) {
    (&Lm[0][0])[e] = 0.0;
    (&Rs[0][0])[e] = 0.0;
  }
  __syncthreads();
  int np = 0;
  if (PIV) {
    const int room = max(0, qcap - d.qold);
    unsigned taken = 0u;
    for (int j = 0; j < BS && j < room; ++j) {
      // pivot: largest remaining diagonal, ties to the lowest column
      double vmax = -1.0;
      int pv = BS;
      for (int c = 0; c < BS; ++c) {
        const double v = Gs[c][c].hi;
        if (!((taken >> c) & 1u) && v > vmax) {
          vmax = v;
          pv = c;
        }
      }
      if (!(vmax > tau2)) break;
      const dd rinv = dd_div(dd{1.0, 0.0}, dd_sqrt(Gs[pv][pv]));
      const dd lx = ((taken >> x) & 1u) ? dd{0.0, 0.0} : dd_mul(Gs[x][pv], rinv);
      dd lb[CPG];
#pragma unroll
      for (int i = 0; i < CPG; ++i) {
        const int b = g * CPG + i;
        lb[i] = (b < BS && !((taken >> b) & 1u)) ? dd_mul(Gs[pv][b], rinv) : dd{0.0, 0.0};
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < CPG; ++i) {
        const int b = g * CPG + i;
        if (g < NG && b < BS) {
          gv[i] = dd_sub(gv[i], dd_mul(lx, lb[i]));
          Gs[x][b] = gv[i];
          if (x == 0) Lm[j][b] = lb[i].hi + lb[i].lo;
        }
      }
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
    // R in pivot order: R(jj, i) = Lm[jj][perm[i]] for i >= jj
    for (int e = t; e < BS * BS; e += APPLY_ROWS) {
      const int jj = e % BS, i = e / BS;
      if (jj < np && i < np && i >= jj) Rs[jj][i] = Lm[jj][perm[i]];
    }
    if (blockIdx.x == 0) {
      if (t < BS) d.piv[t] = perm[t];
      if (t == 0) {
        d.piv[BS] = np;
        *d.q = d.qold + np;
        *d.flag = ((np <= BS - r_min) || (d.qold + np >= qcap)) ? 1 : 0;
      }
    }
  } else {
    np = nc;
    for (int j = 0; j < nc; ++j) {
      dd gj = dd_sqrt(Gs[j][j]);
      if (gj.hi == 0.0) gj = dd{1.0, 0.0};
      const dd rinv = dd_div(dd{1.0, 0.0}, gj);
      const dd lx = (x > j && x < nc) ? dd_mul(Gs[x][j], rinv) : dd{0.0, 0.0};
      dd lb[CPG];
#pragma unroll
      for (int i = 0; i < CPG; ++i) {
        const int b = g * CPG + i;
        lb[i] = (b > j && b < nc) ? dd_mul(Gs[j][b], rinv) : (b == j ? gj : dd{0.0, 0.0});
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < CPG; ++i) {
        const int b = g * CPG + i;
        if (g < NG && b < BS) {
          if (x > j && b > j) {
            gv[i] = dd_sub(gv[i], dd_mul(lx, lb[i]));
            Gs[x][b] = gv[i];
          }
          if (x == 0 && b >= j) Rs[j][b] = lb[i].hi + lb[i].lo;
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // ---- apply: rows of Q_new from Y_P = Q_new R (pass 1) or X = Q_new R
  // (pass 2, in place), by forward substitution along the row
  const int r = blockIdx.x * APPLY_ROWS + t;
  if (r >= m || np == 0) return;
  double* dst = d.Q + (size_t)d.qold * m;
  double xv[BS];
#pragma unroll
  for (int a = 0; a < BS; ++a)
    if (a < np) xv[a] = PIV ? d.Y[r + (size_t)perm[a] * m] : dst[r + (size_t)a * m];
#pragma unroll
  for (int c = 0; c < BS; ++c) {
    if (c < np) {
      double v = xv[c];
#pragma unroll
      for (int a = 0; a < c; ++a) v = fma(-xv[a], Rs[a][c], v);
      v = v / Rs[c][c];
      xv[c] = v;
      dst[r + (size_t)c * m] = v;
    }
  }
}

// ------------------------------------------------------- dynamic batching
// Stable compaction of the active list (slots whose flag is set leave) and
// refill from the waiting list, keeping at most s_max tiles.  One workgroup.
__global__ __launch_bounds__(256) void k_compact(int* act, int* counts, const int* flag,
                                                 const int* waiting, int nwaiting, int s_max,
                                                 const int* info) {
  __shared__ int keep_total;
  __shared__ int scan[256];
  const int tid = threadIdx.x;
  const int n = counts[0];
  if (tid == 0) keep_total = 0;
  __syncthreads();
  // in-place stable compaction, processed in chunks of 256 entries; writes
  // never overtake reads because pos <= index
  for (int base = 0; base < n; base += 256) {
    const int i = base + tid;
    int slot = -1, keep = 0;
    if (i < n) {
      slot = act[i];
      keep = flag[slot] ? 0 : 1;
    }
    scan[tid] = keep;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int v = (tid >= off) ? scan[tid - off] : 0;
      __syncthreads();
      scan[tid] += v;
      __syncthreads();
    }
    const int pos = keep_total + scan[tid] - keep;
    const int chunk_keep = scan[255];
    __syncthreads();
    if (keep) act[pos] = slot;
    __syncthreads();
    if (tid == 0) keep_total += chunk_keep;
    __syncthreads();
  }
  const int kept = keep_total;
  const int cursor = counts[1];
  const int take = max(0, min(min(n - kept, s_max - kept), nwaiting - cursor));
  for (int j = tid; j < take; j += blockDim.x) act[kept + j] = waiting[cursor + j];
  __syncthreads();
  if (tid == 0) {
    counts[0] = kept + take;
    counts[1] = cursor + take;
    if (info) counts[2] = *info;
  }
}

// order[p] = rows sorted by (rank descending, row ascending): the position of
// element i is the number of elements that precede it.
__global__ void k_sort_ranks(const int* ranks, const int* rows, int n, int* order) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ri = ranks[i], wi = rows[i];
  int pos = 0;
  for (int j = 0; j < n; ++j) {
    const int rj = ranks[j], wj = rows[j];
    pos += (rj > ri || (rj == ri && wj < wi)) ? 1 : 0;
  }
  order[pos] = wi;
}

}  // namespace

hipError_t launch_randn(double* out, int rows, int cols, int ld, unsigned long long seed, unsigned k,
                        unsigned t, unsigned stream, hipStream_t s) {
  const long long pairs = ((long long)rows * cols + 1) / 2;
  if (pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_randn, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, out, rows,
                     cols, ld, (unsigned)(seed & 0xffffffffu), (unsigned)(seed >> 32), k, t,
                     stream);
  return hipGetLastError();
}

hipError_t launch_philox_raw(unsigned* out, int n, unsigned long long seed, unsigned c1,
                             unsigned c2, unsigned c3, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox_raw, dim3((n + 255) / 256), dim3(256), 0, s, out, n,
                     (unsigned)(seed & 0xffffffffu), (unsigned)(seed >> 32), c1, c2, c3);
  return hipGetLastError();
}

int gram_row_blocks(int m) { return (m + GRAM_ROWS - 1) / GRAM_ROWS; }

hipError_t launch_gram_dd(const OrthDesc* d, int ntiles, int m, int bs, int pass, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (bs > BS_MAX) return hipErrorInvalidValue;
  const int nrb = gram_row_blocks(m);
  hipLaunchKernelGGL(k_gram_dd, dim3(nrb, ntiles), dim3(256), 0, s, d, m, bs, pass, nrb);
  return hipGetLastError();
}

// KERNEL is a template-id whose block-size argument is spelled BS_ARG.
#define TLR_BS_CASE(v, KERNEL, ...)                    \
  case v: {                                            \
    constexpr int BS_ARG = v;                          \
    hipLaunchKernelGGL(KERNEL, __VA_ARGS__);           \
    break;                                             \
  }
#define TLR_BS_DISPATCH(bs, KERNEL, ...)               \
  switch (bs) {                                        \
    TLR_BS_CASE(16, KERNEL, __VA_ARGS__)               \
    TLR_BS_CASE(32, KERNEL, __VA_ARGS__)               \
    TLR_BS_CASE(8, KERNEL, __VA_ARGS__)                \
    TLR_BS_CASE(24, KERNEL, __VA_ARGS__)               \
    TLR_BS_CASE(4, KERNEL, __VA_ARGS__)                \
    TLR_BS_CASE(2, KERNEL, __VA_ARGS__)                \
    TLR_BS_CASE(1, KERNEL, __VA_ARGS__)                \
    default: return hipErrorInvalidValue;              \
  }

bool orth_block_supported(int bs) {
  return bs == 1 || bs == 2 || bs == 4 || bs == 8 || bs == 16 || bs == 24 || bs == 32;
}

hipError_t launch_orth_step(const OrthDesc* d, int ntiles, int m, int bs, int pass, double tau2,
                            int r_min, int qcap, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const int nrb = gram_row_blocks(m);
  const dim3 grid((m + APPLY_ROWS - 1) / APPLY_ROWS, ntiles);
  if (pass == 1) {
    TLR_BS_DISPATCH(bs, (k_orth_step<BS_ARG, true>), grid, dim3(APPLY_ROWS), 0, s, d, m, nrb, tau2,
                    r_min, qcap);
  } else {
    TLR_BS_DISPATCH(bs, (k_orth_step<BS_ARG, false>), grid, dim3(APPLY_ROWS), 0, s, d, m, nrb, tau2,
                    r_min, qcap);
  }
  return hipGetLastError();
}

hipError_t launch_compact(int* act, int* counts, const int* flag, const int* waiting, int nwaiting,
                          int s_max, const int* info, hipStream_t s) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(256), 0, s, act, counts, flag, waiting, nwaiting,
                     s_max, info);
  return hipGetLastError();
}

hipError_t launch_sort_ranks(const int* ranks, const int* rows, int n, int* order, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_ranks, dim3((n + 255) / 256), dim3(256), 0, s, ranks, rows, n, order);
  return hipGetLastError();
}

}  // namespace tlr
