// Dense tile kernels: the latency-bound pieces of the blocked Cholesky and
// unpivoted LDL^T of the diagonal tiles, and the diagonal-block step of the
// blocked triangular solve.
//
// The diagonal tile factorization is the "chol" (Algorithm "Left Looking TLR
// Cholesky") and "ldl" (Algorithm "Left Looking TLR LDL^T", unpivoted with
// scalar pivots) step of the paper.  The tile is factored by blocks of 32
// columns: one launch per block factors the 32 x 32 diagonal block and
// solves the panel below it (L21 = A21 L11^{-T}), the trailing update runs
// as an MFMA GEMM.  The diagonal-block inverses, taken afterwards for all
// blocks in one launch, seed the assembly of L_kk^{-1}, so the batched
// triangular solve of a column ("batchTrsm", one triangle shared by every
// tile) becomes one product.
#include "tlr_internal.h"

namespace tlr {

namespace {

constexpr int NB = 64;   // block size of the blocked triangular solve
constexpr int ND = 32;   // diagonal block of the blocked factorizations

// Broadcast lane `lane` (a compile-time constant) of a double to the wave.
__device__ __forceinline__ double lane_bcast(double v, int lane) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Panel step of the blocked right-looking factorization.  Every workgroup
// (one wave) factors the w x w (w <= 32) diagonal block at (p0, p0) of A on
// its own -- Cholesky, or unit LDL^T with scalar pivots -- and then solves
// for its 64 rows of the panel below: Cholesky L21 = A21 L11^{-T} in place;
// LDL^T W21 = A21 L11^{-T} into W (row p0 + w + i at W[i], ld ldw) and
// L21 = W21 D^{-1} in place.  The factorization is deterministic, so every
// workgroup reaches the same L11; workgroup 0 stores the pivots, the
// failure record and L11 itself -- not into A, whose diagonal block the
// other workgroups may still be reading, but into Lst (ld ldst, zeros above
// the diagonal), from where the diagonal-block inversion moves it into A.
//
// Factor: lanes r and r + 32 hold the two halves of row r of the block in
// registers (rows and columns beyond w are the identity, which leaves the
// real part unchanged).  Right-looking: at step j the lanes holding column
// j put it into LDS, and by symmetry that column is also row j, so each
// lane reads d = S(j, j), its own S(r, j) and the S(c, j) of its half as
// LDS broadcasts and subtracts S(r, j) S(c, j) / d from S(r, c); column j
// of the factor goes to LDS at once.  Two column buffers alternate.  Solve: thread i takes row p0 + w + 64 b
// + i of A21 and runs the forward substitution against L11 (LDS) along it.
template <bool CHOL>
__global__ __launch_bounds__(64) void k_chol_panel(double* A, int lda, int m, int p0, int w,
                                                   double* W, int ldw, double* Lst, int ldst,
                                                   double* dvec, int* info, int row_base,
                                                   const double* tolp) {
  __shared__ double colb[2][ND];
  __shared__ double Ls[ND][ND + 1];   // Ls[r][q] = L(r, q), q <= r
  __shared__ double Rd[ND];           // 1 / L(c, c) (Cholesky)
  __shared__ double Ds[ND];           // LDL^T pivots
  const int lane = threadIdx.x;
  const int r = lane & (ND - 1);
  const int hf = lane >> 5;         // this lane holds columns [16 hf, 16 hf + 16) of row r
  const bool act = lane < ND;
  constexpr int HC = ND / 2;
  double row[HC];
#pragma unroll
  for (int cc = 0; cc < HC; ++cc) {
    const int c = HC * hf + cc;
    double v = (r == c) ? 1.0 : 0.0;
    if (r < w && c < w && c <= r) v = A[(p0 + r) + (size_t)(p0 + c) * lda];
    row[cc] = v;
  }
  // Cholesky with tolp set: modified Cholesky, a non-positive pivot d is
  // replaced by max(|d|, delta), delta = *tolp (a diagonal perturbation of
  // the tile that keeps the pivot as large as the loss it repairs) and
  // counted in info[1] instead of failing
  const bool modify = CHOL && tolp != nullptr;
  const double tol = CHOL ? (modify ? *tolp : 0.0) : *tolp;
  int bad_row = 0, nmod = 0;
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    double* cb = colb[j & 1];
    if (hf == j / HC) cb[r] = row[j % HC];
    // the workgroup is one wave, whose LDS operations complete in issue
    // order: the reads below see the write above without a wait for it
    __builtin_amdgcn_wave_barrier();
    // all reads of the step in flight at once
    double d = cb[j];
    const double a = cb[r];              // S(r, j)
    double cv[HC];
#pragma unroll
    for (int cc = 0; cc < HC; ++cc) cv[cc] = cb[HC * hf + cc];
    __builtin_amdgcn_sched_barrier(0);
    const bool bad = CHOL ? !(d > 0.0) : !(fabs(d) > tol);
    if (bad && modify) {
      if (j < w) ++nmod;
      d = fmax(fabs(d), tol);
    } else if (bad) {
      if (j < w && bad_row == 0) bad_row = row_base + p0 + j + 1;
      d = 1.0;
    }
    // 1/sqrt(d) (Cholesky) or 1/d from the hardware estimate and two Newton
    // steps: a handful of FMAs instead of the division and square-root
    // sequences on the step's dependency chain
    double rs = 0.0, rd;
    if (CHOL) {
      rs = __builtin_amdgcn_rsq(d);
#pragma unroll
      for (int it = 0; it < 2; ++it) rs = fma(0.5 * rs, fma(-d * rs, rs, 1.0), rs);
      rd = rs * rs;
    } else {
      rd = __builtin_amdgcn_rcp(d);
#pragma unroll
      for (int it = 0; it < 2; ++it) rd = fma(rd, fma(-d, rd, 1.0), rd);
    }
    const double mr = a * rd;            // l_rj of the unit factor
    // every column of the half (finished columns and the upper triangle
    // only collect values that are never read again)
#pragma unroll
    for (int cc = 0; cc < HC; ++cc) row[cc] = fma(-mr, cv[cc], row[cc]);
    double lv;
    if (CHOL) {
      lv = (r == j) ? d * rs : (r > j ? a * rs : 0.0);
      if (lane == j) Rd[j] = rs;
    } else {
      lv = (r == j) ? 1.0 : (r > j ? mr : 0.0);
      if (lane == j) Ds[j] = d;
    }
    if (act) Ls[r][j] = lv;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    if (bad_row && lane == 0) atomicCAS(info, 0, bad_row);
    if (nmod && lane == 0) atomicAdd(info + 1, nmod);
#pragma unroll
    for (int q = 0; q < ND; ++q)
      if (act && r < w && q < w) Lst[r + (size_t)q * ldst] = (q <= r) ? Ls[r][q] : 0.0;
    if (!CHOL && act && r < w) dvec[p0 + r] = Ds[r];
  }
  __syncthreads();
  const int i = blockIdx.x * 64 + lane;
  const int gr = p0 + w + i;
  if (gr >= m) return;
  double x[ND];
#pragma unroll
  for (int c = 0; c < ND; ++c) x[c] = (c < w) ? A[gr + (size_t)(p0 + c) * lda] : 0.0;
#pragma unroll
  for (int c = 0; c < ND; ++c) {
    double v = x[c];
#pragma unroll
    for (int q = 0; q < c; ++q) v = fma(-x[q], Ls[c][q], v);
    x[c] = CHOL ? v * Rd[c] : v;
    // x[c] is finished here and row c + 1 of L11 is read only afterwards
    // (the compiler would otherwise read every row first and sink the
    // arithmetic to the stores, holding ~500 values in registers)
    asm volatile("" : "+v"(x[c])::"memory");
  }
#pragma unroll
  for (int c = 0; c < ND; ++c) {
    if (c < w) {
      if (CHOL) {
        A[gr + (size_t)(p0 + c) * lda] = x[c];
      } else {
        W[i + (size_t)c * ldw] = x[c];
        A[gr + (size_t)(p0 + c) * lda] = x[c] / Ds[c];
      }
    }
  }
}

// Diagonal blocks of a factored m x m tile, one wave per block (block b at
// (32 b, 32 b)): the panel steps left each lower factor L_bb in Inv; it is
// moved into A (zeros above its diagonal) and replaced in Inv by its
// inverse (unit diagonal when UNIT).  Lane r holds row r of the block and
// row r of X = L^{-1}: at step p lane p scales its row of X by 1 / L(p, p),
// then rows i > p lose L(i, p) X(p, :), with X(p, :) read from lane p.
template <bool UNIT>
__global__ __launch_bounds__(64) void k_diag_finish(double* A, int lda, int m, double* Inv,
                                                    int ldi) {
  const int p0 = blockIdx.x * ND;
  const int w = min(ND, m - p0);
  const int r = threadIdx.x & (ND - 1);
  const bool act = threadIdx.x < ND;
  double row[ND], x[ND];
#pragma unroll
  for (int c = 0; c < ND; ++c) {
    double v = (r == c) ? 1.0 : 0.0;
    if (r < w && c < w && c <= r) v = Inv[(p0 + r) + (size_t)(p0 + c) * ldi];
    row[c] = (UNIT && r == c) ? 1.0 : v;
    x[c] = (r == c) ? 1.0 : 0.0;
  }
#pragma unroll
  for (int c = 0; c < ND; ++c)
    if (act && r < w && c < w) A[(p0 + r) + (size_t)(p0 + c) * lda] = (c <= r) ? row[c] : 0.0;
#pragma unroll
  for (int p = 0; p < ND; ++p) {
    if (!UNIT) {
      const double inv = 1.0 / row[p];
      if (r == p) {
#pragma unroll
        for (int c = 0; c <= p; ++c) x[c] *= inv;
      }
    }
    const double lip = (r > p) ? row[p] : 0.0;
#pragma unroll
    for (int c = 0; c <= p; ++c) x[c] -= lip * lane_bcast(x[c], p);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int c = 0; c < ND; ++c)
    if (act && r < w && c < w) Inv[(p0 + r) + (size_t)(p0 + c) * ldi] = (r >= c) ? x[c] : 0.0;
}

// out(r, c) = in(r, c) * s[c] or / s[c] (column scaling, LDL^T panels).
__global__ void k_scale_cols(const double* in, int ldi, double* out, int ldo, const double* s,
                             int rows, int cols, int inverse) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)rows * cols) return;
  const int r = (int)(e % rows), c = (int)(e / rows);
  const double v = in[r + (size_t)c * ldi];
  out[r + (size_t)c * ldo] = inverse ? v / s[c] : v * s[c];
}

// X_p = L_pp^{-1} B_p or L_pp^{-T} B_p on rows [p0, p0 + w) of B: 64
// right-hand sides per workgroup, one thread per right-hand side, the
// triangle and the right-hand sides in LDS.
__global__ __launch_bounds__(64) void k_trsm_diag(const double* L, int ldl, double* B, int ldb,
                                                  int p0, int w, int n, int unit, int trans) {
  __shared__ double S[NB][NB + 1];   // S[c][r] = L(p0 + r, p0 + c)
  __shared__ double X[64][NB + 1];   // X[col][row]
  const int tid = threadIdx.x;
  const int col0 = blockIdx.x * 64;
  for (int e = tid; e < w * w; e += 64) {
    const int r = e % w, c = e / w;
    S[c][r] = (c <= r) ? L[(p0 + r) + (size_t)(p0 + c) * ldl] : 0.0;
  }
  for (int c = 0; c < 64; ++c) {
    const int gc = col0 + c;
    if (gc < n && tid < w) X[c][tid] = B[(p0 + tid) + (size_t)gc * ldb];
  }
  __syncthreads();
  if (col0 + tid < n) {
    double* x = X[tid];
    if (!trans) {
      for (int j = 0; j < w; ++j) {
        double v = x[j];
        for (int c = 0; c < j; ++c) v -= S[c][j] * x[c];
        x[j] = unit ? v : v / S[j][j];
      }
    } else {
      for (int j = w - 1; j >= 0; --j) {
        double v = x[j];
        for (int r = j + 1; r < w; ++r) v -= S[j][r] * x[r];
        x[j] = unit ? v : v / S[j][j];
      }
    }
  }
  __syncthreads();
  for (int c = 0; c < 64; ++c) {
    const int gc = col0 + c;
    if (gc < n && tid < w) B[(p0 + tid) + (size_t)gc * ldb] = X[c][tid];
  }
}

}  // namespace

int diag_block_size() { return ND; }

hipError_t launch_chol_panel(bool chol, double* A, int lda, int m, int p0, int w, double* W,
                             int ldw, double* Lst, int ldst, double* dvec, int* info, int row_base,
                             const double* tolp, hipStream_t s) {
  if (w <= 0 || w > ND || p0 < 0 || p0 + w > m || ldst < w) return hipErrorInvalidValue;
  const int rem = m - p0 - w;
  const unsigned nwg = (unsigned)(rem > 0 ? (rem + 63) / 64 : 1);
  if (chol)
    hipLaunchKernelGGL(k_chol_panel<true>, dim3(nwg), dim3(64), 0, s, A, lda, m, p0, w, W, ldw,
                       Lst, ldst, dvec, info, row_base, tolp);
  else
    hipLaunchKernelGGL(k_chol_panel<false>, dim3(nwg), dim3(64), 0, s, A, lda, m, p0, w, W, ldw,
                       Lst, ldst, dvec, info, row_base, tolp);
  return hipGetLastError();
}

hipError_t launch_diag_finish(bool unit, double* A, int lda, int m, double* Inv, int ldi,
                              hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const unsigned nblk = (unsigned)((m + ND - 1) / ND);
  if (unit)
    hipLaunchKernelGGL(k_diag_finish<true>, dim3(nblk), dim3(64), 0, s, A, lda, m, Inv, ldi);
  else
    hipLaunchKernelGGL(k_diag_finish<false>, dim3(nblk), dim3(64), 0, s, A, lda, m, Inv, ldi);
  return hipGetLastError();
}

hipError_t launch_scale_cols(const double* in, int ldi, double* out, int ldo, const double* sc,
                             int rows, int cols, bool inverse, hipStream_t s) {
  const long long n = (long long)rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, ldi, out,
                     ldo, sc, rows, cols, inverse ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_trsm_diag(const double* L, int ldl, double* B, int ldb, int p0, int w, int n,
                            bool unit, bool trans, hipStream_t s) {
  if (w <= 0 || w > NB || n <= 0) return w > NB ? hipErrorInvalidValue : hipSuccess;
  hipLaunchKernelGGL(k_trsm_diag, dim3((n + 63) / 64), dim3(64), 0, s, L, ldl, B, ldb, p0, w, n,
                     unit ? 1 : 0, trans ? 1 : 0);
  return hipGetLastError();
}

}  // namespace tlr
