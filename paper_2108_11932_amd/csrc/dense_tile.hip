// Dense tile kernels: the latency-bound pieces of the blocked Cholesky and
// unpivoted LDL^T of the diagonal tiles, and the diagonal-block step of the
// blocked triangular solve.
//
// The diagonal tile factorization is the "chol" (Algorithm "Left Looking TLR
// Cholesky") and "ldl" (Algorithm "Left Looking TLR LDL^T", unpivoted with
// scalar pivots) step of the paper.  The tile is factored by blocks of 32
// columns: one wave factors the 32 x 32 diagonal block in registers and also
// writes its inverse; the panel below (L21 = A21 L11^{-T}) and the trailing
// update then run as MFMA GEMMs.  The block inverses are reused to assemble
// L_kk^{-1}, so the batched triangular solve of a column ("batchTrsm", one
// triangle shared by every tile) becomes one product.
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

// Factor the diagonal block (p0, p0) of A (w <= 32) in place: Cholesky, or
// unit LDL^T with the pivots in dvec[p0..]; write the inverse of the lower
// factor into Inv (ld ldi).
//
// One wave; lane r holds row r of the block in registers (rows and columns
// beyond w are the identity, which leaves the real part unchanged; lanes
// 32..63 carry copies and store nothing).  Both loops are unrolled, so every
// register index is a constant and every cross-lane value is a readlane into
// scalar registers: no LDS round trip sits on the dependency chain.
// Right-looking: step j takes d = a_jj from lane j, each lane its own a_rj,
// and subtracts (a_rj / d) a_cj from a_rc, a_cj read from lane c.  The
// inverse X = L^{-1} is a forward substitution with row i of X on lane i:
// lane p finishes row p, whose entries are then read from lane p.
template <bool CHOL>
__global__ __launch_bounds__(64) void k_diag_block(double* A, int lda, int p0, int w, double* Inv,
                                                   int ldi, double* dvec, int* info, int row_base,
                                                   const double* tolp) {
  const int r = threadIdx.x & (ND - 1);
  const bool act = threadIdx.x < ND;
  double row[ND];
#pragma unroll
  for (int c = 0; c < ND; ++c) {
    double v = (r == c) ? 1.0 : 0.0;
    if (r < w && c < w && c <= r) v = A[(p0 + r) + (size_t)(p0 + c) * lda];
    row[c] = v;
  }
  const double tol = CHOL ? 0.0 : *tolp;
  int bad_row = 0;
  double dpiv = 1.0;   // this lane's pivot d_r
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    double d = lane_bcast(row[j], j);
    const bool bad = CHOL ? !(d > 0.0) : !(fabs(d) > tol);
    if (bad) {
      if (j < w && bad_row == 0) bad_row = row_base + p0 + j + 1;
      d = 1.0;
    }
    const double a = row[j];     // a_rj (unscaled)
    const double mr = a / d;     // l_rj of the unit factor
#pragma unroll
    for (int c = j + 1; c < ND; ++c) row[c] -= mr * lane_bcast(a, c);
    if (r == j) dpiv = d;
    if (CHOL) {
      const double sq = sqrt(d);
      row[j] = (r == j) ? sq : (r > j ? a / sq : 0.0);
    } else {
      row[j] = (r == j) ? 1.0 : (r > j ? mr : 0.0);
    }
    __builtin_amdgcn_sched_barrier(0);   // keep the scalar broadcasts of a step together
  }
  if (bad_row && threadIdx.x == 0) atomicCAS(info, 0, bad_row);
#pragma unroll
  for (int p = 0; p < ND; ++p)
    if (act && r < w && p < w) A[(p0 + r) + (size_t)(p0 + p) * lda] = (p <= r) ? row[p] : 0.0;
  if (!CHOL && act && r < w) dvec[p0 + r] = dpiv;
  // X = L^{-1}: at step p lane p scales its row by 1 / L(p, p); rows i > p
  // then lose L(i, p) X(p, :) (X(p, c) = 0 for c > p).
  double x[ND];
#pragma unroll
  for (int c = 0; c < ND; ++c) x[c] = (r == c) ? 1.0 : 0.0;
#pragma unroll
  for (int p = 0; p < ND; ++p) {
    if (CHOL) {
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
    if (act && r < w && c < w) Inv[r + (size_t)c * ldi] = (r >= c) ? x[c] : 0.0;
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

hipError_t launch_diag_block(bool chol, double* A, int lda, int p0, int w, double* Inv, int ldi,
                             double* dvec, int* info, int row_base, const double* tolp,
                             hipStream_t s) {
  if (w <= 0 || w > ND) return hipErrorInvalidValue;
  if (chol)
    hipLaunchKernelGGL(k_diag_block<true>, dim3(1), dim3(64), 0, s, A, lda, p0, w, Inv, ldi, dvec,
                       info, row_base, tolp);
  else
    hipLaunchKernelGGL(k_diag_block<false>, dim3(1), dim3(64), 0, s, A, lda, p0, w, Inv, ldi,
                       dvec, info, row_base, tolp);
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
