// Dense tile kernels: the latency-bound pieces of the blocked Cholesky and
// unpivoted LDL^T of the diagonal tiles, and the diagonal-block step of the
// blocked triangular solve.
//
// The diagonal tile factorization is the "chol" (Algorithm "Left Looking TLR
// Cholesky") and "ldl" (Algorithm "Left Looking TLR LDL^T", unpivoted with
// scalar pivots) step of the paper.  The tile is factored by blocks of 64
// columns: one workgroup factors the 64 x 64 diagonal block in LDS and also
// writes its inverse; the panel below (L21 = A21 L11^{-T}) and the trailing
// update then run as MFMA GEMMs.  The block inverses are reused to assemble
// L_kk^{-1}, so the batched triangular solve of a column ("batchTrsm", one
// triangle shared by every tile) becomes one product.
#include "tlr_internal.h"

namespace tlr {

namespace {

constexpr int NB = 64;   // block size of the blocked factorizations

// Factor the w x w lower block S (LDS, S[c][r] = block(r, c)) in LDL^T form
// with unscaled columns: after step j, S[j][r] (r > j) holds l_rj * d_j and
// d[j] the pivot.  One barrier per step.  Pivots failing `bad` are reported
// and replaced by 1 so no NaN spreads.
template <bool CHOL>
__device__ void block_factor(double (*S)[NB + 1], double* d, int w, int* info, int row_base,
                             double tol, bool report) {
  const int tid = threadIdx.x;
  for (int j = 0; j < w; ++j) {
    __syncthreads();
    double dj = S[j][j];
    const bool bad = CHOL ? !(dj > 0.0) : !(fabs(dj) > tol);
    if (bad) {
      if (report && tid == 0) atomicCAS(info, 0, row_base + j + 1);
      dj = 1.0;
    }
    if (tid == 0) d[j] = dj;
    const double inv = 1.0 / dj;
    const int nt = w - j - 1;
    for (int e = tid; e < nt * nt; e += blockDim.x) {
      const int r = j + 1 + e % nt, c = j + 1 + e / nt;
      if (c <= r) S[c][r] -= S[j][r] * S[j][c] * inv;
    }
  }
  __syncthreads();
}

// X = L^{-1} for the w x w lower triangle L held as S (unscaled LDL^T form
// with pivots d; CHOL: L = unit(S) * sqrt(D), else L = unit(S)).
// Column-oriented forward substitution on the identity, two barriers per step.
template <bool CHOL>
__device__ void block_inverse(double (*S)[NB + 1], const double* d, double (*X)[NB + 1], int w) {
  const int tid = threadIdx.x;
  for (int e = tid; e < w * w; e += blockDim.x) X[e / w][e % w] = (e % w == e / w) ? 1.0 : 0.0;
  for (int j = 0; j < w; ++j) {
    __syncthreads();
    // row j of X: divide by the diagonal of L
    const double djj = CHOL ? sqrt(d[j]) : 1.0;
    if (CHOL)
      for (int c = tid; c <= j; c += blockDim.x) X[c][j] /= djj;
    __syncthreads();
    // rows i > j: X[i, c] -= L[i][j] X[j, c], c <= j
    const int nr = w - j - 1;
    for (int e = tid; e < nr * (j + 1); e += blockDim.x) {
      const int i = j + 1 + e % nr, c = e / nr;
      const double lij = CHOL ? S[j][i] / sqrt(d[j]) : S[j][i] / d[j];
      X[c][i] -= lij * X[c][j];
    }
  }
  __syncthreads();
}

// Factor the diagonal block (p0, p0) of A (w <= 64) and write L11 back into
// A, its inverse into Inv (ld ldi), and for LDL^T the pivots into dvec.
template <bool CHOL>
__global__ __launch_bounds__(256) void k_diag_block(double* A, int lda, int p0, int w,
                                                    double* Inv, int ldi, double* dvec, int* info,
                                                    int row_base, const double* tolp) {
  __shared__ double S[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  __shared__ double d[NB];
  const int tid = threadIdx.x;
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int r = e % w, c = e / w;
    S[c][r] = (c <= r) ? A[(p0 + r) + (size_t)(p0 + c) * lda] : 0.0;
  }
  const double tol = CHOL ? 0.0 : *tolp;
  block_factor<CHOL>(S, d, w, info, row_base + p0, tol, true);
  block_inverse<CHOL>(S, d, X, w);
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int r = e % w, c = e / w;
    double l;
    if (CHOL)
      l = (r == c) ? sqrt(d[c]) : (r > c ? S[c][r] / sqrt(d[c]) : 0.0);
    else
      l = (r == c) ? 1.0 : (r > c ? S[c][r] / d[c] : 0.0);
    A[(p0 + r) + (size_t)(p0 + c) * lda] = l;
    Inv[r + (size_t)c * ldi] = (r >= c) ? X[c][r] : 0.0;
  }
  if (!CHOL)
    for (int j = tid; j < w; j += blockDim.x) dvec[p0 + j] = d[j];
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

hipError_t launch_diag_block(bool chol, double* A, int lda, int p0, int w, double* Inv, int ldi,
                             double* dvec, int* info, int row_base, const double* tolp,
                             hipStream_t s) {
  if (w <= 0 || w > NB) return hipErrorInvalidValue;
  if (chol)
    hipLaunchKernelGGL(k_diag_block<true>, dim3(1), dim3(256), 0, s, A, lda, p0, w, Inv, ldi, dvec,
                       info, row_base, tolp);
  else
    hipLaunchKernelGGL(k_diag_block<false>, dim3(1), dim3(256), 0, s, A, lda, p0, w, Inv, ldi,
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
