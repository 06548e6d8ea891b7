// Dense tile kernels: blocked Cholesky and unpivoted LDL^T of the diagonal
// tiles, and the diagonal-block step of the blocked triangular solve.
//
// The diagonal tile factorization is the "chol" (Algorithm "Left Looking TLR
// Cholesky") and "ldl" (Algorithm "Left Looking TLR LDL^T", unpivoted with
// scalar pivots) step of the paper; the triangular solve is "batchTrsm" with
// one shared triangle (all tiles of a column are solved against the same
// L_kk).  The kernels here do the latency-bound panel work in LDS; the
// trailing updates run on the MFMA batched GEMM.
#include "tlr_internal.h"

namespace tlr {

namespace {

constexpr int NBP_MAX = 64;
constexpr int PANEL_ROWS = 256;   // rows of the sub-diagonal panel per workgroup

// Unblocked Cholesky of the w x w block S (LDS, column-major with stride
// NBP_MAX + 1).  Records the 1-based global row of the first non-positive
// pivot in *info and keeps going with a unit pivot so no NaN spreads.
__device__ void chol_lds(double (*S)[NBP_MAX + 1], int w, int* info, int row_base, bool report) {
  const int tid = threadIdx.x;
  for (int j = 0; j < w; ++j) {
    __syncthreads();
    if (tid == 0) {
      double dj = S[j][j];
      if (!(dj > 0.0)) {
        if (report) atomicCAS(info, 0, row_base + j + 1);
        dj = 1.0;
      }
      S[j][j] = sqrt(dj);
    }
    __syncthreads();
    const double piv = S[j][j];
    for (int i = j + 1 + tid; i < w; i += blockDim.x) S[j][i] /= piv;   // S[col][row]
    __syncthreads();
    const int nt = w - j - 1;
    for (int e = tid; e < nt * nt; e += blockDim.x) {
      const int r = j + 1 + e % nt, c = j + 1 + e / nt;
      if (c <= r) S[c][r] -= S[j][r] * S[j][c];
    }
  }
  __syncthreads();
}

// S is stored transposed-by-column: S[c][r] = block(r, c).
__global__ __launch_bounds__(256) void k_potrf_panel(double* A, int lda, int m, int p0, int w,
                                                     int* info, int row_base) {
  __shared__ double S[NBP_MAX][NBP_MAX + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int r = e % w, c = e / w;
    S[c][r] = (c <= r) ? A[(p0 + r) + (size_t)(p0 + c) * lda] : 0.0;
  }
  chol_lds(S, w, info, row_base + p0, blockIdx.x == 0);
  if (blockIdx.x == 0) {
    for (int e = tid; e < w * w; e += blockDim.x) {
      const int r = e % w, c = e / w;
      A[(p0 + r) + (size_t)(p0 + c) * lda] = (c <= r) ? S[c][r] : 0.0;
    }
  }
  // rows below the diagonal block: x L11^T = a, forward substitution per row
  const int r = p0 + w + blockIdx.x * PANEL_ROWS + tid;
  if (r < m) {
    double x[NBP_MAX];
#pragma unroll
    for (int j = 0; j < NBP_MAX; ++j)
      if (j < w) x[j] = A[r + (size_t)(p0 + j) * lda];
#pragma unroll
    for (int j = 0; j < NBP_MAX; ++j) {
      if (j < w) {
        double v = x[j];
#pragma unroll
        for (int c = 0; c < NBP_MAX; ++c)
          if (c < j) v -= x[c] * S[c][j];
        x[j] = v / S[j][j];
      }
    }
#pragma unroll
    for (int j = 0; j < NBP_MAX; ++j)
      if (j < w) A[r + (size_t)(p0 + j) * lda] = x[j];
  }
}

// Unpivoted LDL^T of the block: unit lower in S, pivots in dd.
__device__ void ldlt_lds(double (*S)[NBP_MAX + 1], double* dd, int w, int* info, int row_base,
                         double tol, bool report) {
  const int tid = threadIdx.x;
  for (int j = 0; j < w; ++j) {
    __syncthreads();
    if (tid == 0) {
      double dj = S[j][j];
      if (!(fabs(dj) > tol)) {
        if (report) atomicCAS(info, 0, row_base + j + 1);
        dj = 1.0;
      }
      dd[j] = dj;
      S[j][j] = 1.0;
    }
    __syncthreads();
    const double piv = dd[j];
    const int nt = w - j - 1;
    // trailing update with the unscaled column, then scale it
    for (int e = tid; e < nt * nt; e += blockDim.x) {
      const int r = j + 1 + e % nt, c = j + 1 + e / nt;
      if (c <= r) S[c][r] -= S[j][r] * S[j][c] / piv;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < w; i += blockDim.x) S[j][i] /= piv;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_ldlt_panel(double* A, int lda, int m, int p0, int w,
                                                    double* d, double* W, int ldw, int* info,
                                                    int row_base, const double* tolp) {
  __shared__ double S[NBP_MAX][NBP_MAX + 1];
  __shared__ double dd[NBP_MAX];
  const int tid = threadIdx.x;
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int r = e % w, c = e / w;
    S[c][r] = (c <= r) ? A[(p0 + r) + (size_t)(p0 + c) * lda] : 0.0;
  }
  const double tol = *tolp;
  ldlt_lds(S, dd, w, info, row_base + p0, tol, blockIdx.x == 0);
  if (blockIdx.x == 0) {
    for (int e = tid; e < w * w; e += blockDim.x) {
      const int r = e % w, c = e / w;
      A[(p0 + r) + (size_t)(p0 + c) * lda] = (c <= r) ? S[c][r] : 0.0;
    }
    for (int j = tid; j < w; j += blockDim.x) d[p0 + j] = dd[j];
  }
  // rows below: y L11^T = a (unit), W = y (= L21 D), L21 = y D^{-1}
  const int r = p0 + w + blockIdx.x * PANEL_ROWS + tid;
  if (r < m) {
    double x[NBP_MAX];
#pragma unroll
    for (int j = 0; j < NBP_MAX; ++j)
      if (j < w) x[j] = A[r + (size_t)(p0 + j) * lda];
#pragma unroll
    for (int j = 0; j < NBP_MAX; ++j) {
      if (j < w) {
        double v = x[j];
#pragma unroll
        for (int c = 0; c < NBP_MAX; ++c)
          if (c < j) v -= x[c] * S[c][j];
        x[j] = v;
      }
    }
#pragma unroll
    for (int j = 0; j < NBP_MAX; ++j)
      if (j < w) {
        W[(r - p0 - w) + (size_t)j * ldw] = x[j];
        A[r + (size_t)(p0 + j) * lda] = x[j] / dd[j];
      }
  }
}

// X_p = L_pp^{-1} B_p or L_pp^{-T} B_p on rows [p0, p0 + w) of B, 64
// right-hand sides per workgroup, one thread per right-hand side.
__global__ __launch_bounds__(64) void k_trsm_diag(const double* L, int ldl, double* B, int ldb,
                                                  int p0, int w, int n, int unit, int trans) {
  __shared__ double S[NBP_MAX][NBP_MAX + 1];   // S[c][r] = L(p0 + r, p0 + c)
  __shared__ double X[64][NBP_MAX + 1];        // X[col][row]
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

hipError_t launch_potrf_panel(double* A, int lda, int m, int p0, int w, int* info, int row_base,
                              hipStream_t s) {
  if (w <= 0 || w > NBP_MAX) return hipErrorInvalidValue;
  const int below = m - p0 - w;
  const int grid = below > 0 ? (below + PANEL_ROWS - 1) / PANEL_ROWS : 1;
  hipLaunchKernelGGL(k_potrf_panel, dim3(grid), dim3(PANEL_ROWS), 0, s, A, lda, m, p0, w, info,
                     row_base);
  return hipGetLastError();
}

hipError_t launch_ldlt_panel(double* A, int lda, int m, int p0, int w, double* d, double* W,
                             int ldw, int* info, int row_base, const double* tolp, hipStream_t s) {
  if (w <= 0 || w > NBP_MAX) return hipErrorInvalidValue;
  const int below = m - p0 - w;
  const int grid = below > 0 ? (below + PANEL_ROWS - 1) / PANEL_ROWS : 1;
  hipLaunchKernelGGL(k_ldlt_panel, dim3(grid), dim3(PANEL_ROWS), 0, s, A, lda, m, p0, w, d, W,
                     ldw, info, row_base, tolp);
  return hipGetLastError();
}

hipError_t launch_trsm_diag(const double* L, int ldl, double* B, int ldb, int p0, int w, int n,
                            bool unit, bool trans, hipStream_t s) {
  if (w <= 0 || w > NBP_MAX || n <= 0) return w > NBP_MAX ? hipErrorInvalidValue : hipSuccess;
  hipLaunchKernelGGL(k_trsm_diag, dim3((n + 63) / 64), dim3(64), 0, s, L, ldl, B, ldb, p0, w, n,
                     unit ? 1 : 0, trans ? 1 : 0);
  return hipGetLastError();
}

}  // namespace tlr
