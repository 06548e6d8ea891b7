/* tlr_kernels.h -- the batched building blocks of the TLR library, exposed one
 * by one so that each can be checked against a reference on its own.
 *
 * All pointers marked (device) are HIP device memory, all others host memory.
 * Matrices are column-major FP64.  Every call enqueues on `stream` and
 * synchronises it before returning.  Status codes and tlr_last_error() are
 * those of tlr.h.
 */
#ifndef TLR_KERNELS_H
#define TLR_KERNELS_H

#include "tlr.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One problem of the variable-size batched GEMM that runs every small
 * contraction of the factorization (the sampling products of Eq. (2), their
 * transposes in the projection, the dense updates):
 * C = alpha op(A) op(B) + beta C with op(A) M x K, op(B) K x N. */
typedef struct {
  int M, N, K;
  const double* A; int lda;   /* (device) */
  const double* B; int ldb;   /* (device) */
  double* C; int ldc;         /* (device) */
  double alpha, beta;
} tlrk_gemm_problem;

/* A batch of count problems sharing the transpositions (0 = N, 1 = T). */
tlr_status tlrk_gemm_batched(int trans_a, int trans_b, int count, const tlrk_gemm_problem* problems,
                             void* stream);

/* Dense Cholesky of an m x m tile (device, lower triangle used, upper zeroed
 * on return): the "chol" step of the diagonal tiles.  *info receives the
 * 1-based row of the first non-positive pivot, 0 on success. */
tlr_status tlrk_potrf(int m, double* A, int lda, int* info, void* stream);

/* Unpivoted scalar LDL^T of an m x m tile (device): unit lower L overwrites
 * the lower triangle, d (device, m) the pivots (the "ldl" step of the LDL^T
 * variant, Section 5.3).  *info = 1-based row of a pivot with
 * |d| <= 64 u ||A||_F, else 0. */
tlr_status tlrk_ldlt(int m, double* A, int lda, double* d, int* info, void* stream);

/* B <- L^{-1} B or L^{-T} B, L m x m lower triangular (device), B m x n
 * (device); unit selects a unit diagonal ("batchTrsm" with one shared
 * triangle). */
tlr_status tlrk_trsm(int m, int n, const double* L, int ldl, double* B, int ldb, int unit,
                     int trans, void* stream);

/* Raw Philox4x32-10 words: out (device, 4 n words) holds the outputs for the
 * counters (c, c1, c2, c3), c = 0..n-1, under the key (seed lo, seed hi). */
tlr_status tlrk_philox(int n, unsigned long long seed, unsigned c1, unsigned c2, unsigned c3,
                       unsigned* out, void* stream);

/* The Gaussian test matrix of ARA iteration t of column k ("batchRandn"):
 * element e of the rows x cols column-major matrix is Box-Muller Gaussian
 * (e & 1) of the Philox counter (e >> 1, t, k, s). */
tlr_status tlrk_randn(int rows, int cols, unsigned long long seed, unsigned k, unsigned t,
                      unsigned s, double* out, void* stream);

/* The test matrices of nt consecutive ARA iterations t0 .. t0 + nt - 1 of
 * column k in one launch, as the factorization draws them: matrix t - t0 at
 * out (device) + (t - t0) rows cols_max, rows x cols0 for iteration 0 and
 * rows x cols1 after (cols_max = max(cols0, cols1), leading dimension rows),
 * element for element the matrix tlrk_randn gives for (k, t, s). */
tlr_status tlrk_randn_iters(int rows, int cols0, int cols1, unsigned long long seed, unsigned k,
                            unsigned t0, int nt, unsigned s, double* out, void* stream);

/* Batched adaptive randomized approximation of count explicit m x m tiles
 * (device, tile b at tiles + b m^2), Algorithm "Adaptive Randomized
 * Approximation": on return Q (device, count x m x m) holds orthonormal
 * bases and B (device, count x m x m) the projections B = A^T Q, so
 * A_b ~ Q_b B_b^T with ranks[b] columns; iters[b] = ARA iterations.  bs is
 * one of 1, 2, 4, 8, 16, 24, 32. */
tlr_status tlrk_ara(int m, int count, const double* tiles, double tau, int bs, int r_min,
                    unsigned long long seed, double* Q, double* B, int* ranks, int* iters,
                    void* stream);

/* "sortRanks" (Section 4.2): order (host, n) lists rows (host, n) by ranks
 * (host, n), descending, ties by ascending row.  The factorization takes its
 * order of every column's tiles from this same host routine (the input
 * ranks are known on the host, so the device queue is not drained for it). */
tlr_status tlrk_sort_ranks(int n, const int* ranks, const int* rows, int* order);

/* One "getConvergedTiles"/"updateSubset" step on the device: the active list
 * act (host, in/out, *count entries) loses the slots whose flag (host,
 * indexed by slot, nslots entries) is set, keeping order, and is refilled
 * from waiting (host, nwaiting entries) starting at *cursor, up to s_max
 * entries.  *count and *cursor are updated. */
tlr_status tlrk_compact(int nslots, int* act, int* count, const int* flags, const int* waiting,
                        int nwaiting, int* cursor, int s_max);

#ifdef __cplusplus
}
#endif

#endif /* TLR_KERNELS_H */
