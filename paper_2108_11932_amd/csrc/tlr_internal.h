// Internal declarations shared by the host driver and the HIP kernels of the
// TLR library.  Everything is column-major FP64 unless stated otherwise.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace tlr {

// ---------------------------------------------------------------------------
// Variable-size batched GEMM:  C = alpha * op(A) * op(B) + beta * C.
// op(A) is M x K, op(B) is K x N, C is M x N.  A zero-sized problem (M, N or
// K == 0 with beta handling) is allowed; K == 0 only scales C by beta.
// ---------------------------------------------------------------------------
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  int M, N, K;
  int lda, ldb, ldc;
  double alpha, beta;
};

// One entry per launched workgroup: x = descriptor index, y = output tile
// index inside that descriptor (row tiles vary fastest).
struct BlockMap {
  int desc;
  int tile;
};

// Host-side staging of a batched GEMM; builds the block map and launches.
// trans_a / trans_b are uniform over the batch.
int gemm_tile_n(int N);                     // BN chosen for a problem (16 or 64)
hipError_t launch_gemm_batched(const GemmDesc* d_descs, const BlockMap* d_map, int nblocks,
                               bool trans_a, bool trans_b, int bn, hipStream_t s);

// ---------------------------------------------------------------------------
// Dense tile kernels (one m x m tile, m <= 4096)
// ---------------------------------------------------------------------------
// Panel step of the blocked right-looking Cholesky: factor the nbp x nbp
// diagonal block at (p, p) and solve the rows below it.  info (device int)
// receives the 1-based row of the first non-positive pivot (0 = none).
hipError_t launch_potrf_panel(double* A, int lda, int m, int p, int nbp, int* info, int row_base,
                              hipStream_t s);
// Same for the unpivoted LDL^T: the unit lower factor overwrites A, the
// pivots go to d, and W receives L21 * D (needed by the trailing update).
hipError_t launch_ldlt_panel(double* A, int lda, int m, int p, int nbp, double* d, double* W,
                             int ldw, int* info, int row_base, const double* tolp, hipStream_t s);
// Diagonal-block step of the blocked triangular solve: X_p = L_pp^{-1} B_p
// (or L_pp^{-T}), for all n columns of B.
hipError_t launch_trsm_diag(const double* L, int ldl, double* B, int ldb, int p, int nbp, int n,
                            bool unit, bool trans, hipStream_t s);

// ---------------------------------------------------------------------------
// ARA kernels
// ---------------------------------------------------------------------------
// Gaussian test matrix from Philox4x32-10 + Box-Muller.  Element e of the
// rows x cols column-major matrix uses Gaussian (e & 1) of counter
// (e >> 1, t, k, stream) under key (seed lo, seed hi).
hipError_t launch_randn(double* out, int rows, int cols, int ld, unsigned long long seed, unsigned k,
                        unsigned t, unsigned stream, hipStream_t s);
hipError_t launch_philox_raw(unsigned* out, int n, unsigned long long seed, unsigned c1, unsigned c2,
                             unsigned c3, hipStream_t s);

// Per-tile descriptor for the orthogonalisation of one ARA block.
struct OrthDesc {
  const double* Y; // m x bs sample block (ld m)
  double* Q;       // m x (qcap + bs) basis (ld m); new columns start at qold
  int qold;        // basis width before this iteration
  int* q;          // device basis width (updated by the pivoted Cholesky)
  int* flag;       // set to 1 when the tile has converged
  double* part;    // partial Gram sums: nrb x bs x bs x 2 (hi, lo)
  double* rfac;    // bs x bs inverse triangular factor
  int* piv;        // bs pivots, then the accepted count at [bs]
};
// pass 1: Gram of the bs sample columns; pass 2: of the p new basis columns.
hipError_t launch_gram_dd(const OrthDesc* d, int ntiles, int m, int bs, int pass, hipStream_t s);
hipError_t launch_pivchol(const OrthDesc* d, int ntiles, int m, int bs, double tau2, int r_min,
                          int qcap, hipStream_t s);
hipError_t launch_chol_small(const OrthDesc* d, int ntiles, int m, int bs, hipStream_t s);
hipError_t launch_apply_rinv(const OrthDesc* d, int ntiles, int m, int bs, int pass,
                             hipStream_t s);

// Dynamic batching: stable compaction of the active list by the convergence
// flags (flag[slot] != 0 removes the slot), then refill from the waiting
// list.  counts[0] = active count in/out, counts[1] = waiting cursor.
hipError_t launch_compact(int* act, int* counts, const int* flag, const int* waiting, int nwaiting,
                          int s_max, hipStream_t s);
// Rank sort of a column: order rows by rank descending, ties ascending row.
hipError_t launch_sort_ranks(const int* ranks, const int* rows, int n, int* order, hipStream_t s);

// ---------------------------------------------------------------------------
// Misc kernels
// ---------------------------------------------------------------------------
struct CopyDesc {
  const double* src;
  double* dst;
  int rows, cols, lds, ldd;
};
hipError_t launch_copy_batched(const CopyDesc* d, int n, int max_cols, hipStream_t s);
// dst = src (m x m) + shift on the first nreal diagonal entries.
hipError_t launch_copy_shift(const double* src, double* dst, int m, int nreal, double shift,
                             hipStream_t s);
// out(r, c) = d[r] * in(r, c) (row scaling) or in(r, c) / d[r].
hipError_t launch_scale_rows(const double* in, int ldi, double* out, int ldo, const double* d,
                             int rows, int cols, bool inverse, hipStream_t s);
// Covariance tiles from points.  Tile t covers rows [r0, r0 + m) and
// columns [c0, c0 + m) of the padded matrix; entries outside [0, n) are the
// identity padding.
// kernel < 0 copies the tile from a dense lower-stored matrix `src` (ld lds)
// instead of evaluating a covariance kernel on the points.
struct GenDesc {
  double* out;
  int ld;
  long long r0, c0;
};
hipError_t launch_gen_tiles(const GenDesc* d, int ntiles, const double* pts, int dim, long long n,
                            int m, int kernel, double ell, double diag_add, const double* src,
                            long long lds, hipStream_t s);

}  // namespace tlr
