/* tlr.h -- tile low rank (TLR) Cholesky and LDL^T on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library.  It implements the left-looking TLR factorizations of
 * Boukaram, Zampini, Turkiyyah and Keyes, "H2OPUS-TLR: High Performance Tile
 * Low Rank Symmetric Factorizations using Adaptive Randomized Approximation"
 * (arXiv:2108.11932):
 *
 *   tlr_potrf  -- Algorithm "Left Looking TLR Cholesky" (Section 4.3)
 *   tlr_ldlt   -- Algorithm "Left Looking TLR LDL^T" (Section 5.3)
 *   tlr_solve  -- Algorithm "TLR Triangular Solve" (Section 4.4), forward and
 *                 transposed sweeps
 *   tlr_matvec -- the TLR matrix-vector product (Section 4.4)
 *   tlr_compress, tlr_compress_kernel -- the TLR representation of Section 1
 *                 (dense diagonal tiles, off-diagonal tiles U V^T with adaptive
 *                 ranks), built by adaptive randomized approximation (Section 3.1)
 *
 * Matrix format (Section 1, Figure 1).  An N x N symmetric matrix is cut into
 * nb = ceil(N / m) block rows and columns of size m.  When m does not divide N
 * the last block row and column are padded to m (Section 6): the padded part
 * of the last diagonal tile is the identity and the padded rows of U and V are
 * zero; solves and products ignore the padding.  Diagonal tiles are dense
 * m x m.  Strictly lower tiles (i > j) are U_ij V_ij^T with U_ij, V_ij of size
 * m x r_ij, r_ij >= 0; the upper tiles are implied by symmetry.  All matrices
 * are column-major FP64.
 *
 * Threshold.  The compression threshold eps is an absolute per-tile 2-norm
 * threshold (TLR_EPS_ABS, as in the paper's experiments: every compressed tile
 * satisfies ||S - Q Q^T S||_2 <= tau with tau = eps, with high probability), or
 * relative (TLR_EPS_REL: tau = eps * ||A||_2, the norm estimated by power
 * iteration on the TLR input).
 *
 * Memory.  A handle owns all of its device memory.  It is allocated through
 * the optional allocator callbacks (so a host framework can supply its caching
 * allocator), else with hipMalloc.  Inputs are copied, never retained.  The
 * factorization keeps the input tiles and writes the factor into separate
 * storage of the same handle, so a handle can be refactored (for example with
 * another threshold or shift) and the input stays available to products.
 *
 * Streams.  Every call enqueues its work on `stream` (a hipStream_t; NULL is
 * the default stream) and returns after a final synchronisation of that
 * stream, so results and status are valid on return.
 *
 * Errors.  Negative codes are caller or system errors, positive codes are
 * numerical breakdowns.  tlr_last_error() returns a thread-local message for
 * the last failing call.  On TLR_ERR_ARG nothing is modified.  On a
 * breakdown, stats->info holds the 1-based global row of the failing pivot
 * (LAPACK convention) and the factor is marked invalid.
 */
#ifndef TLR_H
#define TLR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tlr_matrix_s* tlr_matrix_t;

typedef enum {
  TLR_OK = 0,
  TLR_ERR_ARG = -1,        /* invalid argument */
  TLR_ERR_OOM = -2,        /* device or pinned host allocation failed */
  TLR_ERR_DEVICE = -3,     /* HIP runtime error */
  TLR_ERR_STATE = -4,      /* handle not in the state the call needs */
  TLR_ERR_NOT_SPD = 1,     /* a diagonal tile lost definiteness (Section 5.1) */
  TLR_ERR_ZERO_PIVOT = 2   /* unpivoted LDL^T met a zero pivot */
} tlr_status;

enum { TLR_EPS_ABS = 0, TLR_EPS_REL = 1 };
/* Precision of the Schur-complement sampling of Eq. (2).  TLR_FP64: all in
 * FP64.  The mixed forms keep packed low-precision copies of the factor's
 * block-row U panels and form a tile's panel term U_i* Z_i on the FP32
 * (TLR_MIXED_FP32) or BF16 matrix cores with FP32 accumulation, Z_i rounded
 * to the same precision, whenever that rounding stays below the threshold:
 *   (2 u_p + sqrt(R_i) u_32) nu_ik <= tau / 16,
 *   nu_ik = ||A_ik||_F + sum_j ||L_ij||_F ||L_kj||_F,
 * u_p the unit roundoff of the copy (2^-24 FP32, 2^-8 BF16) and R_i the
 * panel width; the other tiles sample in FP64.  TLR_MIXED_BF16 tries BF16
 * first, then FP32.  TLR_MIXED_AUTO is TLR_MIXED_BF16 when tau >= 1e-3
 * ||A||_2 (the norm estimated by power iteration on the input) and
 * TLR_MIXED_FP32 otherwise.  In every form the input-tile term of the
 * sampling, the dense diagonal work, the orthogonalisation (FP64 and
 * double-double Cholesky QR, two Gram-Schmidt passes), the final projection
 * and the triangular solve stay FP64; the LDL^T variant samples in FP64. */
enum { TLR_FP64 = 0, TLR_MIXED_FP32 = 1, TLR_MIXED_BF16 = 2, TLR_MIXED_AUTO = 3 };
enum { TLR_KERNEL_EXP = 0, TLR_KERNEL_MATERN15 = 1 };
enum { TLR_INPUT = 0, TLR_FACTOR = 1 };

/* Device memory callbacks.  alloc returns NULL on failure; free receives
 * pointers returned by alloc.  `stream` is the stream the memory is used on. */
typedef struct {
  void* ctx;
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* p, void* stream);
} tlr_allocator;

/* Options of compression and factorization. */
typedef struct {
  int bs;                  /* ARA block size: samples per iteration, one of
                              1, 2, 4, 8, 16, 24, 32; the paper uses 16 in 2D
                              and 32 in 3D (Section 6) */
  int eps_mode;            /* TLR_EPS_ABS (default) or TLR_EPS_REL */
  int precision;           /* TLR_FP64 (default), TLR_MIXED_FP32, TLR_MIXED_BF16
                              or TLR_MIXED_AUTO */
  double shift;            /* factor A + shift * I (diagonal shift, Section 5.1);
                              a negative value means shift = tau */
  int max_active;          /* size of the active subset of tiles per column
                              (Algorithm "Left Looking Cholesky TLR ARA Update",
                              "subset"); <= 0 means all tiles of the column */
  int r_min;               /* a tile has converged once at least r_min samples of
                              a block stay below tau after orthogonalisation
                              (1..bs; 0 means the default, half the smallest
                              block: the samples left over by the pivoted
                              Cholesky QR are the smallest of their block, so
                              a single one underestimates the error) */
  unsigned long long seed; /* seed of the Philox4x32-10 test-matrix stream */
  int flags;               /* TLR_FLAG_* bits */
  int bs_tail;             /* samples per ARA iteration after the first one of a
                              column (0: bs); one of the bs values.  A larger
                              value finishes the few high-rank tiles that keep
                              a column's ARA going in fewer iterations */
  int tail_active;         /* > 0: bs_tail is used only by the iterations that
                              start with at most this many tiles of the column
                              still active (as known to the host two iterations
                              earlier); the others draw bs.  0: every iteration
                              after the first draws bs_tail */
  int auto_shift;          /* nonzero: when a diagonal tile loses definiteness
                              (TLR_ERR_NOT_SPD) and the shift in use is 0, factor
                              once more with the diagonal shift s = tau, the
                              perturbation below the compression threshold of
                              Section 5.1; stats->shift reports the shift used */
  int sample_strip;        /* rows of a tile that one workgroup of the
                              Schur-complement sampling product computes: 0
                              chooses 64 when enough tiles are active to fill
                              the GPU and 16 otherwise; 16 or 64 forces one.
                              Both give the same samples bit for bit */
  double conv_factor;      /* the ARA accepts new directions and tests
                              convergence at tau / conv_factor (>= 1; 0 means
                              the default).  The convergence test reads the
                              leftover samples of a block, which the pivoted
                              selection leaves biased towards small norms;
                              the factor makes the compression error of a
                              tile stay below tau with high probability */
} tlr_opts;

/* opts.flags.  TLR_FLAG_KERNEL_TIMING: record HIP events around every launch
 * of the Schur-complement sampling product and report its time and
 * algorithmic bytes in tlr_stats.sample_*.  TLR_FLAG_PHASE_TIMING: record
 * HIP events at the phase boundaries of every column and report the GPU time
 * per phase in tlr_stats.t_phase.  TLR_FLAG_SERIAL_SAMPLING: draw every ARA
 * iteration's samples in launches of their own after the previous iteration
 * (by default, when every tile of the column is active from the start and
 * the block size is 16 or 32, the samples of iteration t + 1 are drawn in
 * the launches of iteration t's second Gram-Schmidt pass; the result is the
 * same bit for bit).
 * TLR_FLAG_MODIFIED_CHOL (Cholesky only; Section 5.1.2, "Modified Cholesky"):
 * a diagonal tile that loses definiteness is not an error; each
 * non-positive pivot d of its Cholesky is replaced by max(|d|, tau) as it is
 * met, which factors the tile plus a non-negative diagonal perturbation
 * (E = 0 for a definite tile); tlr_stats.modified_pivots counts them.
 * TLR_FLAG_DIAG_GRAPH: the handle captures the launch sequence of a diagonal
 * tile's factorization once as a HIP graph on buffers of its own and
 * replays it for every column (one graph launch per column on the
 * diagonal-tile stream, then one copy of the results to their places)
 * instead of launching it kernel by kernel; the result is the same bit for
 * bit.  Off by default: that stream is not on the critical path, and the
 * replay measured 1.6 % slower on the 2D covariance workload (N = 131072,
 * tile 1024).
 * TLR_FLAG_SCHUR_COMP (unpivoted Cholesky; Section
 * 5.1.1, "Schur Compensation"): the accumulated update D_k of each diagonal
 * tile is compressed to tau by its truncated eigen-decomposition (the
 * eigenvalues above tau kept), and the absolute row sums of the dropped
 * part D_k - Dbar_k (positive semidefinite, 2-norm <= tau) are added to the
 * diagonal: the tile factored is A_kk - D_k + diag(rowsum |D_k - Dbar_k|).
 * The dropped part is formed as D_k P with P = (I - sign(D_k - tau I)) / 2,
 * the sign function by 30 steps of an odd quintic and 12 Newton-Schulz
 * steps (114 m x m x m products, on the matrix cores) per column on the
 * diagonal-tile stream.  Rejected with TLR_ERR_ARG by tlr_ldlt, tlr_potrf_pivoted and the
 * batched factorizations. */
enum { TLR_FLAG_KERNEL_TIMING = 1, TLR_FLAG_PHASE_TIMING = 2, TLR_FLAG_SERIAL_SAMPLING = 4,
       TLR_FLAG_MODIFIED_CHOL = 8, TLR_FLAG_DIAG_GRAPH = 16, TLR_FLAG_SCHUR_COMP = 32 };

/* Phases of a column step (indices of tlr_stats.t_phase).  Phases 0-6 run on
 * the caller's stream one after another, so their times add up to that
 * stream's span of the factorization; phase 7 runs on a second stream,
 * overlapped with them.
 *   TLR_PHASE_GBLOCKS  the products G_ij = V_ij^T V_kj of the newest column
 *   TLR_PHASE_SAMPLE   test matrices and the Schur-complement sampling of
 *                      Eq. (2): batchRandn, sampleLeft
 *   TLR_PHASE_ORTH     block Gram-Schmidt and Cholesky QR: batchOrthog
 *   TLR_PHASE_BATCH    getConvergedTiles, updateSubset (dynamic batching)
 *   TLR_PHASE_PROJECT  the projection B = S^T Q: sampleLeftT
 *   TLR_PHASE_TRSM     batchTrsm (and batchIDMult), including the wait for
 *                      the diagonal tile
 *   TLR_PHASE_APPEND   updateTiles: the new tiles appended to the row panels
 *   TLR_PHASE_DIAG     second stream: updateDense, chol / ldl of the diagonal
 *                      tile and its inverse, and the G_ij of the next column */
enum {
  TLR_PHASE_GBLOCKS = 0, TLR_PHASE_SAMPLE = 1, TLR_PHASE_ORTH = 2, TLR_PHASE_BATCH = 3,
  TLR_PHASE_PROJECT = 4, TLR_PHASE_TRSM = 5, TLR_PHASE_APPEND = 6, TLR_PHASE_DIAG = 7,
  TLR_NPHASE = 8
};

/* Results of a factorization. */
typedef struct {
  int info;                /* 1-based global row of a failed pivot, 0 = success */
  double tau;              /* absolute per-tile threshold used */
  double norm_a;           /* ||A||_2 estimate (TLR_EPS_REL only, else 0) */
  double flops;            /* floating point operations executed on the GPU */
  double flops_paper;      /* operation count of the paper's formulation */
  double bytes_alg;        /* algorithmic HBM bytes of the sampling kernels */
  long long ara_iters;     /* sum over columns of ARA iterations (launch batches) */
  long long tile_iters;    /* sum over tiles of ARA iterations */
  long long full_rank_tiles; /* tiles whose rank reached m */
  int max_rank;            /* largest rank of the factor */
  double mean_rank;        /* mean rank of the strictly lower tiles of the factor */
  double factor_bytes;     /* device bytes held by the factor */
  long long sample_launches; /* TLR_FLAG_KERNEL_TIMING: launches of the sampling product */
  double sample_ms;        /* their summed duration (HIP events), milliseconds */
  double sample_bytes;     /* their algorithmic HBM bytes: U panels, Z, Y read and write */
  double sample_flops;     /* their flops */
  long long fp32_tile_iters; /* mixed forms: tile iterations sampled from FP32 panels */
  double shift;            /* diagonal shift the factor was computed with */
  int shift_retries;       /* factorizations repeated by opts.auto_shift (0 or 1) */
  double t_total;          /* host wall time of the call, milliseconds */
  double t_phase[TLR_NPHASE]; /* TLR_FLAG_PHASE_TIMING: GPU time per phase (TLR_PHASE_*),
                              milliseconds */
  long long bf16_tile_iters; /* mixed forms: tile iterations sampled from BF16 panels */
  double t_host_issue;     /* host time issuing the ARA iterations' launches, ms */
  double t_host_wait;      /* host time waiting for the ARA iterations' results, ms */
  long long modified_pivots; /* TLR_FLAG_MODIFIED_CHOL: pivots raised to tau */
} tlr_stats;

/* Fill *opts with the defaults: bs 16, absolute eps, FP64, shift 0, all tiles
 * active, r_min 0 (half the block), seed 0x5eed, no automatic shift,
 * automatic strip height. */
void tlr_opts_default(tlr_opts* opts);

/* Create an N x N matrix with tile size m and the given ranks of the strictly
 * lower tiles (ranks[i * nb + j] for i > j, other entries ignored; host
 * memory; NULL means all zero).  Diagonal tiles start as the identity, factors
 * as zero; fill them with tlr_set_diag / tlr_set_tile.  allocator may be NULL.
 * Errors: TLR_ERR_ARG for N <= 0, m <= 0, m > N rounded up, a negative rank or
 * a rank above m; TLR_ERR_OOM. */
tlr_status tlr_create(long long N, int m, const int* ranks, const tlr_allocator* allocator,
                      void* stream, tlr_matrix_t* out);

/* Copy the m x m diagonal tile k (leading dimension ld) from host
 * (on_device = 0) or device memory.  For the last, padded tile only the real
 * rows and columns are read. */
tlr_status tlr_set_diag(tlr_matrix_t A, int k, const double* D, int ld, int on_device);

/* Copy U_ij and V_ij (m x r_ij each, leading dimension ld >= m) of the strictly
 * lower tile (i, j), i > j.  Padded rows are set to zero. */
tlr_status tlr_set_tile(tlr_matrix_t A, int i, int j, const double* U, const double* V, int ld,
                        int on_device);

/* Build the TLR form of the dense symmetric N x N matrix A (device memory,
 * leading dimension lda >= N; only the lower triangle is read) with tile size
 * m: diagonal tiles are copied and every strictly lower tile is compressed by
 * adaptive randomized approximation at threshold eps (opts->eps_mode is
 * ignored: eps is absolute).  opts may be NULL. */
tlr_status tlr_compress(const double* A, long long lda, long long N, int m, double eps,
                        const tlr_opts* opts, const tlr_allocator* allocator, void* stream,
                        tlr_matrix_t* out);

/* Build the TLR form of the covariance matrix K(x_a, x_b) + diag_add * I of N
 * points (device memory, row-major N x dim, dim 1..3) without forming it:
 * tiles are generated on the device and compressed as in tlr_compress.
 * kernel: TLR_KERNEL_EXP, exp(-r / ell), or TLR_KERNEL_MATERN15,
 * (1 + sqrt(3) r / ell) exp(-sqrt(3) r / ell); r is the Euclidean distance. */
tlr_status tlr_compress_kernel(const double* points, int dim, long long N, int kernel, double ell,
                               double diag_add, int m, double eps, const tlr_opts* opts,
                               const tlr_allocator* allocator, void* stream, tlr_matrix_t* out);

/* Left-looking TLR Cholesky A + shift I = L L^T (Algorithm "Left Looking TLR
 * Cholesky").  Column k: dense update of the diagonal tile with the low rank
 * products of row k, dense Cholesky, batched ARA of the Schur-complement
 * tiles of column k sampled through Eq. (1)-(2) with dynamic batching, batched
 * triangular solve with L_kk.  Every off-diagonal tile of L is compressed
 * once, at threshold tau.  stats may be NULL.  Returns TLR_ERR_NOT_SPD when a
 * diagonal tile is not positive definite after its update (with
 * opts->auto_shift: when it still is with the shift s = tau). */
tlr_status tlr_potrf(tlr_matrix_t A, double eps, const tlr_opts* opts, tlr_stats* stats,
                     void* stream);

/* Tile-size autotuner (the factorization time depends strongly on the tile
 * size, Table 1 of the paper).  For the covariance problem of
 * tlr_compress_kernel (points in device memory), builds the TLR input at
 * each of the ncand candidate tile sizes at threshold eps and times one
 * tlr_potrf with opts after an untimed one; *best receives the fastest
 * candidate, ms (host, ncand entries, may be NULL) the times in
 * milliseconds (INFINITY for a candidate that failed to factor).  The choice
 * is remembered per problem class (ceil(log2 N), dim, kernel, eps,
 * opts->eps_mode, opts->precision, opts->bs and the candidate set): a class
 * seen before returns at once with *cached = 1 (cached may be NULL) and ms
 * untouched.  Device memory comes from the allocator (NULL: hipMalloc) and
 * is released before returning.  TLR_ERR_NOT_SPD if no candidate could be
 * factored. */
tlr_status tlr_tune_tile(const double* points, int dim, long long N, int kernel, double ell,
                         double diag_add, double eps, const tlr_opts* opts, const int* candidates,
                         int ncand, const tlr_allocator* allocator, void* stream, int* best,
                         double* ms, int* cached);
/* Forget every choice tlr_tune_tile remembered. */
void tlr_tune_reset(void);

/* Pivoted left-looking TLR Cholesky (Algorithm "Pivoted Left Looking TLR
 * Cholesky", Section 5.2): at column k every block position t >= k not yet
 * factored holds its updated diagonal tile A_tt - sum_{j<k} L_tj L_tj^T; the
 * one with the largest Frobenius norm (the first of equal ones) becomes
 * position k, its block row and column trading places with block k.  On
 * return the handle holds L with P A P^T = L L^T, where position t of the
 * factor is original block perm[t] (perm: host array of nb ints, may be
 * NULL; tlr_get_perm returns it later).  tlr_get_tile / tlr_get_diag of the
 * factor use positions; tlr_solve applies P and P^T itself.  The sampling
 * runs in FP64 (opts->precision TLR_FP64, else TLR_ERR_ARG); other options,
 * errors and stats as tlr_potrf (stats->info is the global row of the
 * position that failed). */
tlr_status tlr_potrf_pivoted(tlr_matrix_t A, double eps, const tlr_opts* opts, int* perm,
                             tlr_stats* stats, void* stream);
/* The block permutation of the factor (identity for an unpivoted one):
 * perm (host, nb ints), position t = original block perm[t].
 * TLR_ERR_STATE if the handle holds no factor. */
tlr_status tlr_get_perm(tlr_matrix_t A, int* perm);

/* Left-looking TLR LDL^T A = L D L^T, L unit lower triangular, D diagonal
 * (Algorithm "Left Looking TLR LDL^T", Eq. (3)); the diagonal tiles use an
 * unpivoted LDL^T with scalar pivots.  D (device, N entries, may be NULL)
 * receives the pivots.  Returns TLR_ERR_ZERO_PIVOT when a pivot satisfies
 * |d| <= 64 u ||A_kk||_F. */
tlr_status tlr_ldlt(tlr_matrix_t A, double eps, const tlr_opts* opts, double* D, tlr_stats* stats,
                    void* stream);

/* Batched form of tlr_potrf (ldl = 0) and tlr_ldlt (ldl != 0) over count
 * independent matrices (dynamic batching across problems, Section 4.2; the
 * batching of many factorizations the conclusions, Section 7, propose).
 * Matrices of one tile size step through their block columns together: at
 * step k every matrix with more than k block columns does its column k, and
 * the ARA of all their Schur-complement tiles is one pooled set of launches
 * over the union of the active tiles, ordered by input rank (sortRanks over
 * the union); matrices of different tile sizes form separate groups.  Each
 * tile keeps its own matrix's threshold (eps, or eps ||A|| in relative
 * mode).  Every matrix is set to `stream`; each keeps its own diagonal-tile
 * stream.  A: count distinct handles.  D: NULL, or count device pointers
 * (N_i doubles each, NULL entries allowed) that receive the LDL^T pivots.
 * stats: NULL or count entries; stats[i].info is the failing row of matrix
 * i.  Returns TLR_OK, or the first failure (TLR_ERR_NOT_SPD /
 * TLR_ERR_ZERO_PIVOT leave the other matrices' factors usable). */
tlr_status tlr_factor_batched(int count, tlr_matrix_t* A, int ldl, double eps,
                              const tlr_opts* opts, double* const* D, tlr_stats* stats,
                              void* stream);

/* tlr_factor_batched with one threshold per matrix: eps (host, count
 * entries, each > 0) is matrix i's eps, absolute or relative to its own
 * ||A_i|| as opts->eps_mode says.  tlr_potrf_batched is the Cholesky form,
 * tlr_ldlt_batched the LDL^T form (D as in tlr_factor_batched).
 * opts->auto_shift is not supported in the batched forms (TLR_ERR_ARG). */
tlr_status tlr_potrf_batched(int count, tlr_matrix_t* A, const double* eps, const tlr_opts* opts,
                             tlr_stats* stats, void* stream);
tlr_status tlr_ldlt_batched(int count, tlr_matrix_t* A, const double* eps, const tlr_opts* opts,
                            double* const* D, tlr_stats* stats, void* stream);

/* B <- (L L^T)^{-1} B or (L D L^T)^{-1} B with the factor held by the handle
 * (Algorithm "TLR Triangular Solve" and its transpose).  B is N x nrhs,
 * device memory, leading dimension ldb >= N.  TLR_ERR_STATE if the handle
 * holds no factor. */
tlr_status tlr_solve(tlr_matrix_t A, int nrhs, double* B, long long ldb, void* stream);

/* tlr_solve without any allocation, for callers that cannot allocate device
 * or host memory during the call (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, result and
 * errors as tlr_solve; the workspace, (nb m + m + T) nrhs doubles with T the
 * largest number of factor columns of one block column or block row (plus
 * nb m nrhs for a pivoted factor), lives
 * in a fixed device array of tlr_solve_noalloc_max_bytes() bytes (32 MiB)
 * that each GPU keeps until the process ends.  A larger need, or launch
 * descriptors that do not fit the handle's staging ring, is TLR_ERR_ARG.
 * All calls on one GPU share that array: calls that overlap on one GPU (two
 * streams, two threads) race and must be serialised by the caller. */
tlr_status tlr_solve_noalloc(tlr_matrix_t A, int nrhs, double* B, long long ldb, void* stream);
size_t tlr_solve_noalloc_max_bytes(void);

/* Preconditioned conjugate gradients for A x = b, the use of the
 * factorization as a preconditioner in Section 6: A is applied by
 * tlr_matvec of the input matrix of handle A, the preconditioner by
 * tlr_solve of the factor held by handle F (typically a looser threshold;
 * NULL: no preconditioner).  b and x are N-vectors in device memory; x holds
 * the initial guess on entry and the solution on return.  Stops when
 * ||b - A x||_2 <= rtol ||b||_2 or after maxit iterations; *iters receives
 * the iterations taken and *relres the final relative residual (the
 * recurrence's).  The two inner products of an iteration are reduced in a
 * fixed order and read back to the host.  TLR_ERR_NOT_SPD if a search
 * direction has p^T A p <= 0; TLR_ERR_STATE if F holds no factor. */
tlr_status tlr_pcg(tlr_matrix_t A, tlr_matrix_t F, const double* b, double* x, double rtol,
                   int maxit, int* iters, double* relres, void* stream);

/* SVD post-recompression (Section 6.2: the ARA's ranks exceed the smallest
 * ones its threshold allows by a few percent, which a pass applying the SVD
 * to every low rank tile removes).  Every strictly lower tile U V^T of the
 * input (which = TLR_INPUT) or of the factor (TLR_FACTOR) is replaced by its
 * truncated SVD at the absolute 2-norm threshold tau: the singular values
 * sigma_j > tau are kept, so each tile takes the smallest rank whose error
 * is at most tau and changes by sigma_{r+1} <= tau in the 2-norm (the
 * factorization's own threshold is stats->tau).  The new U has orthonormal
 * columns, the new V = right singular vectors times sigma.  The tile's
 * singular values are taken as the square roots of the eigenvalues of
 * V^T V, which assumes orthonormal U: true of the factor and of input built
 * by tlr_compress or tlr_compress_kernel; input with tiles from
 * tlr_set_tile returns TLR_ERR_STATE.  The Gram matrix squares the spread of
 * the singular values, so thresholds below about 1e-7 times a tile's norm
 * are not resolved.  Tiles of rank above 2048 are kept as they are.  The
 * panels shrink to the new ranks (offsets as tlr_get_offsets reports them);
 * the factor stays usable by tlr_solve and tlr_pcg.
 * Errors: TLR_ERR_ARG (tau negative or not finite, bad which; nothing
 * changes), TLR_ERR_STATE (no factor, or input of unknown U), TLR_ERR_OOM
 * when the work buffers cannot be allocated (nothing changes); a device
 * error after tiles have moved leaves the factor invalid (the input
 * undefined). */
tlr_status tlr_recompress(tlr_matrix_t A, int which, double tau, void* stream);

/* Y <- A X for the TLR input matrix (which = TLR_INPUT), X and Y N x nrhs in
 * device memory. */
tlr_status tlr_matvec(tlr_matrix_t A, int nrhs, const double* X, long long ldx, double* Y,
                      long long ldy, void* stream);

/* Sizes and bookkeeping.  which = TLR_INPUT or TLR_FACTOR. */
tlr_status tlr_get_info(tlr_matrix_t A, long long* N, int* m, int* nb, int* factored);
/* ranks: host array of nb * nb ints, row-major, strictly lower part filled. */
tlr_status tlr_get_ranks(tlr_matrix_t A, int which, int* ranks);
/* offsets: host array of nb * nb long longs: column of tile (i, j) in the
 * arena that holds all U (or V) factors side by side (input: row-major lower
 * order), or inside block row i's panel (factor); -1 off the strict lower
 * part. */
tlr_status tlr_get_offsets(tlr_matrix_t A, int which, long long* offsets);
/* Copy tile factors / diagonal tiles to host memory (ld >= m). */
tlr_status tlr_get_tile(tlr_matrix_t A, int which, int i, int j, double* U, double* V, int ld);
tlr_status tlr_get_diag(tlr_matrix_t A, int which, int k, double* D, int ld);
/* LDL^T pivots (nb * m entries including the padding) to host memory. */
tlr_status tlr_get_pivots(tlr_matrix_t A, double* d);
/* The "sortRanks" order (Section 4.2) in which the last factorization
 * presented the tiles of column k to its ARA: rows (host, nb - k - 1
 * entries) receives the block rows i > k by input rank a_ik descending, ties
 * by ascending i.  TLR_ERR_STATE if the handle holds no factor. */
tlr_status tlr_get_sort_order(tlr_matrix_t A, int k, int* rows);

tlr_status tlr_destroy(tlr_matrix_t A);
const char* tlr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TLR_H */
