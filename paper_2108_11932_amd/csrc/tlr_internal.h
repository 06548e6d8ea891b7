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
  int flags;   // GEMM_* bits
  double alpha, beta;
  int koff;    // K offset of this slice of a split contraction (triangle clipping)
};
// Only output tiles that reach the lower triangle (row >= col) are computed.
constexpr int GEMM_LOWER_C = 1;
// op(A) is lower triangular (k <= row): the K loop of a row tile stops at
// its last row.
constexpr int GEMM_TRIL_A = 2;
// op(A) is upper triangular (k >= row): the K loop starts at the tile's
// first row.
constexpr int GEMM_TRIU_A = 4;
// C receives the transpose of the product (element (r, c) of op(A) op(B) at
// C[c + r ldc]); transposed-A products on the LDS-streamed kernel only.
constexpr int GEMM_STORE_T = 8;

// One entry per launched workgroup: x = descriptor index, y = output tile
// index inside that descriptor (row tiles vary fastest).
struct BlockMap {
  int desc;
  int tile;
};

// Host-side staging of a batched GEMM; builds the block map and launches.
// trans_a / trans_b are uniform over the batch.
int gemm_tile_n(int N);                     // BN chosen for a problem (16 or 64)
// Output tile (rows x cols) of the kernel that runs a batch with these
// transpositions and largest N; the block map enumerates tiles of this shape.
void gemm_tile_shape(bool trans_a, bool trans_b, int maxn, int* tm, int* tn);
// bn = 0 selects 16 x 16 tiles (transposed A only).
// Transposed-A batches streamed through LDS: tiles bm x bn in {16 x 16,
// 64 x 16, 64 x 32}; every problem must pass gemm_tn_lds_ok.
bool gemm_tn_lds_ok(const GemmDesc& d);
hipError_t launch_gemm_tn_lds(const GemmDesc* d_descs, const BlockMap* d_map, int nblocks, int bm,
                              int bn, hipStream_t s);
// C = alpha * sum_s part_s + beta * C over an M x N block, the S partial
// products stored one after another (M x N each, leading dimension M) and
// added in order s = 0, 1, ...
hipError_t launch_splitk_sum(double* C, int ldc, int M, int N, const double* part, int S,
                             double alpha, double beta, hipStream_t s);
// max_k: the largest K of the batch (picks the depth of the K slices).
hipError_t launch_gemm_batched(const GemmDesc* d_descs, const BlockMap* d_map, int nblocks,
                               bool trans_a, bool trans_b, int bn, int max_k, hipStream_t s);

// ---------------------------------------------------------------------------
// Dense tile kernels (one m x m tile, m <= 4096)
// ---------------------------------------------------------------------------
// Width of the diagonal blocks the factorization kernel handles (32).
int diag_block_size();
// Blocked factorization of the m x m tile A by panels of diag_block_size()
// columns: Cholesky A = L L^T, or unit LDL^T A = L D L^T with scalar pivots
// into dvec (device, m).  Inv (ld ldi) receives the inverse of every
// diagonal block of L (unit for LDL^T) at (32 b, 32 b), zeros above its
// diagonal.  info (device, two ints) receives the 1-based row (row_base +
// row + 1) of the first failing pivot in info[0]; tolp (device) is the
// LDL^T pivot tolerance, or, for Cholesky, the floor of modified Cholesky
// (a non-positive pivot becomes max(|d|, *tolp) and is counted in info[1]
// instead of failing); nullptr for plain Cholesky.
//   launch_potrf_first: the first diagonal block (one wave);
//   launch_potrf_step: panel p0 (p0 a multiple of 32, p0 + 32 < m): the
//     panel below its block into Lp (ld ldp, same positions as in A), the
//     trailing update of A, and the next diagonal block factored into A;
//   launch_tri_finish: the panels from Lp into A, zeros above the diagonal.
hipError_t launch_potrf_first(bool chol, double* A, int lda, int m, double* Inv, int ldi,
                              double* dvec, int* info, int row_base, const double* tolp,
                              hipStream_t s);
hipError_t launch_potrf_step(bool chol, double* A, int lda, int m, int p0, double* Lp, int ldp,
                             double* Inv, int ldi, double* dvec, int* info, int row_base,
                             const double* tolp, hipStream_t s);
hipError_t launch_tri_finish(double* A, int lda, const double* Lp, int ldp, int m, hipStream_t s);
// After a replay of the captured diagonal-tile factorization: the factor A
// and the inverse Linv (m x m, ld m) to Adst and Ldst (ld m), the pivots D
// to Ddst (both NULL for Cholesky), and the graph's status word ginfo (two
// ints, rows local to the tile) into info (first failing row row_base +
// ginfo[0], modified pivots added), ginfo then cleared.
hipError_t launch_diag_out(const double* A, double* Adst, const double* Linv, double* Ldst,
                           const double* D, double* Ddst, int m, int* ginfo, int* info,
                           int row_base, hipStream_t s);
// out(r, c) = in(r, c) * s[c] (or / s[c]).
hipError_t launch_scale_cols(const double* in, int ldi, double* out, int ldo, const double* sc,
                             int rows, int cols, bool inverse, hipStream_t s);
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
// The test matrices of nt consecutive iterations t0 .. t0 + nt - 1 in one
// launch (rows x cols0 for iteration 0, rows x cols1 after, leading
// dimension rows, matrix t - t0 at out + (t - t0) * stride): the values
// launch_randn gives for each t.
hipError_t launch_randn_iters(double* out, int rows, size_t stride, int cols0, int cols1,
                              unsigned long long seed, unsigned k, unsigned t0, int nt,
                              unsigned stream, hipStream_t s);
hipError_t launch_philox_raw(unsigned* out, int n, unsigned long long seed, unsigned c1, unsigned c2,
                             unsigned c3, hipStream_t s);

// Per-tile descriptor for the orthogonalisation of one ARA block.
// ---------------------------------------------------------------------------
// Device-driven ARA iterations (Algorithm "Left Looking Cholesky TLR ARA
// Update"): every kernel of an iteration reads the active list, its count and
// the basis widths from device memory, so the host enqueues iterations
// without waiting for the previous one.  Grids are sized by host-side upper
// bounds; blocks beyond the current active set or basis width exit.
// ---------------------------------------------------------------------------
// Static description of one slot (one tile) for a whole ARA run.
struct AraSlotDesc {
  // sample Y = A0 B0 + A1 B1 (m x bs)
  const double* a0;       // m x k0 (ld lda0): U^A_ik, or the explicit tile
  const double* b0;       // k0 x bs (ld ldb0): W^A below, or Omega
  const void* a1;         // m x k1: the row panel U_i*, FP64 column-major (ld
                          // lda1), or its packed FP32 / BF16 copy (lda1 = row
                          // blocks of the packing), as a1_prec says
  const double* b1;       // k1 x bs (ld ldb1): Z below
  int lda0, ldb0, k0, lda1, ldb1, k1;
  int a1_prec;            // 0 FP64, 1 packed FP32, 2 packed BF16 (FP32 accumulation)
  // W^A = V^A_ik^T Omega (a x bs, ld a), when a > 0
  const double* va;
  double* wa;
  int a;
  // Z = -[G_ij P_j]_j (R x bs, ld R) over the tiles [zseg, zseg + nz)
  int zseg, nz, R;
  double* z;
  double tau2;            // squared absolute threshold of this tile
  // workspace
  double* y;              // m x bs
  double* q;              // m x (qcap + bs) basis
  double* c;              // m x bs, C = -Q^T Y
  double* part1;          // Gram partials of Y per 16-row strip: nstrip x bs x bs x 2
  double* part2;          // Gram partials of the new columns X
  int* piv;               // pivots, then the accepted count at [bs]
};
// One 32-row tile of a product P_g = U_g^T Omega (U_g m x M, ld m) stored at
// C (leading dimension ldp) from row row0: the P of one problem of a batch.
struct PTile {
  const double* A;
  double* C;
  int M, row0;
};
// One 16-row piece of a block of Z:
// Z(zrow + r, :) = -G(r, 0 : cols) P(prow : prow + cols, :), r < rows <= 16,
// G column-major with leading dimension ldg.
struct ZSeg {
  const double* g;
  int ldg, rows, cols, zrow, prow;
};
// Device state of one ARA run (passed by value).
struct AraDev {
  const AraSlotDesc* slots;
  int* act;     // active slots of this iteration, counts[0] of them
  int* counts;  // [0] active, [1] waiting cursor, [2] status word copy, [3] max basis width of the active slots
  // the next iteration's list and counters, formed by the compaction (two
  // copies alternate by iteration, so that the compaction can run while
  // this iteration's launches still read its list)
  int* act_next;
  int* counts_next;
  // basis width per slot at the start of this iteration (qin) and after it
  // (qout, set by pass 1); two copies alternate by iteration
  const int* qin;
  int* qout;
  int* q;       // latest basis width per slot (the run's result)
  int* qnew;    // basis width after this iteration's pass 1
  int* flag;    // converged
  int* iters;   // iterations per slot
  int* qsum;    // sum over iterations of the samples times the prior basis width
  int* ncol;    // samples drawn per slot
  int m, bs, qcap, nstrip;
  // the iteration's sample block and Gram partials: slot descriptor's y and
  // part1 plus these offsets (doubles), so that the sampling of the next
  // iteration can fill the other copy while this one is orthogonalised
  long long yoff, poff;
  // when set, the sampling launches skip the slots with skip[slot] != 0
  // (the convergence flags of the iteration before)
  const int* skip;
};
// Precision choice of one slot under mixed precision.  With
// nu_tot = nu + fro[irow] fro[0] (no device term when irow < 0; fro holds the
// Frobenius norms of the previous column's factor tiles, row k - 1 + 1 + s
// at s, on the device) the slot samples its panel from the packed BF16 copy
// a1_16 when nu_tot <= lim16, else from the packed FP32 copy a1_32 when
// nu_tot <= lim32, else in FP64 (a NULL copy is never chosen).  nrb: row
// blocks of the packing.
struct GuardDesc {
  const void* a1_32;
  const void* a1_16;
  const double* fro;
  double nu, lim32, lim16;
  int irow, nrb;
};
// Applies the choice to the n slot descriptors (panel pointer, leading
// dimension and precision) and stores it in prec[slot] (0 FP64, 1 FP32,
// 2 BF16).
hipError_t launch_mixed_guard(AraSlotDesc* slots, const GuardDesc* g, int n, int* prec,
                              hipStream_t s);
// Block sizes the orthogonalisation kernels are built for (1, 2, 4, 8, 16,
// 24, 32).
bool orth_block_supported(int bs);
// mode 0: the P tiles (P_g = U_g^T Omega, one group of tiles per problem,
//         all stored with leading dimension ldp) and W^A = V^A^T Omega per
//         active slot (tps tiles per slot);
// mode 1: C = -Q^T Y; mode 2: C = -Q^T X, X = Q(:, q : q + bs) (tps tiles).
// K is split over workgroups whose partial tiles go to scratch and are
// summed by a second launch; ara_tn_scratch gives the doubles of scratch for
// `tiles` output tiles (and returns the tile height).
int ara_tn_scratch(int m, int bs, long long tiles, size_t* doubles);
hipError_t launch_ara_tn(const AraDev& D, int mode, const double* omega, const PTile* ptiles,
                         int p_tiles, int ldp, int count_bound, int tps, double* scratch,
                         hipStream_t s);
// Z of every active slot (bps blocks of four Z pieces per slot).
hipError_t launch_ara_z(const AraDev& D, const ZSeg* segs, const double* P, int ldp,
                        int count_bound, int bps, hipStream_t s);
// mode 0: sample Y; mode 1: Y += Q C; mode 2: X += Q C; all write the Gram
// partials of their output (part1 for modes 0/1, part2 for mode 2).
// Mode 0 computes 64-row strips per workgroup when strip is 64, or when it
// is 0 and the launch has enough of them to fill the GPU, else 16-row strips
// (same result bit for bit).  With start/stop events (mode 0 only) the
// events record the launch's own begin and end.
hipError_t launch_ara_seg(const AraDev& D, int mode, int count_bound, hipStream_t s, int strip = 0,
                          hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// Fused launches of one ARA iteration step: the sampling of iteration t + 1
// (Da / Dz / D0: mode 0, its tiles less the ones the flags of t name)
// together with the second Gram-Schmidt pass of iteration t (Db / Ds / D2).
// Block sizes 16 and 32 only (fused_block_supported), the same in both.
// launch_fused_tn also runs the compaction of iteration t (the work of
// launch_ara_compact for Db, with the same arguments) in one more block.
bool fused_block_supported(int bs);
hipError_t launch_fused_tn(const AraDev& Da, const double* omega, const PTile* ptiles, int p_tiles,
                           int ldp, int cba, int tpsa, double* scra, const AraDev& Db, int cbb,
                           int tpsb, double* scrb, const int* waiting, int nwaiting, int s_max,
                           const int* info, int* host_out, int* host_res, int res_ints,
                           hipStream_t s);
hipError_t launch_fused_z_seg(const AraDev& Dz, const ZSeg* segs, const double* P, int ldp, int cbz,
                              int bps, const AraDev& Ds, int cbs, hipStream_t s);
hipError_t launch_fused_seg_orth(const AraDev& D0, int cb0, int strip, const AraDev& D2, int cb2,
                                 int r_min, hipStream_t s);
// Cholesky QR step of pass 1 (pivoted, thresholded: appends the accepted
// directions of Y to Q, sets qnew, flag, pivots, iteration counters and the
// Gram partials of the new columns) or pass 2 (re-orthonormalises the new
// columns in place).
// The threshold of each tile is its slot's tau2.
hipError_t launch_orth_step(const AraDev& D, int pass, int r_min, int count_bound, hipStream_t s);
// Compact the active list D.act into D.act_next and refill it (see
// launch_compact; D.counts to D.counts_next), and record the status word and
// the largest basis width (D.qout) on the new list; counts_next[0..3] are
// also stored to host_out (pinned host memory) when given;
// when no tile is left active, the res_ints ints from D.q (the per-slot
// results, laid out contiguously) are stored to host_res as well.
hipError_t launch_ara_compact(const AraDev& D, const int* waiting, int nwaiting, int s_max,
                              const int* info, int* host_out, int* host_res, int res_ints,
                              hipStream_t s);

// Dynamic batching: stable compaction of the active list by the convergence
// flags (flag[slot] != 0 removes the slot), then refill from the waiting
// list.  counts[0] = active count in/out, counts[1] = waiting cursor.
// When info is not NULL, counts[2] receives a copy of *info (status word
// read back together with the active list).
hipError_t launch_compact(int* act, int* counts, const int* flag, const int* waiting, int nwaiting,
                          int s_max, const int* info, hipStream_t s);

// ---------------------------------------------------------------------------
// Misc kernels
// ---------------------------------------------------------------------------
struct CopyDesc {
  const double* src;
  double* dst;
  int rows, cols, lds, ldd;
  // optional packed FP32 / BF16 copies of the destination (the layout of
  // pack_index, ceil(rows / 16) row blocks), written at columns pcol ..
  float* dst32 = nullptr;
  unsigned short* dst16 = nullptr;
  int pcol = 0;
};
// Frobenius norm of a rows x cols block (ld) into *out.
struct NormDesc {
  const double* p;
  int rows, cols, ld;
  double* out;
  double* host;   // when set, the norm is also stored here (pinned host memory)
};
hipError_t launch_fro_norms(const NormDesc* d, int n, hipStream_t s);
// Squared Frobenius norms of n symmetric m x m tiles (lower triangle, ld;
// tiles: device array of n pointers) as G partial sums per tile at out[t G
// + g] (the sum of a tile's partials in order is its squared norm).
hipError_t launch_sym_fro_parts(const double* const* tiles, int n, int m, int ld, int G,
                                double* out, hipStream_t s);
hipError_t launch_copy_batched(const CopyDesc* d, int n, int max_cols, hipStream_t s);

// SVD post-recompression (Section 6.2): symmetric eigensolver of the Gram
// matrices V^T V of low rank tiles.  G (q x q, ld q) is overwritten with the
// eigenvectors in descending order of the eigenvalues; res[0] receives the
// number r of eigenvalues with sqrt(lambda) > tau, res[1] their sum.  W is a
// q x q workspace for classes 2 and 3.  Classes: 0 for q <= kEigLdsSmall,
// 1 for q <= kEigLdsLarge (G and W in LDS), 2 for q <= kEigPacked (G packed
// in LDS, W in global memory), 3 for q <= kEigMaxRank (global memory).
// abs_scale > 0 adds the absolute rotation threshold abs_scale max_j g_jj
// to the relative one (the first of the two passes).
constexpr int kEigLdsSmall = 32, kEigLdsLarge = 96, kEigPacked = 180, kEigMaxRank = 2048;
struct EigDesc {
  double* G;
  double* W;
  double* res;
  int q;
};
// The solver class of a q x q problem (-1: above kEigMaxRank).
inline int eig_class(int q) {
  if (q <= kEigLdsSmall) return 0;
  if (q <= kEigLdsLarge) return 1;
  if (q <= kEigPacked) return 2;
  if (q <= kEigMaxRank) return 3;
  return -1;
}
hipError_t launch_sym_eig(const EigDesc* d, int n, int cls, double tau, double abs_scale,
                          hipStream_t s);
// Schur compensation (Section 5.1.1).  X = D - tau I (m x m, full).
hipError_t launch_schur_shift(const double* D, int m, double tau, double* X, hipStream_t s);
// T(j, j) += sum_i |E(i, j)| for j < nreal (E symmetric: the column sums are
// the row sums; one workgroup per column, a fixed-order sum).
hipError_t launch_schur_diag(const double* E, int m, double* T, int ldt, int nreal, hipStream_t s);
// dst = src (m x m) + shift on the first nreal diagonal entries.
hipError_t launch_copy_shift(const double* src, double* dst, int m, int nreal, double shift,
                             hipStream_t s);
// W(:, c) = V(:, c) .* Dv(:, colj[c]) (Dv m x nb, colj device, ncols entries).
hipError_t launch_scale_panel(const double* V, int ldv, double* W, int ldw, int m, int ncols,
                              const int* colj, const double* Dv, hipStream_t s);
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
