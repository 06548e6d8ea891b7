// Batched adaptive randomized approximation with dynamic batching, shared by
// the factorization (Schur-complement tiles of a column, sampled through the
// left-looking update) and the compression (explicit tiles).
//
// Algorithm "Left Looking Cholesky TLR ARA Update" (Section 4.2): the tiles
// of the batch are ordered (sortRanks), a subset is active; every iteration
// draws a Gaussian block, samples the active operators, orthogonalises the
// samples against the current bases by two passes of block Gram-Schmidt
// whose QR steps are Cholesky QR with a double-double Gram (pass 1 pivoted
// and thresholded), appends the new directions, flags the converged tiles
// and compacts/refills the active subset.
//
// The loop is device-driven: the active list, its count and the basis widths
// live in device memory and every kernel of an iteration reads them, so the
// host enqueues iteration t + 1 before it reads back the state after
// iteration t (one iteration of lookahead; a speculative iteration after
// convergence finds no active tile and does nothing).  Launch sizes come
// from host-side bounds on the active count and basis widths.
#pragma once

#include <functional>

#include "host.h"

namespace tlr {

struct AraConfig {
  int m = 0;          // rows of every operator
  int bs = 16;        // samples per iteration (the first iteration)
  int bs_tail = 0;    // samples per iteration after the first (0: bs)
  int tail_active = 0;   // > 0: bs_tail only while at most this many tiles are active
  int qcap = 0;       // basis capacity (columns)
  double tau = 0.0;   // absolute 2-norm threshold
  int r_min = 1;
  int s_max = 0;      // active subset size (<= 0: all)
  unsigned long long seed = 0;
  unsigned stream_id = 0;   // Philox counter word 2 (column index or batch id)
  int strip = 0;      // rows per workgroup of the sampling product (0: automatic, 16, 64)
  // sample iteration t + 1 in the launches of iteration t's second
  // Gram-Schmidt pass (only when no tile waits for a place in the active
  // subset, so that the next active list is the current one less the tiles
  // that converge, and for block sizes 16 and 32)
  bool overlap = true;
  // samples drawn by iteration `iter`, `active` tiles being active at its start
  int bs_for(int iter, int active) const {
    if (iter == 0 || bs_tail <= 0) return bs;
    return (tail_active <= 0 || active <= tail_active) ? bs_tail : bs;
  }
  int bs_max() const { return bs_tail > bs ? bs_tail : bs; }
};

// Per-slot workspace of an ARA batch (views into the handle's workspace).
struct AraSlots {
  int n = 0;
  int m = 0, bs = 0, nstrip = 0;
  double* Y = nullptr;      // 2 copies of n x (m x bs), yalt doubles apart
  double* Q = nullptr;      // n x (m x (qcap + bs))
  double* C = nullptr;      // n x (m x bs)
  double* part1 = nullptr;  // 2 copies of n x (nstrip x bs x bs x 2), palt doubles apart
  double* part2 = nullptr;
  int* counts = nullptr;    // 8
  int* act = nullptr;       // n
  int* q = nullptr;         // n
  int* qnew = nullptr;      // n
  int* flag = nullptr;      // n
  int* iters = nullptr;     // n
  int* qsum = nullptr;      // n
  int* ncol = nullptr;      // n: samples drawn per slot
  int* f32 = nullptr;       // n: precision chosen per slot
  int* qpa = nullptr;       // n: basis widths at the start of even iterations
  int* qpb = nullptr;       // n: ... of odd iterations
  int* counts2 = nullptr;   // 8: the counters of odd iterations
  int* act2 = nullptr;      // n: the active list of odd iterations
  int* piv = nullptr;       // n x (bs + 1)
  int* waiting = nullptr;   // n
  long long yalt = 0, palt = 0;
  size_t qstride = 0;       // doubles per slot in Q
  double* y(int s) const { return Y + (size_t)s * m * bs; }
  double* qb(int s) const { return Q + (size_t)s * qstride; }
  double* c(int s) const { return C + (size_t)s * m * bs; }
  double* p1(int s) const { return part1 + (size_t)s * nstrip * bs * bs * 2; }
  double* p2(int s) const { return part2 + (size_t)s * nstrip * bs * bs * 2; }
};

// P_g = U_g^T Omega of one problem of the batch (U_g m x rk, its row-k
// panel), stored in rows [roff, roff + rk) of the shared P.
struct PGroup {
  const double* uk;
  int rk, roff;
};

// What each slot samples, fixed for the whole run.  The caller fills the
// sampling fields of every AraSlotDesc (a0/b0/a1/b1, W^A and Z, whose
// pieces address P by absolute row); ara_run fills the workspace fields
// and the thresholds.
struct AraSpec {
  std::vector<AraSlotDesc> slots;
  std::vector<ZSeg> zseg;
  std::vector<PGroup> pg;       // the P products (none for explicit tiles)
  double* p = nullptr;          // P of every group, leading dimension ldp
  int ldp = 0;
  std::vector<double> tau;      // per-slot absolute threshold (empty: the config's)
  int a_max = 0;                // largest W^A height over the slots
  int r_max = 0;                // largest Z height over the slots
  // sampling cost per slot: bytes per iteration = samp_bytes + samp_bytes_col
  // * (samples of the iteration); flops = samp_flops_col * samples
  std::vector<double> samp_bytes, samp_bytes_col, samp_flops_col;
  // mixed precision: one precision choice per slot, made on the device
  // before the first iteration; samp_bytes32 replaces samp_bytes for the
  // slots that take their FP32 panel
  std::vector<GuardDesc> guard;
  std::vector<double> samp_bytes32, samp_bytes16;
  // when set, HIP events are recorded around every sampling launch
  std::vector<std::pair<hipEvent_t, hipEvent_t>>* events = nullptr;
  // when set, the phase boundaries of every iteration are marked on it
  PhaseTimer* pt = nullptr;
};

struct AraResult {
  std::vector<int> q;          // final basis width per slot
  std::vector<int> iters;      // iterations per slot
  std::vector<int> cols;       // samples drawn per slot
  std::vector<int> f32;        // precision of the slot's panel term: 0 FP64, 1 FP32, 2 BF16
  std::vector<int> iter_bs;    // samples per slot of every launched iteration
  std::vector<double> flops_paper_orth;  // per slot: orthogonalisation flops
  long long launches = 0;      // ARA iterations (batches)
  double t_issue = 0.0, t_wait = 0.0;   // host ms issuing launches / waiting for results
  double flops = 0.0;          // executed flops (sampling, Gram-Schmidt, orthogonalisation)
  double samp_bytes = 0.0, samp_flops = 0.0;   // of the sampling launches
  // the same per slot
  std::vector<double> flops_slot, samp_bytes_slot, samp_flops_slot;
};

// Spec of n explicit m x m tiles (tile t at tiles + t * ld * m, ld >= m):
// Y_t = T_t Omega.
tlr_status ara_explicit_spec(Handle* h, const AraConfig& c, int n, const double* tiles, int ld,
                             AraSpec* spec);

// Allocate the slot buffers for n slots.
tlr_status ara_slots(Handle* h, const AraConfig& c, int n, AraSlots* s);
// The Gaussian test-matrix buffer the iterations draw into: kOmegaBatch
// matrices of m x bs_max (the test matrices of that many consecutive
// iterations are drawn by one launch); explicit tiles use the first.
constexpr int kOmegaBatch = 16;
tlr_status ara_omega(Handle* h, const AraConfig& c, double** omega);

// Run the ARA loop.  `order` lists the slots in processing order (the
// sortRanks order); the first s_max start active.  `info_abort` is checked
// after the first iteration (a failed diagonal factorization ends the run).
// `idle`, when set, is called once per iteration while the host would
// otherwise wait for the device (the factorization issues the launches of
// the diagonal-tile stream from it).
tlr_status ara_run(Handle* h, const AraConfig& c, const AraSlots& s, const std::vector<int>& order,
                   AraSpec& spec, AraResult* res, bool* info_abort,
                   const std::function<tlr_status()>& idle = nullptr);

}  // namespace tlr
