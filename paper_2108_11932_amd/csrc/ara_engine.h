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
// and compacts/refills the active subset on the device.
#pragma once

#include <functional>

#include "host.h"

namespace tlr {

struct AraConfig {
  int m = 0;          // rows of every operator
  int bs = 16;        // samples per iteration
  int qcap = 0;       // basis capacity (columns)
  double tau = 0.0;   // absolute 2-norm threshold
  int r_min = 1;
  int s_max = 0;      // active subset size (<= 0: all)
  unsigned long long seed = 0;
  unsigned stream_id = 0;   // Philox counter word 2 (column index or batch id)
};

// Per-slot buffers of one ARA batch (views into the handle's workspace).
struct AraSlots {
  int n = 0;
  int m = 0, bs = 0;
  double* Y = nullptr;   // n x (m x bs)
  double* Q = nullptr;   // n x (m x (qcap + bs))
  double* C = nullptr;   // n x (m x bs)
  double* part = nullptr;
  // contiguous read-back block: counts[2], status word copy, pad, act[n], qv[n]
  int* counts = nullptr; // 2 (+ 2)
  int* act = nullptr;    // n
  int* qv = nullptr;     // n
  int* flag = nullptr;   // n
  int* piv = nullptr;    // n x (bs + 1)
  int* waiting = nullptr;// n
  size_t qstride = 0;    // doubles per slot in Q
  double* y(int s) const { return Y + (size_t)s * m * bs; }
  double* q(int s) const { return Q + (size_t)s * qstride; }
  double* c(int s) const { return C + (size_t)s * m * bs; }
};

struct AraResult {
  std::vector<int> q;          // final basis width per slot
  std::vector<int> iters;      // iterations per slot
  std::vector<double> flops_paper_orth;  // per slot: orthogonalisation flops
  long long launches = 0;      // ARA iterations (batches)
  double flops = 0.0;          // executed flops (GEMM + orthogonalisation)
};

// Allocate the slot buffers for n slots.
tlr_status ara_slots(Handle* h, const AraConfig& c, int n, AraSlots* s);

// Sample callback: add to `plan` the launches that fill Y(s) = S_s * omega
// for every slot in `act`.
using SampleFn = std::function<tlr_status(const std::vector<int>& act, const double* omega,
                                          Plan& plan)>;

// Run the ARA loop.  `order` lists the slots in processing order (the
// sortRanks order); the first s_max start active.  `info_abort` is checked
// after the first iteration (a failed diagonal factorization ends the run).
tlr_status ara_run(Handle* h, const AraConfig& c, const AraSlots& s, const std::vector<int>& order,
                   const SampleFn& sample, AraResult* res, bool* info_abort);

}  // namespace tlr
