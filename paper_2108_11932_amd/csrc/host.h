// Host-side state of the TLR library: the matrix handle, device memory,
// descriptor staging and batched-launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tlr.h"
#include "tlr_internal.h"

struct tlr_matrix_s;

namespace tlr {

using Handle = ::tlr_matrix_s;

void set_error(const char* fmt, ...);

// Status-propagating checks.
#define TLR_HIP(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      ::tlr::set_error("%s:%d: %s failed: %s", __FILE__, __LINE__, #expr,               \
                       hipGetErrorString(e_));                                          \
      return TLR_ERR_DEVICE;                                                            \
    }                                                                                   \
  } while (0)
#define TLR_TRY(expr)                  \
  do {                                 \
    tlr_status s_ = (expr);            \
    if (s_ != TLR_OK) return s_;       \
  } while (0)

// Device memory through the user allocator or hipMalloc.
struct Mem {
  tlr_allocator alloc{};
  bool custom = false;
  hipStream_t stream = nullptr;
  size_t live = 0;
  tlr_status get(void** p, size_t bytes);
  void put(void* p);
};

// A growable device buffer.  grow() keeps nothing; its old contents may be
// discarded because every use is ordered on the handle's stream.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  tlr_status ensure(Mem& mem, size_t bytes);
  void release(Mem& mem);
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Pinned host staging for descriptors and device read-backs.  Regions handed
// out stay valid until the next sync(), which waits for the stream and then
// recycles the staging areas.
struct Staging {
  char* host = nullptr;
  char* dev = nullptr;
  size_t cap = 0, used = 0;
  // when set, an upload larger than the whole ring fails (TLR_ERR_ARG)
  // instead of growing the ring: callers that must not allocate
  bool fixed = false;
  tlr_status init(Mem& mem, size_t bytes);
  void release(Mem& mem);
  // Copy `bytes` of host data to device memory on stream s (default: the
  // handle's main stream); returns the device address.
  tlr_status upload(Handle* h, const void* data, size_t bytes, void** dptr,
                    hipStream_t s = nullptr);
  // Copy `bytes` of host data straight into the device buffer `dst` (one
  // copy, through the pinned host ring).
  tlr_status upload_to(Handle* h, const void* data, size_t bytes, void* dst,
                       hipStream_t s = nullptr);
};

// One batch of GEMMs with uniform transposition.
struct GemmBatch {
  bool ta = false, tb = false;
  std::vector<GemmDesc> d;
  double flops = 0.0;
  GemmBatch(bool ta_, bool tb_) : ta(ta_), tb(tb_) {}
  void add(int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C,
           int ldc, double alpha, double beta, int flags = 0) {
    if (M <= 0 || N <= 0) return;
    d.push_back(GemmDesc{A, B, C, M, N, K, lda > 0 ? lda : 1, ldb > 0 ? ldb : 1, ldc, flags, alpha,
                         beta});
    flops += 2.0 * M * N * (double)K;
  }
  // Stage descriptors and block map in one copy, then launch on stream s
  // (default: the handle's main stream).
  tlr_status run(Handle* h, hipStream_t s = nullptr);
};

// A sequence of launches whose descriptors are staged with a single copy:
// add() batches in launch order, then run() uploads everything once and
// issues the launches on the plan's stream.
struct Plan {
  Handle* h;
  hipStream_t s;
  std::vector<char> blob;
  std::vector<std::function<hipError_t(const char*)>> steps;
  double flops = 0.0;
  Plan(Handle* h_, hipStream_t s_ = nullptr);
  // stage raw bytes; returns the offset of the copy inside the device blob
  size_t stage(const void* p, size_t n);
  void gemm(const GemmBatch& b);
  // a launch that reads staged bytes at `off` (device address passed in)
  void launch(size_t off, std::function<hipError_t(const char*)> f);
  // a launch that needs no staged data
  void launch(std::function<hipError_t()> f);
  // Issue all launches (run) or the next max_steps of them (run_some; the
  // first call uploads the staged bytes).  With `persist` set, the staged
  // bytes are copied into that buffer, so a plan may stay partly unlaunched
  // while the staging area is recycled.
  tlr_status run();
  tlr_status run_some(size_t max_steps);
  bool pending() const { return !steps.empty(); }
  DevBuf* persist = nullptr;
  // With `splitk` set, a batch of one long product with few output tiles
  // may be computed as partial products over K slices in this buffer (when
  // it is large enough), followed by their sum.
  DevBuf* splitk = nullptr;
  size_t cursor = 0;
  bool started = false;
  const char* base = nullptr;
};

// A host thread that issues the launches of the diagonal-tile stream, so
// that the thread driving the ARA iterations spends no time on them.  Tasks
// run in submission order on device `dev`.
class SideWorker {
 public:
  explicit SideWorker(int dev);
  ~SideWorker();
  void submit(std::function<tlr_status()> f);
  // Until every submitted task has run; the first failure since the last wait.
  tlr_status wait();

 private:
  void loop(int dev);
  std::mutex mu_;
  std::condition_variable cv_, idle_cv_;
  std::deque<std::function<tlr_status()>> q_;
  bool stop_ = false, busy_ = false;
  tlr_status err_ = TLR_OK;
  std::thread th_;
};

// Per-column workspace of the factorization.
struct Work {
  DevBuf G, W, omega, P, Z, T, Ta, H, Ball, C, Wa, Y, Q, part, ints, orth, dscale, tol,
      compact, Bt, fro, tnpart, tnpart2, splitk, G2, Gk, Sg, Sw, Snorm;
  // buffers of the diagonal-tile stream (never touched by the main stream)
  DevBuf Wd, dW, dtol, sideblob, sideblob2, Wn;
  // Schur compensation: D_k, the sign iterates X and X', X^2, E (m x m
  // each), the norm's partial sums and the norm
  DevBuf schur;
  int slots = 0;   // slot capacity of the per-tile buffers
  void release_all(Mem& mem) {
    DevBuf* bufs[] = {&G, &W, &omega, &P, &Z, &T, &Ta, &H, &Ball, &C, &Wa, &Y, &Q, &part,
                      &ints, &orth, &dscale, &tol, &compact, &Bt, &fro, &tnpart, &tnpart2,
                      &splitk, &G2, &Sg, &Sw, &Snorm,
                      &Gk, &Wd, &dW, &dtol, &sideblob, &sideblob2, &Wn, &schur};
    for (DevBuf* b : bufs) b->release(mem);
  }
};

// The blocked factorization of a diagonal tile (the launches of
// dense_factor) captured once as a HIP graph on fixed buffers, and replayed
// for every column: one graph launch on the diagonal-tile stream instead of
// one launch per panel.  mode: 0 Cholesky, 1 modified Cholesky (pivot floor
// read from tol, filled before each replay), 2 LDL^T.  The graph writes its
// status word (rows local to the tile) to info; the caller merges and
// clears it after each replay (launch_diag_out).
struct DiagGraph {
  int m = 0, mode = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;   // capture stream: records, never executes
  DevBuf A, Linv, W, D, info, tol, desc;
  void destroy(Mem& mem);
};

// Phase timing of one stream (TLR_FLAG_PHASE_TIMING): events recorded at the
// phase boundaries; the GPU time between a mark and the next one is charged
// to the phase of the first (phase < 0: not charged, e.g. an idle gap on the
// second stream).  The events are pooled and reused across calls.
struct PhaseTimer {
  bool on = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ph;
  size_t n = 0;
  void reset(bool enable) {
    on = enable;
    n = 0;
    ph.clear();
  }
  hipError_t mark(int phase, hipStream_t s);
  // after the stream has completed: add the charged times (ms) to t
  tlr_status collect(double* t);
  void destroy();
};

}  // namespace tlr

// The matrix handle behind the opaque tlr_matrix_t.
struct tlr_matrix_s {
  using Mem = tlr::Mem;
  using Staging = tlr::Staging;
  using Work = tlr::Work;
  long long N = 0;
  int m = 0, nb = 0, dev = 0;
  Mem mem;
  hipStream_t stream = nullptr;   // caller's stream: everything is ordered on it
  hipStream_t side = nullptr;     // library stream for the diagonal tiles (default priority)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_gnext = nullptr;
  std::unique_ptr<tlr::SideWorker> worker;   // issues the side-stream launches
  Staging stage;
  tlr::PhaseTimer pt_main, pt_side;   // TLR_FLAG_PHASE_TIMING

  // input matrix
  double* Ad = nullptr;           // nb diagonal tiles, m x m each
  std::vector<int> a_rank;        // nb * nb, strictly lower
  std::vector<long long> a_off;   // arena column of tile (i, j)
  long long a_cols = 0;
  double* UA = nullptr;
  double* VA = nullptr;
  double norm_a = 0.0;            // ||A||_2 estimate, 0 = not computed
  bool a_orth = false;            // every input U has orthonormal columns (compressed input)
  std::vector<double> a_fro;      // ||A_ij||_F bound per tile (mixed precision), empty = stale

  // factor
  int factored = 0;               // 0 none, 1 Cholesky, 2 LDL^T
  double* Ld = nullptr;
  double* Li = nullptr;           // nb tiles L_kk^{-1}, m x m each
  double* Dv = nullptr;           // nb * m LDL^T pivots
  std::vector<int> l_rank;
  std::vector<long long> l_off;   // column of tile (i, j) inside row i's panel
  std::vector<int> R, cap;        // panel width and capacity per block row
  std::vector<double*> UL, VL;
  // packed FP32 / BF16 copies of the U panels (mixed precision; layout of
  // pack_index, capacity cap[i] columns)
  std::vector<float*> UL32;
  std::vector<unsigned short*> UL16;
  // panels replaced by larger ones during a factorization: queued work may
  // still read them, so they are released once the factorization has
  // synchronised (or with the factor)
  std::vector<void*> retired;
  // copies the current factorization keeps: 0 none, 1 UL32, 2 UL32 and UL16
  int mixed = 0;
  std::vector<double> l_fro;      // ||L_ij||_F per tile (U orthonormal: ||V_ij||_F)
  // sortRanks order of every column's tiles in the last factorization
  // (global block rows, column k at sort_log[k])
  std::vector<std::vector<int>> sort_log;
  // pivoted factorization (Section 5.2): position -> original block of the
  // factor's block order (empty: unpivoted), and the updated diagonal tiles
  // A_tt - sum_j L_tj L_tj^T of the positions not yet factored (nb tiles of
  // m x m; position t at Sd + spos[t] m^2)
  std::vector<int> fperm;
  double* Sd = nullptr;
  std::vector<int> spos;
  double* pin_norm = nullptr;     // pinned read-back of a column's V norms
  int* pin_ring = nullptr;        // pinned read-back ring of the ARA iterations (2 x 8)
  int* pin_res = nullptr;         // pinned read-back of an ARA run's per-slot results
  size_t pin_res_n = 0;
  hipEvent_t ev_rb[2] = {nullptr, nullptr};
  size_t pin_norm_n = 0;

  Work ws;
  int* d_info = nullptr;          // device status word
  tlr::DiagGraph dg;              // captured diagonal-tile factorization

  int nreal(int k) const {
    const long long r = N - (long long)k * m;
    return r >= m ? m : (int)r;
  }
  double* diagA(int k) const { return Ad + (size_t)k * m * m; }
  double* diagL(int k) const { return Ld + (size_t)k * m * m; }
  double* invL(int k) const { return Li + (size_t)k * m * m; }
  double* ua(int i, int j) const { return UA + (size_t)a_off[(size_t)i * nb + j] * m; }
  double* va(int i, int j) const { return VA + (size_t)a_off[(size_t)i * nb + j] * m; }
  int ar(int i, int j) const { return a_rank[(size_t)i * nb + j]; }
  // Input tile (i, j), i > j, in the block order of the current
  // factorization: position t holds the original block fperm[t] (empty
  // fperm: the original order).  A pair that lies above the diagonal in the
  // original order is the transpose of the stored tile (U and V swapped).
  int pr(int i, int j) const {
    if (fperm.empty()) return ar(i, j);
    const int a = fperm[i], b = fperm[j];
    return a > b ? ar(a, b) : ar(b, a);
  }
  double* pu(int i, int j) const {
    if (fperm.empty()) return ua(i, j);
    const int a = fperm[i], b = fperm[j];
    return a > b ? ua(a, b) : va(b, a);
  }
  double* pv(int i, int j) const {
    if (fperm.empty()) return va(i, j);
    const int a = fperm[i], b = fperm[j];
    return a > b ? va(a, b) : ua(b, a);
  }
  int lr(int i, int j) const { return l_rank[(size_t)i * nb + j]; }
  double* ul(int i, int j) const { return UL[i] + (size_t)l_off[(size_t)i * nb + j] * m; }
  double* vl(int i, int j) const { return VL[i] + (size_t)l_off[(size_t)i * nb + j] * m; }
  long long lo(int i, int j) const { return l_off[(size_t)i * nb + j]; }

  tlr_status sync();          // both streams; recycles the staging area
  tlr_status sync_main();     // the caller's stream only
  tlr_status init_streams();
  tlr_status pinned_norms(size_t n, double** p);
  tlr_status readback_ring(int** p);
  tlr_status readback_results(size_t n, int** p);   // pinned, n ints
  void release_host();            // pinned buffers and events
};

namespace tlr {

// Dense tile operations built from the diagonal-block kernel and the batched
// GEMM, on stream s.  The factor overwrites A (lower, upper part zeroed);
// Linv (ld m) receives the inverse of the lower factor.  For LDL^T the
// factor is unit lower and d the pivots.
tlr_status dense_potrf(Handle* h, double* A, int lda, int m, int row_base, double* Linv,
                       hipStream_t s);
tlr_status dense_ldlt(Handle* h, double* A, int lda, int m, double* d, int row_base, double* Linv,
                      hipStream_t s);
tlr_status dense_trsm(Handle* h, const double* L, int ldl, double* B, int ldb, int m, int n,
                      bool unit, bool trans);
// Append the blocked factorization of A and the assembly of Linv to a plan
// (on the plan's stream); d is the pivot vector for LDL^T (chol = false).
// chol with mod_delta > 0: modified Cholesky (non-positive pivots replaced by
// mod_delta and counted in d_info[1]).
tlr_status dense_factor(Handle* h, struct Plan& plan, bool chol, double* A, int lda, int m,
                        double* d, int row_base, double* Linv, double mod_delta = 0.0);
// The handle's captured diagonal-tile factorization for tile size m and
// mode (DiagGraph), built on first use (or when m or mode change: then both
// streams are drained first).
tlr_status diag_graph(Handle* h, int m, int mode, DiagGraph** out);

// Kernel wrappers not declared in tlr_internal.h.
// p[0 .. n) = v
hipError_t launch_fill(double* p, long long n, double v, hipStream_t s);
// tol[0] = 64 u ||A||_F for the m x m tile A (lower triangle); tol must hold
// kPivotTolDoubles doubles (partial sums beside the result).
constexpr int kPivotTolDoubles = 32 + 256;
hipError_t launch_pivot_tol(const double* A, int lda, int m, double* tol, hipStream_t s);
// *out = ||x||_2 (device; parts: kPivotTolDoubles - 32 doubles of device
// scratch), summed in a fixed order; x = y / *sc (y where *sc is zero).
hipError_t launch_norm2(const double* x, long long n, double* out, double* parts, hipStream_t s);
hipError_t launch_scale_by(const double* y, long long n, const double* sc, double* x,
                           hipStream_t s);

// Batched ARA over a set of explicitly sampled operators: shared by the
// factorization (Schur-complement tiles) and the compression (explicit tiles).
struct AraProblem;

// "sortRanks" (Section 4.2): the permutation idx of 0 .. n - 1 that orders
// the entries by rank descending, ties by row ascending, then by index.
void sort_ranks(const int* ranks, const int* rows, int n, int* idx);

// piv: the pivoted Cholesky (Section 5.2; ldl false, FP64 sampling).
tlr_status factorize(Handle* h, double eps, const tlr_opts& o, tlr_stats* st, bool ldl,
                     bool piv = false);
// count problems at once, problem i at threshold eps[i] (st: count entries or
// NULL); problems of one tile size step through their columns together with
// pooled ARA launches.  All handles must use the same main stream.
tlr_status factorize_batch(Handle* const* hs, int count, const double* eps, const tlr_opts& o,
                           tlr_stats* st, bool ldl, bool piv = false);
tlr_status compress(Handle* h, const double* A, long long lda, const double* pts, int dim,
                    int kernel, double ell, double diag_add, double eps, const tlr_opts& o);
tlr_status estimate_norm(Handle* h, double* out);
tlr_status recompress(Handle* h, int which, double tau);
tlr_status matvec(Handle* h, int nrhs, const double* X, long long ldx, double* Y, long long ldy);
tlr_status solve(Handle* h, int nrhs, double* B, long long ldb);
// Doubles of workspace the solve of nrhs right-hand sides needs.
size_t solve_workspace(const Handle* h, int nrhs);
// The solve with a caller-provided workspace of solve_workspace() doubles
// (device memory); allocates nothing.
tlr_status solve_in(Handle* h, int nrhs, double* B, long long ldb, double* work);
tlr_status alloc_input(Handle* h, const int* ranks);
void free_factor(Handle* h);

}  // namespace tlr
