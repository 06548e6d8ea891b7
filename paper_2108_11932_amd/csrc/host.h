// Host-side state of the TLR library: the matrix handle, device memory,
// descriptor staging and batched-launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
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
  tlr_status init(Mem& mem, size_t bytes);
  void release(Mem& mem);
  // Copy `bytes` of host data to device memory; returns the device address.
  tlr_status upload(Handle* h, const void* data, size_t bytes, void** dptr);
};

// One batch of GEMMs with uniform transposition.
struct GemmBatch {
  bool ta = false, tb = false;
  std::vector<GemmDesc> d;
  double flops = 0.0;
  GemmBatch(bool ta_, bool tb_) : ta(ta_), tb(tb_) {}
  void add(int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C,
           int ldc, double alpha, double beta) {
    if (M <= 0 || N <= 0) return;
    d.push_back(GemmDesc{A, B, C, M, N, K, lda > 0 ? lda : 1, ldb > 0 ? ldb : 1, ldc, alpha, beta});
    flops += 2.0 * M * N * (double)K;
  }
  tlr_status run(Handle* h);
};

// Per-column workspace of the factorization.
struct Work {
  DevBuf G, W, omega, P, Z, T, Ta, H, Ball, C, Wa, Y, Q, part, rfac, ints, orth, dscale, tol,
      compact;
  int slots = 0;   // slot capacity of the per-tile buffers
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
  hipStream_t stream = nullptr;
  Staging stage;

  // input matrix
  double* Ad = nullptr;           // nb diagonal tiles, m x m each
  std::vector<int> a_rank;        // nb * nb, strictly lower
  std::vector<long long> a_off;   // arena column of tile (i, j)
  long long a_cols = 0;
  double* UA = nullptr;
  double* VA = nullptr;
  double norm_a = 0.0;            // ||A||_2 estimate, 0 = not computed

  // factor
  int factored = 0;               // 0 none, 1 Cholesky, 2 LDL^T
  double* Ld = nullptr;
  double* Dv = nullptr;           // nb * m LDL^T pivots
  std::vector<int> l_rank;
  std::vector<long long> l_off;   // column of tile (i, j) inside row i's panel
  std::vector<int> R, cap;        // panel width and capacity per block row
  std::vector<double*> UL, VL;

  Work ws;
  int* d_info = nullptr;          // device status word

  int nreal(int k) const {
    const long long r = N - (long long)k * m;
    return r >= m ? m : (int)r;
  }
  double* diagA(int k) const { return Ad + (size_t)k * m * m; }
  double* diagL(int k) const { return Ld + (size_t)k * m * m; }
  double* ua(int i, int j) const { return UA + (size_t)a_off[(size_t)i * nb + j] * m; }
  double* va(int i, int j) const { return VA + (size_t)a_off[(size_t)i * nb + j] * m; }
  int ar(int i, int j) const { return a_rank[(size_t)i * nb + j]; }
  int lr(int i, int j) const { return l_rank[(size_t)i * nb + j]; }
  double* ul(int i, int j) const { return UL[i] + (size_t)l_off[(size_t)i * nb + j] * m; }
  double* vl(int i, int j) const { return VL[i] + (size_t)l_off[(size_t)i * nb + j] * m; }
  long long lo(int i, int j) const { return l_off[(size_t)i * nb + j]; }

  tlr_status sync();
};

namespace tlr {

// Dense tile operations built from the panel kernels and the batched GEMM.
tlr_status dense_potrf(Handle* h, double* A, int lda, int m, int row_base);
tlr_status dense_ldlt(Handle* h, double* A, int lda, int m, double* d, int row_base);
tlr_status dense_trsm(Handle* h, const double* L, int ldl, double* B, int ldb, int m, int n,
                      bool unit, bool trans);

// Kernel wrappers not declared in tlr_internal.h.
hipError_t launch_zero_upper(double* A, int lda, int m, hipStream_t s);
hipError_t launch_pivot_tol(const double* A, int lda, int m, double* tol, hipStream_t s);
int gram_row_blocks(int m);

// Batched ARA over a set of explicitly sampled operators: shared by the
// factorization (Schur-complement tiles) and the compression (explicit tiles).
struct AraProblem;

tlr_status factorize(Handle* h, double eps, const tlr_opts& o, tlr_stats* st, bool ldl);
tlr_status compress(Handle* h, const double* A, long long lda, const double* pts, int dim,
                    int kernel, double ell, double diag_add, double eps, const tlr_opts& o);
tlr_status estimate_norm(Handle* h, double* out);
tlr_status matvec(Handle* h, int nrhs, const double* X, long long ldx, double* Y, long long ldy);
tlr_status solve(Handle* h, int nrhs, double* B, long long ldb);
tlr_status alloc_input(Handle* h, const int* ranks);
void free_factor(Handle* h);

}  // namespace tlr
