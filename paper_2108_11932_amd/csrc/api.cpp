// C ABI of the TLR library (include/tlr.h): argument validation, handle life
// cycle, data transfer in and out of the handle.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "host.h"

using namespace tlr;

namespace tlr {
const char* last_error();
}

#define TLR_ARG(cond, ...)          \
  do {                              \
    if (!(cond)) {                  \
      ::tlr::set_error(__VA_ARGS__); \
      return TLR_ERR_ARG;           \
    }                               \
  } while (0)

static constexpr int M_MAX = 8192;

extern "C" {

void tlr_opts_default(tlr_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->bs = 16;
  o->eps_mode = TLR_EPS_ABS;
  o->precision = TLR_FP64;
  o->shift = 0.0;
  o->max_active = 0;
  o->r_min = 0;
  o->seed = 0x5eedULL;
  o->flags = 0;
  o->bs_tail = 0;
  o->tail_active = 0;
}

const char* tlr_last_error(void) { return tlr::last_error(); }

}  // extern "C"

// Default of opts.conv_factor.
static constexpr double kConvFactor = 1.0;

static tlr_status check_opts(const tlr_opts* in, tlr_opts* out) {
  if (in)
    *out = *in;
  else
    tlr_opts_default(out);
  TLR_ARG(orth_block_supported(out->bs), "opts.bs must be one of 1, 2, 4, 8, 16, 24, 32, got %d",
          out->bs);
  TLR_ARG(out->eps_mode == TLR_EPS_ABS || out->eps_mode == TLR_EPS_REL, "opts.eps_mode invalid");
  TLR_ARG(out->precision >= TLR_FP64 && out->precision <= TLR_MIXED_AUTO,
          "opts.precision must be TLR_FP64, TLR_MIXED_FP32, TLR_MIXED_BF16 or TLR_MIXED_AUTO");
  TLR_ARG(out->r_min >= 0 && out->r_min <= out->bs, "opts.r_min must be in 0..bs");
  if (out->r_min == 0) {
    // half the smallest block of the run
    const int b = (out->bs_tail > 0 && out->bs_tail < out->bs) ? out->bs_tail : out->bs;
    out->r_min = b > 1 ? b / 2 : 1;
  }
  TLR_ARG(out->bs_tail == 0 || (orth_block_supported(out->bs_tail) && out->r_min <= out->bs_tail),
          "opts.bs_tail must be 0 or a supported block size >= r_min, got %d", out->bs_tail);
  TLR_ARG(out->tail_active >= 0, "opts.tail_active must be >= 0, got %d", out->tail_active);
  TLR_ARG(std::isfinite(out->shift), "opts.shift must be finite");
  TLR_ARG(out->sample_strip == 0 || out->sample_strip == 16 || out->sample_strip == 64,
          "opts.sample_strip must be 0, 16 or 64, got %d", out->sample_strip);
  TLR_ARG(out->conv_factor == 0.0 || (out->conv_factor >= 1.0 && std::isfinite(out->conv_factor)),
          "opts.conv_factor must be 0 (default) or >= 1");
  if (out->conv_factor == 0.0) out->conv_factor = kConvFactor;
  return TLR_OK;
}

static tlr_status new_handle(long long N, int m, const tlr_allocator* alloc, void* stream,
                             Handle** out) {
  TLR_ARG(out != nullptr, "output handle pointer is NULL");
  *out = nullptr;
  TLR_ARG(N > 0, "N must be positive, got %lld", N);
  TLR_ARG(m > 0 && m <= M_MAX, "tile size m must be in 1..%d, got %d", M_MAX, m);
  TLR_ARG(N <= (1LL << 31) - 1, "N too large");
  TLR_ARG(alloc == nullptr || (alloc->alloc && alloc->free), "allocator callbacks missing");
  Handle* h = new Handle();
  h->N = N;
  h->m = m;
  h->nb = (int)((N + m - 1) / m);
  h->stream = (hipStream_t)stream;
  h->mem.stream = h->stream;
  if (alloc) {
    h->mem.alloc = *alloc;
    h->mem.custom = true;
  }
  if (hipGetDevice(&h->dev) != hipSuccess) {
    (void)hipGetLastError();
    delete h;
    set_error("no HIP device available");
    return TLR_ERR_DEVICE;
  }
  tlr_status st = h->stage.init(h->mem, (size_t)16 << 20);
  if (st == TLR_OK) st = h->mem.get((void**)&h->d_info, 256);
  if (st == TLR_OK && hipMemsetAsync(h->d_info, 0, 256, h->stream) != hipSuccess) {
    set_error("hipMemsetAsync of the status word failed");
    st = TLR_ERR_DEVICE;
  }
  if (st == TLR_OK) st = h->mem.get((void**)&h->Ad, sizeof(double) * (size_t)h->nb * m * m);
  if (st != TLR_OK) {
    tlr_destroy(h);
    return st;
  }
  h->a_rank.assign((size_t)h->nb * h->nb, 0);
  h->a_off.assign((size_t)h->nb * h->nb, -1);
  free_factor(h);
  *out = h;
  return TLR_OK;
}

namespace tlr {
tlr_status alloc_input(Handle* h, const int* ranks) {
  const int nb = h->nb, m = h->m;
  long long cols = 0;
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < i; ++j) {
      const int r = ranks ? ranks[(size_t)i * nb + j] : 0;
      h->a_rank[(size_t)i * nb + j] = r;
      h->a_off[(size_t)i * nb + j] = cols;
      cols += r;
    }
  h->a_cols = cols;
  TLR_TRY(h->mem.get((void**)&h->UA, sizeof(double) * (size_t)std::max(cols, 1LL) * m));
  TLR_TRY(h->mem.get((void**)&h->VA, sizeof(double) * (size_t)std::max(cols, 1LL) * m));
  TLR_HIP(hipMemsetAsync(h->UA, 0, sizeof(double) * (size_t)std::max(cols, 1LL) * m, h->stream));
  TLR_HIP(hipMemsetAsync(h->VA, 0, sizeof(double) * (size_t)std::max(cols, 1LL) * m, h->stream));
  // identity diagonal tiles
  TLR_HIP(hipMemsetAsync(h->Ad, 0, sizeof(double) * (size_t)nb * m * m, h->stream));
  for (int k = 0; k < nb; ++k)
    TLR_HIP(launch_copy_shift(h->diagA(k), h->diagA(k), m, m, 1.0, h->stream));
  return h->sync();
}
}  // namespace tlr

extern "C" {

tlr_status tlr_create(long long N, int m, const int* ranks, const tlr_allocator* allocator,
                      void* stream, tlr_matrix_t* out) {
  Handle* h = nullptr;
  TLR_TRY(new_handle(N, m, allocator, stream, &h));
  if (ranks) {
    for (int i = 0; i < h->nb; ++i)
      for (int j = 0; j < i; ++j) {
        const int r = ranks[(size_t)i * h->nb + j];
        if (r < 0 || r > m) {
          tlr_destroy(h);
          set_error("rank of tile (%d, %d) is %d, must be in 0..m", i, j, r);
          return TLR_ERR_ARG;
        }
      }
  }
  tlr_status st = alloc_input(h, ranks);
  if (st != TLR_OK) {
    tlr_destroy(h);
    return st;
  }
  *out = h;
  return TLR_OK;
}

static hipMemcpyKind kind_in(int on_device) {
  return on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}

tlr_status tlr_set_diag(tlr_matrix_t A, int k, const double* D, int ld, int on_device) {
  TLR_ARG(A && D, "NULL argument");
  TLR_ARG(k >= 0 && k < A->nb, "tile index %d out of range", k);
  const int nr = A->nreal(k);
  TLR_ARG(ld >= nr, "leading dimension too small");
  TLR_HIP(hipMemcpy2DAsync(A->diagA(k), sizeof(double) * A->m, D, sizeof(double) * ld,
                           sizeof(double) * nr, nr, kind_in(on_device), A->stream));
  A->norm_a = 0.0;
  A->a_fro.clear();
  return A->sync();
}

tlr_status tlr_set_tile(tlr_matrix_t A, int i, int j, const double* U, const double* V, int ld,
                        int on_device) {
  TLR_ARG(A, "NULL handle");
  TLR_ARG(i >= 0 && i < A->nb && j >= 0 && j < i, "tile (%d, %d) is not strictly lower", i, j);
  const int r = A->ar(i, j);
  if (r == 0) return TLR_OK;
  TLR_ARG(U && V, "NULL factor");
  const int m = A->m;
  TLR_ARG(ld >= A->nreal(i) && ld >= A->nreal(j), "leading dimension too small");
  TLR_HIP(hipMemsetAsync(A->ua(i, j), 0, sizeof(double) * (size_t)m * r, A->stream));
  TLR_HIP(hipMemsetAsync(A->va(i, j), 0, sizeof(double) * (size_t)m * r, A->stream));
  TLR_HIP(hipMemcpy2DAsync(A->ua(i, j), sizeof(double) * m, U, sizeof(double) * ld,
                           sizeof(double) * A->nreal(i), r, kind_in(on_device), A->stream));
  TLR_HIP(hipMemcpy2DAsync(A->va(i, j), sizeof(double) * m, V, sizeof(double) * ld,
                           sizeof(double) * A->nreal(j), r, kind_in(on_device), A->stream));
  A->norm_a = 0.0;
  A->a_fro.clear();
  A->a_orth = false;
  return A->sync();
}

tlr_status tlr_compress(const double* Adense, long long lda, long long N, int m, double eps,
                        const tlr_opts* opts, const tlr_allocator* allocator, void* stream,
                        tlr_matrix_t* out) {
  TLR_ARG(Adense, "NULL matrix");
  TLR_ARG(lda >= N, "lda < N");
  TLR_ARG(eps > 0.0 && std::isfinite(eps), "eps must be positive");
  tlr_opts o;
  TLR_TRY(check_opts(opts, &o));
  Handle* h = nullptr;
  TLR_TRY(new_handle(N, m, allocator, stream, &h));
  tlr_status st = compress(h, Adense, lda, nullptr, 0, -1, 1.0, 0.0, eps, o);
  if (st != TLR_OK) {
    tlr_destroy(h);
    return st;
  }
  *out = h;
  return TLR_OK;
}

tlr_status tlr_compress_kernel(const double* points, int dim, long long N, int kernel, double ell,
                               double diag_add, int m, double eps, const tlr_opts* opts,
                               const tlr_allocator* allocator, void* stream, tlr_matrix_t* out) {
  TLR_ARG(points, "NULL points");
  TLR_ARG(dim >= 1 && dim <= 3, "dim must be 1..3");
  TLR_ARG(kernel == TLR_KERNEL_EXP || kernel == TLR_KERNEL_MATERN15, "unknown kernel");
  TLR_ARG(ell > 0.0 && std::isfinite(ell), "ell must be positive");
  TLR_ARG(std::isfinite(diag_add), "diag_add must be finite");
  TLR_ARG(eps > 0.0 && std::isfinite(eps), "eps must be positive");
  tlr_opts o;
  TLR_TRY(check_opts(opts, &o));
  Handle* h = nullptr;
  TLR_TRY(new_handle(N, m, allocator, stream, &h));
  tlr_status st = compress(h, nullptr, 0, points, dim, kernel, ell, diag_add, eps, o);
  if (st != TLR_OK) {
    tlr_destroy(h);
    return st;
  }
  *out = h;
  return TLR_OK;
}

static double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

static tlr_status factor_entry(tlr_matrix_t A, double eps, const tlr_opts* opts, tlr_stats* stats,
                               bool ldl, double* D, bool piv = false) {
  const auto t0 = std::chrono::steady_clock::now();
  TLR_ARG(A, "NULL handle");
  TLR_ARG(eps > 0.0 && std::isfinite(eps), "eps must be positive");
  tlr_opts o;
  TLR_TRY(check_opts(opts, &o));
  TLR_ARG(!piv || o.precision == TLR_FP64, "the pivoted Cholesky samples in FP64 (opts.precision)");
  TLR_ARG(!(o.flags & TLR_FLAG_SCHUR_COMP) || (!ldl && !piv),
          "Schur compensation (TLR_FLAG_SCHUR_COMP) applies to the unpivoted Cholesky");

  if (stats) std::memset(stats, 0, sizeof *stats);
  tlr_status st = factorize(A, eps, o, stats, ldl, piv);
  // Section 5.1: a shift s <= eps of the diagonal keeps the perturbation
  // below the compression threshold; with auto_shift a Cholesky that lost
  // definiteness without a shift is repeated once with s = tau
  if (st == TLR_ERR_NOT_SPD && !ldl && o.auto_shift && o.shift == 0.0) {
    o.shift = -1.0;
    st = factorize(A, eps, o, stats, ldl, piv);
    if (stats) stats->shift_retries = 1;
  }
  if (st == TLR_OK && ldl && D) {
    TLR_HIP(hipMemcpyAsync(D, A->Dv, sizeof(double) * A->N, hipMemcpyDeviceToDevice, A->stream));
    st = A->sync();
  }
  if (st < 0 && st != TLR_ERR_ARG) A->factored = 0;
  if (stats) stats->t_total = ms_since(t0);
  return st;
}

tlr_status tlr_potrf(tlr_matrix_t A, double eps, const tlr_opts* opts, tlr_stats* stats,
                     void* stream) {
  if (A) A->stream = A->mem.stream = (hipStream_t)stream;
  return factor_entry(A, eps, opts, stats, false, nullptr);
}

tlr_status tlr_potrf_pivoted(tlr_matrix_t A, double eps, const tlr_opts* opts, int* perm,
                             tlr_stats* stats, void* stream) {
  if (A) A->stream = A->mem.stream = (hipStream_t)stream;
  const tlr_status st = factor_entry(A, eps, opts, stats, false, nullptr, true);
  if (st == TLR_OK && perm)
    for (int t = 0; t < A->nb; ++t) perm[t] = A->fperm[t];
  return st;
}

tlr_status tlr_get_perm(tlr_matrix_t A, int* perm) {
  TLR_ARG(A && perm, "NULL argument");
  if (!A->factored) {
    set_error("the handle holds no factor");
    return TLR_ERR_STATE;
  }
  for (int t = 0; t < A->nb; ++t) perm[t] = A->fperm.empty() ? t : A->fperm[t];
  return TLR_OK;
}

tlr_status tlr_ldlt(tlr_matrix_t A, double eps, const tlr_opts* opts, double* D, tlr_stats* stats,
                    void* stream) {
  if (A) A->stream = A->mem.stream = (hipStream_t)stream;
  return factor_entry(A, eps, opts, stats, true, D);
}

static tlr_status batched_entry(int count, tlr_matrix_t* A, bool ldl, const double* eps,
                                const tlr_opts* opts, double* const* D, tlr_stats* stats,
                                void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  TLR_ARG(count > 0 && A && eps, "empty batch");
  for (int i = 0; i < count; ++i) {
    TLR_ARG(A[i], "NULL handle in the batch");
    TLR_ARG(eps[i] > 0.0 && std::isfinite(eps[i]), "eps of matrix %d must be positive", i);
    for (int j = 0; j < i; ++j) TLR_ARG(A[j] != A[i], "a handle appears twice in the batch");
    TLR_ARG(A[i]->dev == A[0]->dev, "the batch spans several devices");
  }
  tlr_opts o;
  TLR_TRY(check_opts(opts, &o));
  TLR_ARG(!o.auto_shift, "opts.auto_shift is not supported by the batched factorizations");
  TLR_ARG(!(o.flags & TLR_FLAG_SCHUR_COMP),
          "Schur compensation is not supported by the batched factorizations");
  if (stats) std::memset(stats, 0, sizeof(tlr_stats) * count);
  for (int i = 0; i < count; ++i) A[i]->stream = A[i]->mem.stream = (hipStream_t)stream;
  tlr_status st = factorize_batch(A, count, eps, o, stats, ldl);
  if (ldl && D)
    for (int i = 0; i < count; ++i)
      if (D[i] && A[i]->factored == 2)
        TLR_HIP(hipMemcpyAsync(D[i], A[i]->Dv, sizeof(double) * A[i]->N, hipMemcpyDeviceToDevice,
                               A[i]->stream));
  if (ldl && D) {
    const tlr_status s2 = A[0]->sync();
    if (st == TLR_OK) st = s2;
  }
  if (st < 0 && st != TLR_ERR_NOT_SPD && st != TLR_ERR_ZERO_PIVOT && st != TLR_ERR_ARG)
    for (int i = 0; i < count; ++i) A[i]->factored = 0;
  if (stats) {
    const double t = ms_since(t0);
    for (int i = 0; i < count; ++i) stats[i].t_total = t;
  }
  return st;
}

tlr_status tlr_factor_batched(int count, tlr_matrix_t* A, int ldl, double eps,
                              const tlr_opts* opts, double* const* D, tlr_stats* stats,
                              void* stream) {
  TLR_ARG(count > 0 && A, "empty batch");
  const std::vector<double> e(count, eps);
  return batched_entry(count, A, ldl != 0, e.data(), opts, D, stats, stream);
}

tlr_status tlr_potrf_batched(int count, tlr_matrix_t* A, const double* eps, const tlr_opts* opts,
                             tlr_stats* stats, void* stream) {
  return batched_entry(count, A, false, eps, opts, nullptr, stats, stream);
}

tlr_status tlr_ldlt_batched(int count, tlr_matrix_t* A, const double* eps, const tlr_opts* opts,
                            double* const* D, tlr_stats* stats, void* stream) {
  return batched_entry(count, A, true, eps, opts, D, stats, stream);
}

tlr_status tlr_solve(tlr_matrix_t A, int nrhs, double* B, long long ldb, void* stream) {
  TLR_ARG(A && B, "NULL argument");
  TLR_ARG(nrhs >= 0, "nrhs must be non-negative");
  TLR_ARG(ldb >= A->N, "ldb < N");
  if (!A->factored) {
    set_error("the handle holds no factor");
    return TLR_ERR_STATE;
  }
  if (nrhs == 0) return TLR_OK;
  A->stream = A->mem.stream = (hipStream_t)stream;
  return solve(A, nrhs, B, ldb);
}

tlr_status tlr_matvec(tlr_matrix_t A, int nrhs, const double* X, long long ldx, double* Y,
                      long long ldy, void* stream) {
  TLR_ARG(A && X && Y, "NULL argument");
  TLR_ARG(nrhs >= 0, "nrhs must be non-negative");
  TLR_ARG(ldx >= A->N && ldy >= A->N, "leading dimension < N");
  if (nrhs == 0) return TLR_OK;
  A->stream = A->mem.stream = (hipStream_t)stream;
  TLR_TRY(matvec(A, nrhs, X, ldx, Y, ldy));
  return A->sync();
}

tlr_status tlr_recompress(tlr_matrix_t A, int which, double tau, void* stream) {
  TLR_ARG(A, "NULL handle");
  TLR_ARG(which == TLR_INPUT || which == TLR_FACTOR, "which must be TLR_INPUT or TLR_FACTOR");
  TLR_ARG(std::isfinite(tau) && tau >= 0.0, "tau must be finite and non-negative");
  if (which == TLR_FACTOR && !A->factored) {
    set_error("the handle holds no factor");
    return TLR_ERR_STATE;
  }
  if (which == TLR_INPUT && !A->a_orth) {
    set_error("the input tiles were set with tlr_set_tile: their U need not be orthonormal");
    return TLR_ERR_STATE;
  }
  A->stream = A->mem.stream = (hipStream_t)stream;
  return recompress(A, which, tau);
}

tlr_status tlr_get_info(tlr_matrix_t A, long long* N, int* m, int* nb, int* factored) {
  TLR_ARG(A, "NULL handle");
  if (N) *N = A->N;
  if (m) *m = A->m;
  if (nb) *nb = A->nb;
  if (factored) *factored = A->factored;
  return TLR_OK;
}

tlr_status tlr_get_ranks(tlr_matrix_t A, int which, int* ranks) {
  TLR_ARG(A && ranks, "NULL argument");
  TLR_ARG(which == TLR_INPUT || which == TLR_FACTOR, "which must be TLR_INPUT or TLR_FACTOR");
  if (which == TLR_FACTOR && !A->factored) {
    set_error("the handle holds no factor");
    return TLR_ERR_STATE;
  }
  const auto& src = which == TLR_INPUT ? A->a_rank : A->l_rank;
  std::copy(src.begin(), src.end(), ranks);
  return TLR_OK;
}

tlr_status tlr_get_offsets(tlr_matrix_t A, int which, long long* offsets) {
  TLR_ARG(A && offsets, "NULL argument");
  TLR_ARG(which == TLR_INPUT || which == TLR_FACTOR, "which must be TLR_INPUT or TLR_FACTOR");
  if (which == TLR_FACTOR && !A->factored) {
    set_error("the handle holds no factor");
    return TLR_ERR_STATE;
  }
  const auto& src = which == TLR_INPUT ? A->a_off : A->l_off;
  for (int i = 0; i < A->nb; ++i)
    for (int j = 0; j < A->nb; ++j) offsets[(size_t)i * A->nb + j] = j < i ? src[(size_t)i * A->nb + j] : -1;
  return TLR_OK;
}

tlr_status tlr_get_tile(tlr_matrix_t A, int which, int i, int j, double* U, double* V, int ld) {
  TLR_ARG(A, "NULL handle");
  TLR_ARG(which == TLR_INPUT || which == TLR_FACTOR, "which must be TLR_INPUT or TLR_FACTOR");
  TLR_ARG(i >= 0 && i < A->nb && j >= 0 && j < i, "tile (%d, %d) is not strictly lower", i, j);
  TLR_ARG(ld >= A->m, "ld < m");
  if (which == TLR_FACTOR && !A->factored) {
    set_error("the handle holds no factor");
    return TLR_ERR_STATE;
  }
  const int r = which == TLR_INPUT ? A->ar(i, j) : A->lr(i, j);
  if (r == 0) return TLR_OK;
  TLR_ARG(U && V, "NULL output");
  const double* su = which == TLR_INPUT ? A->ua(i, j) : A->ul(i, j);
  const double* sv = which == TLR_INPUT ? A->va(i, j) : A->vl(i, j);
  TLR_HIP(hipMemcpy2D(U, sizeof(double) * ld, su, sizeof(double) * A->m, sizeof(double) * A->m, r,
                      hipMemcpyDeviceToHost));
  TLR_HIP(hipMemcpy2D(V, sizeof(double) * ld, sv, sizeof(double) * A->m, sizeof(double) * A->m, r,
                      hipMemcpyDeviceToHost));
  return TLR_OK;
}

tlr_status tlr_get_diag(tlr_matrix_t A, int which, int k, double* D, int ld) {
  TLR_ARG(A && D, "NULL argument");
  TLR_ARG(which == TLR_INPUT || which == TLR_FACTOR, "which must be TLR_INPUT or TLR_FACTOR");
  TLR_ARG(k >= 0 && k < A->nb, "tile index out of range");
  TLR_ARG(ld >= A->m, "ld < m");
  if (which == TLR_FACTOR && !A->factored) {
    set_error("the handle holds no factor");
    return TLR_ERR_STATE;
  }
  const double* src = which == TLR_INPUT ? A->diagA(k) : A->diagL(k);
  TLR_HIP(hipMemcpy2D(D, sizeof(double) * ld, src, sizeof(double) * A->m, sizeof(double) * A->m,
                      A->m, hipMemcpyDeviceToHost));
  return TLR_OK;
}

tlr_status tlr_get_pivots(tlr_matrix_t A, double* d) {
  TLR_ARG(A && d, "NULL argument");
  if (A->factored != 2) {
    set_error("the handle holds no LDL^T factor");
    return TLR_ERR_STATE;
  }
  TLR_HIP(hipMemcpy(d, A->Dv, sizeof(double) * (size_t)A->nb * A->m, hipMemcpyDeviceToHost));
  return TLR_OK;
}

tlr_status tlr_get_sort_order(tlr_matrix_t A, int k, int* rows) {
  TLR_ARG(A && rows, "NULL argument");
  TLR_ARG(k >= 0 && k < A->nb, "column %d out of range", k);
  if (!A->factored || (int)A->sort_log.size() != A->nb) {
    set_error("the handle holds no factor");
    return TLR_ERR_STATE;
  }
  const std::vector<int>& o = A->sort_log[k];
  std::copy(o.begin(), o.end(), rows);
  return TLR_OK;
}

tlr_status tlr_destroy(tlr_matrix_t A) {
  if (!A) return TLR_OK;
  A->worker.reset();
  (void)hipStreamSynchronize(A->stream);
  free_factor(A);
  Mem& mem = A->mem;
  mem.put(A->Ad);
  mem.put(A->Ld);
  mem.put(A->Li);
  mem.put(A->Dv);
  mem.put(A->UA);
  mem.put(A->VA);
  mem.put(A->d_info);
  if (A->side) (void)hipStreamSynchronize(A->side);
  A->ws.release_all(mem);
  A->dg.destroy(mem);
  A->stage.release(mem);
  A->release_host();
  if (A->ev_fork) (void)hipEventDestroy(A->ev_fork);
  if (A->ev_join) (void)hipEventDestroy(A->ev_join);
  if (A->ev_gnext) (void)hipEventDestroy(A->ev_gnext);
  if (A->side) (void)hipStreamDestroy(A->side);
  delete A;
  return TLR_OK;
}

}  // extern "C"
