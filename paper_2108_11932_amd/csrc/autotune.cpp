// Tile-size autotuner.  The factorization time of a TLR matrix depends
// strongly on the tile size (Table 1 of the paper: a factor of two between
// tile sizes at one N, with the best size growing with N), and no formula
// picks it: each candidate is measured.  For a covariance problem the tuner
// builds the TLR input at every candidate tile size and times one
// factorization after an untimed one; the fastest candidate is remembered
// per problem class, so that a batch of many problems of similar sizes pays
// for one measurement per class.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "host.h"

namespace {

// Problem class: ceil(log2 N), dimension, kernel, threshold, and the options
// that change the work (threshold mode, precision, block size), plus the
// candidate set.
using Key = std::tuple<int, int, int, double, int, int, int, std::vector<int>>;

std::mutex g_mu;
std::map<Key, int> g_cache;

int ceil_log2(long long n) {
  int l = 0;
  while ((1LL << l) < n) ++l;
  return l;
}

}  // namespace

extern "C" {

tlr_status tlr_tune_tile(const double* points, int dim, long long N, int kernel, double ell,
                         double diag_add, double eps, const tlr_opts* opts, const int* candidates,
                         int ncand, const tlr_allocator* allocator, void* stream, int* best,
                         double* ms, int* cached) {
  using namespace tlr;
  if (!points || !candidates || !best || ncand <= 0) {
    set_error("NULL argument or empty candidate set");
    return TLR_ERR_ARG;
  }
  for (int c = 0; c < ncand; ++c)
    if (candidates[c] <= 0) {
      set_error("tile size candidates must be positive");
      return TLR_ERR_ARG;
    }
  tlr_opts o;
  if (opts)
    o = *opts;
  else
    tlr_opts_default(&o);
  const Key key{ceil_log2(N), dim, kernel, eps, o.eps_mode, o.precision, o.bs,
                std::vector<int>(candidates, candidates + ncand)};
  if (cached) *cached = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      *best = it->second;
      if (cached) *cached = 1;
      return TLR_OK;
    }
  }
  using clk = std::chrono::steady_clock;
  double best_ms = INFINITY;
  int best_m = 0;
  for (int c = 0; c < ncand; ++c) {
    const int m = candidates[c];
    double t = INFINITY;
    tlr_matrix_t h = nullptr;
    tlr_status st = tlr_compress_kernel(points, dim, N, kernel, ell, diag_add, m, eps, &o,
                                        allocator, stream, &h);
    if (st < 0 && st != TLR_ERR_ARG) return st;
    if (st == TLR_OK) {
      tlr_stats s;
      st = tlr_potrf(h, eps, &o, &s, stream);   // untimed: workspaces, code objects
      if (st == TLR_OK) {
        const auto t0 = clk::now();
        st = tlr_potrf(h, eps, &o, &s, stream);
        t = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
      }
      tlr_destroy(h);
      // a candidate that cannot be factored is not chosen; a system error
      // ends the tuning
      if (st < 0 && st != TLR_ERR_ARG) return st;
      if (st != TLR_OK) t = INFINITY;
    }
    if (ms) ms[c] = t;
    if (t < best_ms) {
      best_ms = t;
      best_m = m;
    }
  }
  if (best_m == 0) {
    set_error("no tile size candidate could be factored");
    return TLR_ERR_NOT_SPD;
  }
  *best = best_m;
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[key] = best_m;
  return TLR_OK;
}

void tlr_tune_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache.clear();
}

}  // extern "C"
