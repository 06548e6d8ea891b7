// Runtime pieces of the TLR library: error text, device memory, descriptor
// staging, batched GEMM launches and the dense tile operations.
#include <algorithm>
#include <cstdarg>

#include "host.h"

namespace tlr {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

const char* last_error() { return g_err.c_str(); }

// ---------------------------------------------------------------- memory
tlr_status Mem::get(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~(size_t)255;
  if (custom) {
    *p = alloc.alloc(alloc.ctx, bytes, (void*)stream);
  } else {
    if (hipMalloc(p, bytes) != hipSuccess) *p = nullptr;
  }
  if (!*p) {
    (void)hipGetLastError();
    set_error("device allocation of %zu bytes failed", bytes);
    return TLR_ERR_OOM;
  }
  live += bytes;
  return TLR_OK;
}

void Mem::put(void* p) {
  if (!p) return;
  if (custom)
    alloc.free(alloc.ctx, p, (void*)stream);
  else
    (void)hipFree(p);
}

tlr_status DevBuf::ensure(Mem& mem, size_t bytes) {
  if (bytes <= cap && p) return TLR_OK;
  size_t want = bytes + bytes / 2 + 4096;
  mem.put(p);
  p = nullptr;
  cap = 0;
  TLR_TRY(mem.get(&p, want));
  cap = want;
  return TLR_OK;
}

void DevBuf::release(Mem& mem) {
  mem.put(p);
  p = nullptr;
  cap = 0;
}

// ---------------------------------------------------------------- staging
tlr_status Staging::init(Mem& mem, size_t bytes) {
  if (hipHostMalloc((void**)&host, bytes, hipHostMallocDefault) != hipSuccess) {
    host = nullptr;
    set_error("pinned host allocation of %zu bytes failed", bytes);
    return TLR_ERR_OOM;
  }
  void* d = nullptr;
  tlr_status st = mem.get(&d, bytes);
  if (st != TLR_OK) {
    (void)hipHostFree(host);
    host = nullptr;
    return st;
  }
  dev = (char*)d;
  cap = bytes;
  used = 0;
  return TLR_OK;
}

void Staging::release(Mem& mem) {
  if (host) (void)hipHostFree(host);
  mem.put(dev);
  host = dev = nullptr;
  cap = used = 0;
}

tlr_status Staging::upload(Handle* h, const void* data, size_t bytes, void** dptr,
                           hipStream_t s) {
  const size_t need = (bytes + 255) & ~(size_t)255;
  if (used + need > cap) {
    TLR_TRY(h->sync());
    if (need > cap) {
      if (fixed) {
        set_error("%zu bytes of launch descriptors exceed the %zu-byte staging ring", need, cap);
        return TLR_ERR_ARG;
      }
      Mem& mem = h->mem;
      release(mem);
      TLR_TRY(init(mem, need * 2));
    }
  }
  std::memcpy(host + used, data, bytes);
  TLR_HIP(hipMemcpyAsync(dev + used, host + used, bytes, hipMemcpyHostToDevice,
                         s ? s : h->stream));
  *dptr = dev + used;
  used += need;
  return TLR_OK;
}

tlr_status Staging::upload_to(Handle* h, const void* data, size_t bytes, void* dst,
                              hipStream_t s) {
  if (bytes == 0) return TLR_OK;
  const size_t need = (bytes + 255) & ~(size_t)255;
  if (used + need > cap) {
    TLR_TRY(h->sync());
    if (need > cap) {
      if (fixed) {
        set_error("%zu bytes of launch descriptors exceed the %zu-byte staging ring", need, cap);
        return TLR_ERR_ARG;
      }
      Mem& mem = h->mem;
      release(mem);
      TLR_TRY(init(mem, need * 2));
    }
  }
  // the host bytes stay untouched until the ring wraps, which waits for
  // the queued copies first
  std::memcpy(host + used, data, bytes);
  TLR_HIP(hipMemcpyAsync(dst, host + used, bytes, hipMemcpyHostToDevice, s ? s : h->stream));
  used += need;
  return TLR_OK;
}

}  // namespace tlr

namespace tlr {

SideWorker::SideWorker(int dev) : th_([this, dev]() { loop(dev); }) {}

SideWorker::~SideWorker() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  th_.join();
}

void SideWorker::submit(std::function<tlr_status()> f) {
  {
    std::lock_guard<std::mutex> lk(mu_);
    q_.push_back(std::move(f));
  }
  cv_.notify_one();
}

tlr_status SideWorker::wait() {
  std::unique_lock<std::mutex> lk(mu_);
  idle_cv_.wait(lk, [this]() { return q_.empty() && !busy_; });
  const tlr_status e = err_;
  err_ = TLR_OK;
  return e;
}

void SideWorker::loop(int dev) {
  (void)hipSetDevice(dev);
  std::unique_lock<std::mutex> lk(mu_);
  for (;;) {
    cv_.wait(lk, [this]() { return stop_ || !q_.empty(); });
    if (q_.empty()) return;   // stop requested and nothing left
    std::function<tlr_status()> f = std::move(q_.front());
    q_.pop_front();
    busy_ = true;
    lk.unlock();
    const tlr_status e = f();
    lk.lock();
    busy_ = false;
    if (err_ == TLR_OK && e != TLR_OK) err_ = e;
    if (q_.empty()) idle_cv_.notify_all();
  }
}

}  // namespace tlr

tlr_status tlr_matrix_s::sync() {
  TLR_HIP(hipStreamSynchronize(stream));
  if (side) TLR_HIP(hipStreamSynchronize(side));
  stage.used = 0;
  return TLR_OK;
}

tlr_status tlr_matrix_s::sync_main() {
  TLR_HIP(hipStreamSynchronize(stream));
  return TLR_OK;
}

tlr_status tlr_matrix_s::init_streams() {
  if (!side) {
    TLR_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    TLR_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
    TLR_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
    TLR_HIP(hipEventCreateWithFlags(&ev_gnext, hipEventDisableTiming));
  }
  return TLR_OK;
}

tlr_status tlr_matrix_s::readback_ring(int** p) {
  if (!pin_ring) {
    if (hipHostMalloc((void**)&pin_ring, sizeof(int) * 16, hipHostMallocDefault) != hipSuccess) {
      pin_ring = nullptr;
      tlr::set_error("pinned host allocation failed");
      return TLR_ERR_OOM;
    }
  }
  for (int i = 0; i < 2; ++i)
    if (!ev_rb[i]) TLR_HIP(hipEventCreateWithFlags(&ev_rb[i], hipEventDisableTiming));
  *p = pin_ring;
  return TLR_OK;
}

tlr_status tlr_matrix_s::readback_results(size_t n, int** p) {
  if (n > pin_res_n) {
    if (pin_res) (void)hipHostFree(pin_res);
    pin_res = nullptr;
    pin_res_n = 0;
    if (hipHostMalloc((void**)&pin_res, sizeof(int) * n, hipHostMallocDefault) != hipSuccess) {
      pin_res = nullptr;
      tlr::set_error("pinned host allocation failed");
      return TLR_ERR_OOM;
    }
    pin_res_n = n;
  }
  *p = pin_res;
  return TLR_OK;
}

void tlr_matrix_s::release_host() {
  pt_main.destroy();
  pt_side.destroy();
  if (pin_norm) (void)hipHostFree(pin_norm);
  if (pin_ring) (void)hipHostFree(pin_ring);
  if (pin_res) (void)hipHostFree(pin_res);
  pin_res = nullptr;
  pin_res_n = 0;
  pin_norm = nullptr;
  pin_ring = nullptr;
  pin_norm_n = 0;
  for (hipEvent_t& e : ev_rb) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
}

tlr_status tlr_matrix_s::pinned_norms(size_t n, double** p) {
  if (n > pin_norm_n) {
    if (pin_norm) (void)hipHostFree(pin_norm);
    pin_norm = nullptr;
    pin_norm_n = 0;
    if (hipHostMalloc((void**)&pin_norm, sizeof(double) * n, hipHostMallocDefault) != hipSuccess) {
      pin_norm = nullptr;
      tlr::set_error("pinned host allocation failed");
      return TLR_ERR_OOM;
    }
    pin_norm_n = n;
  }
  *p = pin_norm;
  return TLR_OK;
}

namespace tlr {

// ---------------------------------------------------------------- sortRanks
void sort_ranks(const int* ranks, const int* rows, int n, int* idx) {
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx, idx + n, [&](int a, int b) {
    if (ranks[a] != ranks[b]) return ranks[a] > ranks[b];
    if (rows[a] != rows[b]) return rows[a] < rows[b];
    return a < b;
  });
}

// ---------------------------------------------------------------- phase timing
hipError_t PhaseTimer::mark(int phase, hipStream_t s) {
  if (!on) return hipSuccess;
  if (n == ev.size()) {
    hipEvent_t e = nullptr;
    const hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    ev.push_back(e);
  }
  ph.push_back(phase);
  return hipEventRecord(ev[n++], s);
}

tlr_status PhaseTimer::collect(double* t) {
  for (size_t i = 0; i + 1 < n; ++i) {
    if (ph[i] < 0 || ph[i] >= TLR_NPHASE) continue;
    float ms = 0.f;
    TLR_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
    t[ph[i]] += ms;
  }
  n = 0;
  ph.clear();
  return TLR_OK;
}

void PhaseTimer::destroy() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  ev.clear();
  ph.clear();
  n = 0;
}

// ---------------------------------------------------------------- GEMM batch
tlr_status GemmBatch::run(Handle* h, hipStream_t s) {
  Plan p(h, s);
  p.gemm(*this);
  return p.run();
}


// ---------------------------------------------------------------- plans
Plan::Plan(Handle* h_, hipStream_t s_) : h(h_), s(s_ ? s_ : h_->stream) {}

size_t Plan::stage(const void* p, size_t n) {
  const size_t off = blob.size();
  const size_t pad = (n + 255) & ~(size_t)255;
  blob.resize(off + pad);
  if (n) std::memcpy(blob.data() + off, p, n);
  return off;
}

void Plan::launch(size_t off, std::function<hipError_t(const char*)> f) {
  steps.push_back([off, f](const char* base) { return f(base + off); });
}

void Plan::launch(std::function<hipError_t()> f) {
  steps.push_back([f](const char*) { return f(); });
}

// Block map of the problems `idx` of a batch with tiles TM x TN.
static void build_map(const std::vector<GemmDesc>& d, const std::vector<int>& idx, int TM, int TN,
                      std::vector<BlockMap>* map) {
  for (int i : idx) {
    const int tm = (d[i].M + TM - 1) / TM, tn = (d[i].N + TN - 1) / TN;
    for (int t = 0; t < tm * tn; ++t) {
      if ((d[i].flags & GEMM_LOWER_C) && (t / tm) * TN >= (t % tm) * TM + TM) continue;
      map->push_back(BlockMap{i, t});
    }
  }
}

void Plan::gemm(const GemmBatch& b) {
  if (b.d.empty()) return;
  const bool ta = b.ta, tb = b.tb;
  hipStream_t st = s;
  // Transposed-A problems that meet the LDS-streamed kernel's requirements
  // run on it (coalesced loads), oriented so that the operand with more
  // columns is A (a product with more columns than rows is formed
  // transposed and stored back transposed); the others run on the
  // register-tiled kernels.  Each kernel takes classes by tile shape, so
  // that small problems (most of the per-tile products G_ij, U_ij^T Q_i of
  // the method) do not run on large, mostly idle tiles.
  std::vector<GemmDesc> dv = b.d;
  std::vector<int> l16, l64n, l64w, small, large;
  long long n64n = 0, n64w = 0;   // workgroups of the narrow / wide classes on large tiles
  int maxn = 0;
  for (size_t i = 0; i < dv.size(); ++i) {
    GemmDesc& d = dv[i];
    if (ta && !tb && gemm_tn_lds_ok(d)) {
      if (d.N > d.M && d.N > 16) {
        std::swap(d.A, d.B);
        std::swap(d.lda, d.ldb);
        std::swap(d.M, d.N);
        d.flags |= GEMM_STORE_T;
      }
      if (d.M <= 16 && d.N <= 16) {
        l16.push_back((int)i);
      } else if (d.N <= 16) {
        l64n.push_back((int)i);
        n64n += (d.M + 63) / 64;
      } else {
        l64w.push_back((int)i);
        n64w += (long long)((d.M + 63) / 64) * ((d.N + 31) / 32);
      }
      continue;
    }
    const bool sm = ta && !tb && d.M <= 16 && d.N <= 16;
    (sm ? small : large).push_back((int)i);
    if (!sm) maxn = std::max(maxn, d.N);
  }
  // A class too small to give every CU a large tile runs on 16 x 16 tiles
  // instead: a workgroup's chunks are sequential, so with few workgroups
  // the launch takes the latency of one large tile's K loop.
  constexpr long long kFill = 256;
  if (n64n < kFill) {
    l16.insert(l16.end(), l64n.begin(), l64n.end());
    l64n.clear();
  }
  if (n64w < kFill) {
    l16.insert(l16.end(), l64w.begin(), l64w.end());
    l64w.clear();
  }
  const size_t od = stage(dv.data(), dv.size() * sizeof(GemmDesc));
  auto push = [&](const std::vector<int>& idx, int tm, int tn, bool lds, int bn) {
    if (idx.empty()) return;
    std::vector<BlockMap> map;
    build_map(dv, idx, tm, tn, &map);
    int maxk = 0;
    for (int i : idx) maxk = std::max(maxk, dv[i].K);
    const size_t om = stage(map.data(), map.size() * sizeof(BlockMap));
    const int nblk = (int)map.size();
    steps.push_back([=](const char* base) {
      const GemmDesc* pd = (const GemmDesc*)(base + od);
      const BlockMap* pm = (const BlockMap*)(base + om);
      return lds ? launch_gemm_tn_lds(pd, pm, nblk, tm, tn, st)
                 : launch_gemm_batched(pd, pm, nblk, ta, tb, bn, maxk, st);
    });
  };
  push(l16, 16, 16, true, 0);
  push(l64n, 64, 16, true, 0);
  push(l64w, 64, 32, true, 0);
  push(small, 16, 16, false, 0);
  if (!large.empty()) {
    int TM = 64, bn = 16;
    gemm_tile_shape(ta, tb, maxn, &TM, &bn);
    // One long product with few output tiles (the triangular solve with
    // L_kk^{-1}, the U_k* term of the projection: ~160 tiles of 64 x 64 and
    // K ~ 1000) leaves a third of the CUs idle and each busy one on a long
    // K loop: its K range is cut into slices of 64-multiples whose partial
    // products go to the split buffer and are added in a fixed order.
    int S = 1, kc = 0;
    if (splitk && !ta && large.size() == 1) {
      const GemmDesc& d = dv[large[0]];
      const long long tiles = (long long)((d.M + TM - 1) / TM) * ((d.N + bn - 1) / bn);
      if ((d.flags & ~GEMM_TRIL_A) == 0 && tiles < kFill && d.K >= 256) {
        S = (int)std::min<long long>(std::min<long long>((2 * kFill + tiles - 1) / tiles, d.K / 128), 8);
        kc = ((d.K + S - 1) / S + 63) / 64 * 64;
        S = (d.K + kc - 1) / kc;
        if ((size_t)S * d.M * d.N * sizeof(double) > splitk->cap) S = 1;
      }
    }
    if (S >= 2) {
      const GemmDesc d = dv[large[0]];
      double* part = splitk->as<double>();
      std::vector<GemmDesc> sd;
      for (int s = 0; s < S; ++s) {
        GemmDesc e = d;
        const int k0 = s * kc;
        e.A = d.A + (size_t)k0 * d.lda;
        e.B = tb ? d.B + (size_t)k0 * d.ldb : d.B + k0;
        e.K = std::min(d.K, k0 + kc) - k0;
        e.C = part + (size_t)s * d.M * d.N;
        e.ldc = d.M;
        e.alpha = 1.0;
        e.beta = 0.0;
        e.koff = k0;
        sd.push_back(e);
      }
      std::vector<int> idx(S);
      for (int s = 0; s < S; ++s) idx[s] = s;
      std::vector<BlockMap> map;
      build_map(sd, idx, TM, bn, &map);
      const size_t osd = stage(sd.data(), sd.size() * sizeof(GemmDesc));
      const size_t om = stage(map.data(), map.size() * sizeof(BlockMap));
      const int nblk = (int)map.size();
      const int maxk = kc;
      steps.push_back([=](const char* base) {
        return launch_gemm_batched((const GemmDesc*)(base + osd), (const BlockMap*)(base + om), nblk,
                                   ta, tb, bn, maxk, st);
      });
      steps.push_back([=](const char*) {
        return launch_splitk_sum(d.C, d.ldc, d.M, d.N, part, S, d.alpha, d.beta, st);
      });
    } else {
      push(large, TM, bn, false, bn);
    }
  }
  flops += b.flops;
}

tlr_status Plan::run() { return run_some(steps.size()); }

tlr_status Plan::run_some(size_t max_steps) {
  if (!started) {
    started = true;
    base = nullptr;
    if (!blob.empty()) {
      void* dp = nullptr;
      if (persist) {
        if (persist->cap < blob.size()) {
          TLR_TRY(h->sync());   // the old buffer may still be read by queued work
          TLR_TRY(persist->ensure(h->mem, blob.size() + blob.size() / 2));
        }
        TLR_TRY(h->stage.upload_to(h, blob.data(), blob.size(), persist->p, s));
        dp = persist->p;
      } else {
        TLR_TRY(h->stage.upload(h, blob.data(), blob.size(), &dp, s));
      }
      base = (const char*)dp;
    }
  }
  const size_t end = std::min(steps.size(), cursor + max_steps);
  for (; cursor < end; ++cursor) TLR_HIP(steps[cursor](base));
  if (cursor == steps.size()) {
    steps.clear();
    blob.clear();
    cursor = 0;
    started = false;
  }
  return TLR_OK;
}

// ---------------------------------------------------------------- dense tiles
static constexpr int NBP = 64;

// Off-diagonal blocks of the inverse of a lower triangular m x m matrix L
// whose diagonal blocks (diag_block_size() wide) are already inverted in Linv:
// [A 0; B C]^{-1} = [A^{-1} 0; -C^{-1} B A^{-1}  C^{-1}], applied bottom-up
// over a binary split of the block rows; nodes of one level are batched.
// W is an m x m workspace.
static void inverse_assemble(Plan& plan, const double* L, int ldl, int m, double* Linv, double* W) {
  struct Node {
    int lo, mid, hi;
  };
  std::vector<std::vector<Node>> levels;
  std::vector<std::pair<std::pair<int, int>, int>> stack = {{{0, m}, 0}};
  while (!stack.empty()) {
    auto it = stack.back();
    stack.pop_back();
    const int lo = it.first.first, hi = it.first.second, dep = it.second;
    const int nd = diag_block_size();
    if (hi - lo <= nd) continue;
    const int nblk = (hi - lo + nd - 1) / nd;
    const int mid = lo + ((nblk + 1) / 2) * nd;
    if ((int)levels.size() <= dep) levels.resize(dep + 1);
    levels[dep].push_back(Node{lo, mid, hi});
    stack.push_back({{lo, mid}, dep + 1});
    stack.push_back({{mid, hi}, dep + 1});
  }
  for (int dep = (int)levels.size() - 1; dep >= 0; --dep) {
    GemmBatch g1(false, false), g2(false, false);
    for (const Node& n : levels[dep]) {
      const int a = n.mid - n.lo, c = n.hi - n.mid;
      // W = B A^{-1}
      g1.add(c, a, a, L + n.mid + (size_t)n.lo * ldl, ldl, Linv + n.lo + (size_t)n.lo * m, m,
             W + n.mid + (size_t)n.lo * m, m, 1.0, 0.0);
      // X21 = -C^{-1} W
      g2.add(c, a, c, Linv + n.mid + (size_t)n.mid * m, m, W + n.mid + (size_t)n.lo * m, m,
             Linv + n.mid + (size_t)n.lo * m, m, -1.0, 0.0, GEMM_TRIL_A);
    }
    plan.gemm(g1);
    plan.gemm(g2);
  }
}

// The launches of the blocked factorization of the m x m tile A (ld lda)
// and of the assembly of Linv, on the workspace W (m x m), the device word
// tol and the status word info.  modify: modified Cholesky, its pivot floor
// already in tol (Cholesky only); LDL^T forms its pivot tolerance in tol.
static void factor_launches(Plan& plan, bool chol, double* A, int lda, int m, double* d,
                            int row_base, double* Linv, double* W, double* tol, int* info,
                            bool modify) {
  hipStream_t s = plan.s;
  plan.launch([=]() { return launch_fill(Linv, (long long)m * m, 0.0, s); });
  if (!chol) plan.launch([=]() { return launch_pivot_tol(A, lda, m, tol, s); });
  const double* tolk = (chol && !modify) ? nullptr : tol;
  const int nd = diag_block_size();
  // W holds the panels below the diagonal blocks until the last step (A's
  // panel columns are read while they are formed)
  plan.launch([=]() { return launch_potrf_first(chol, A, lda, m, Linv, m, d, info, row_base, tolk, s); });
  for (int p0 = 0; p0 + nd < m; p0 += nd)
    plan.launch([=]() {
      return launch_potrf_step(chol, A, lda, m, p0, W, m, Linv, m, d, info, row_base, tolk, s);
    });
  plan.launch([=]() { return launch_tri_finish(A, lda, W, m, m, s); });
  inverse_assemble(plan, A, lda, m, Linv, W);
}

tlr_status dense_factor(Handle* h, Plan& plan, bool chol, double* A, int lda, int m, double* d,
                        int row_base, double* Linv, double mod_delta) {
  Work& w = h->ws;
  hipStream_t s = plan.s;
  const size_t need = sizeof(double) * (size_t)m * m;
  const size_t ntol = sizeof(double) * kPivotTolDoubles;
  if (w.dW.cap < need || w.dtol.cap < ntol) {
    TLR_HIP(hipStreamSynchronize(s));
    TLR_TRY(w.dW.ensure(h->mem, need));
    TLR_TRY(w.dtol.ensure(h->mem, ntol));
  }
  double* tol = w.dtol.as<double>();
  // modified Cholesky: the pivot floor for the panel kernels
  const bool modify = chol && mod_delta > 0.0;
  if (modify) plan.launch([=]() { return launch_fill(tol, 1, mod_delta, s); });
  factor_launches(plan, chol, A, lda, m, d, row_base, Linv, w.dW.as<double>(), tol, h->d_info,
                  modify);
  return TLR_OK;
}

void DiagGraph::destroy(Mem& mem) {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  exec = nullptr;
  graph = nullptr;
  if (cap) (void)hipStreamDestroy(cap);
  cap = nullptr;
  DevBuf* bufs[] = {&A, &Linv, &W, &D, &info, &tol, &desc};
  for (DevBuf* b : bufs) b->release(mem);
  m = 0;
  mode = -1;
}

tlr_status diag_graph(Handle* h, int m, int mode, DiagGraph** out) {
  DiagGraph& g = h->dg;
  *out = &g;
  if (g.exec && g.m == m && g.mode == mode) return TLR_OK;
  // the buffers of a previous graph may still be read by queued work
  TLR_TRY(h->sync());
  g.destroy(h->mem);
  const size_t mm = sizeof(double) * (size_t)m * m;
  TLR_TRY(g.A.ensure(h->mem, mm));
  TLR_TRY(g.Linv.ensure(h->mem, mm));
  TLR_TRY(g.W.ensure(h->mem, mm));
  TLR_TRY(g.D.ensure(h->mem, sizeof(double) * (size_t)m));
  TLR_TRY(g.info.ensure(h->mem, 256));
  TLR_TRY(g.tol.ensure(h->mem, sizeof(double) * kPivotTolDoubles));
  TLR_HIP(hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking));
  TLR_HIP(hipMemsetAsync(g.info.p, 0, 256, g.cap));
  const bool chol = mode != 2;
  Plan plan(h, g.cap);
  plan.persist = &g.desc;
  factor_launches(plan, chol, g.A.as<double>(), m, m, chol ? nullptr : g.D.as<double>(), 0,
                  g.Linv.as<double>(), g.W.as<double>(), g.tol.as<double>(), g.info.as<int>(),
                  mode == 1);
  // the GEMM descriptors go up before the capture (the graph reads them
  // where they stay); then every launch is recorded, none executed
  TLR_TRY(plan.run_some(0));
  TLR_HIP(hipStreamSynchronize(g.cap));
  TLR_HIP(hipStreamBeginCapture(g.cap, hipStreamCaptureModeRelaxed));
  const tlr_status st = plan.run();
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(g.cap, &graph);
  if (st != TLR_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    if (st != TLR_OK) return st;
    TLR_HIP(e);
  }
  g.graph = graph;
  TLR_HIP(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
  g.m = m;
  g.mode = mode;
  return TLR_OK;
}

tlr_status dense_potrf(Handle* h, double* A, int lda, int m, int row_base, double* Linv,
                       hipStream_t s) {
  Plan plan(h, s);
  TLR_TRY(dense_factor(h, plan, true, A, lda, m, nullptr, row_base, Linv));
  return plan.run();
}

tlr_status dense_ldlt(Handle* h, double* A, int lda, int m, double* d, int row_base, double* Linv,
                      hipStream_t s) {
  Plan plan(h, s);
  TLR_TRY(dense_factor(h, plan, false, A, lda, m, d, row_base, Linv));
  return plan.run();
}

// Blocked triangular solve with the diagonal-block kernel (used by the
// kernel-level entry point).
tlr_status dense_trsm(Handle* h, const double* L, int ldl, double* B, int ldb, int m, int n,
                      bool unit, bool trans) {
  if (n <= 0) return TLR_OK;
  const int np = (m + NBP - 1) / NBP;
  for (int q = 0; q < np; ++q) {
    const int p = trans ? np - 1 - q : q;
    const int p0 = p * NBP;
    const int w = m - p0 < NBP ? m - p0 : NBP;
    TLR_HIP(launch_trsm_diag(L, ldl, B, ldb, p0, w, n, unit, trans, h->stream));
    if (!trans) {
      const int rem = m - p0 - w;
      if (rem > 0) {
        GemmBatch g(false, false);
        g.add(rem, n, w, L + (p0 + w) + (size_t)p0 * ldl, ldl, B + p0, ldb, B + p0 + w, ldb, -1.0,
              1.0);
        TLR_TRY(g.run(h));
      }
    } else if (p0 > 0) {
      GemmBatch g(true, false);
      g.add(p0, n, w, L + p0, ldl, B + p0, ldb, B, ldb, -1.0, 1.0);
      TLR_TRY(g.run(h));
    }
  }
  return TLR_OK;
}

}  // namespace tlr
