// Runtime pieces of the TLR library: error text, device memory, descriptor
// staging, batched GEMM launches and the dense tile operations.
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

tlr_status Staging::upload(Handle* h, const void* data, size_t bytes, void** dptr) {
  const size_t need = (bytes + 255) & ~(size_t)255;
  if (used + need > cap) {
    TLR_TRY(h->sync());
    if (need > cap) {
      Mem& mem = h->mem;
      release(mem);
      TLR_TRY(init(mem, need * 2));
    }
  }
  std::memcpy(host + used, data, bytes);
  TLR_HIP(hipMemcpyAsync(dev + used, host + used, bytes, hipMemcpyHostToDevice, h->stream));
  *dptr = dev + used;
  used += need;
  return TLR_OK;
}

}  // namespace tlr

tlr_status tlr_matrix_s::sync() {
  TLR_HIP(hipStreamSynchronize(stream));
  stage.used = 0;
  return TLR_OK;
}

namespace tlr {

// ---------------------------------------------------------------- GEMM batch
tlr_status GemmBatch::run(Handle* h) {
  if (d.empty()) return TLR_OK;
  int maxn = 0;
  for (const auto& g : d) maxn = g.N > maxn ? g.N : maxn;
  const int bn = gemm_tile_n(maxn);
  std::vector<BlockMap> map;
  map.reserve(d.size() * 4);
  for (size_t i = 0; i < d.size(); ++i) {
    const int tiles = ((d[i].M + 63) / 64) * ((d[i].N + bn - 1) / bn);
    for (int t = 0; t < tiles; ++t) map.push_back(BlockMap{(int)i, t});
  }
  void* dd = nullptr;
  void* dm = nullptr;
  TLR_TRY(h->stage.upload(h, d.data(), d.size() * sizeof(GemmDesc), &dd));
  TLR_TRY(h->stage.upload(h, map.data(), map.size() * sizeof(BlockMap), &dm));
  TLR_HIP(launch_gemm_batched((const GemmDesc*)dd, (const BlockMap*)dm, (int)map.size(), ta, tb,
                              bn, h->stream));
  return TLR_OK;
}

// ---------------------------------------------------------------- dense tiles
static constexpr int NBP = 64;

tlr_status dense_potrf(Handle* h, double* A, int lda, int m, int row_base) {
  for (int p0 = 0; p0 < m; p0 += NBP) {
    const int w = m - p0 < NBP ? m - p0 : NBP;
    TLR_HIP(launch_potrf_panel(A, lda, m, p0, w, h->d_info, row_base, h->stream));
    const int rem = m - p0 - w;
    if (rem > 0) {
      GemmBatch g(false, true);
      const double* l21 = A + (p0 + w) + (size_t)p0 * lda;
      g.add(rem, rem, w, l21, lda, l21, lda, A + (p0 + w) + (size_t)(p0 + w) * lda, lda, -1.0, 1.0);
      TLR_TRY(g.run(h));
    }
  }
  TLR_HIP(launch_zero_upper(A, lda, m, h->stream));
  return TLR_OK;
}

tlr_status dense_ldlt(Handle* h, double* A, int lda, int m, double* d, int row_base) {
  Work& w = h->ws;
  TLR_TRY(w.tol.ensure(h->mem, sizeof(double)));
  TLR_TRY(w.dscale.ensure(h->mem, sizeof(double) * (size_t)m * NBP));
  TLR_HIP(launch_pivot_tol(A, lda, m, w.tol.as<double>(), h->stream));
  double* W = w.dscale.as<double>();
  for (int p0 = 0; p0 < m; p0 += NBP) {
    const int wd = m - p0 < NBP ? m - p0 : NBP;
    TLR_HIP(launch_ldlt_panel(A, lda, m, p0, wd, d, W, m, h->d_info, row_base, w.tol.as<double>(),
                              h->stream));
    const int rem = m - p0 - wd;
    if (rem > 0) {
      GemmBatch g(false, true);
      const double* l21 = A + (p0 + wd) + (size_t)p0 * lda;
      g.add(rem, rem, wd, W, m, l21, lda, A + (p0 + wd) + (size_t)(p0 + wd) * lda, lda, -1.0, 1.0);
      TLR_TRY(g.run(h));
    }
  }
  TLR_HIP(launch_zero_upper(A, lda, m, h->stream));
  return TLR_OK;
}

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
