// C ABI of the individual building blocks (include/tlr_kernels.h).  Each
// call runs on a small transient context: staging, status word and stream.
#include <algorithm>
#include <memory>

#include "../../include/tlr_kernels.h"
#include "ara_engine.h"

using namespace tlr;

namespace {

struct Ctx {
  Handle h;
  tlr_status init(void* stream, int m) {
    h.stream = (hipStream_t)stream;
    h.mem.stream = h.stream;
    h.m = m;
    h.N = m;
    h.nb = 1;
    TLR_TRY(h.stage.init(h.mem, (size_t)4 << 20));
    TLR_TRY(h.mem.get((void**)&h.d_info, 256));
    TLR_HIP(hipMemsetAsync(h.d_info, 0, sizeof(int), h.stream));
    return TLR_OK;
  }
  ~Ctx() {
    (void)hipStreamSynchronize(h.stream);
    h.ws.release_all(h.mem);
    h.mem.put(h.d_info);
    h.stage.release(h.mem);
    h.release_host();
  }
  tlr_status info(int* out) {
    TLR_TRY(h.sync());
    TLR_HIP(hipMemcpy(out, h.d_info, sizeof(int), hipMemcpyDeviceToHost));
    return TLR_OK;
  }
};

}  // namespace

#define KARG(cond, msg)        \
  do {                         \
    if (!(cond)) {             \
      set_error("%s", msg);    \
      return TLR_ERR_ARG;      \
    }                          \
  } while (0)

extern "C" {

tlr_status tlrk_gemm_batched(int ta, int tb, int count, const tlrk_gemm_problem* p, void* stream) {
  KARG(count >= 0 && (count == 0 || p), "invalid batch");
  for (int i = 0; i < count; ++i) {
    KARG(p[i].M >= 0 && p[i].N >= 0 && p[i].K >= 0, "negative size");
    const int arows = ta ? p[i].K : p[i].M;
    const int brows = tb ? p[i].N : p[i].K;
    KARG(p[i].lda >= std::max(1, arows) && p[i].ldb >= std::max(1, brows) &&
             p[i].ldc >= std::max(1, p[i].M),
         "leading dimension too small");
  }
  Ctx c;
  TLR_TRY(c.init(stream, 1));
  GemmBatch g(ta != 0, tb != 0);
  for (int i = 0; i < count; ++i)
    g.add(p[i].M, p[i].N, p[i].K, p[i].A, p[i].lda, p[i].B, p[i].ldb, p[i].C, p[i].ldc, p[i].alpha,
          p[i].beta);
  TLR_TRY(g.run(&c.h));
  return c.h.sync();
}

tlr_status tlrk_potrf(int m, double* A, int lda, int* info, void* stream) {
  KARG(m > 0 && A && lda >= m && info, "invalid argument");
  Ctx c;
  TLR_TRY(c.init(stream, m));
  void* inv = nullptr;
  TLR_TRY(c.h.mem.get(&inv, sizeof(double) * (size_t)m * m));
  tlr_status st = dense_potrf(&c.h, A, lda, m, 0, (double*)inv, c.h.stream);
  if (st == TLR_OK) st = c.info(info);
  c.h.mem.put(inv);
  return st;
}

tlr_status tlrk_ldlt(int m, double* A, int lda, double* d, int* info, void* stream) {
  KARG(m > 0 && A && d && lda >= m && info, "invalid argument");
  Ctx c;
  TLR_TRY(c.init(stream, m));
  void* inv = nullptr;
  TLR_TRY(c.h.mem.get(&inv, sizeof(double) * (size_t)m * m));
  tlr_status st = dense_ldlt(&c.h, A, lda, m, d, 0, (double*)inv, c.h.stream);
  if (st == TLR_OK) st = c.info(info);
  c.h.mem.put(inv);
  return st;
}

tlr_status tlrk_trsm(int m, int n, const double* L, int ldl, double* B, int ldb, int unit, int trans,
                     void* stream) {
  KARG(m > 0 && n >= 0 && L && B && ldl >= m && ldb >= m, "invalid argument");
  Ctx c;
  TLR_TRY(c.init(stream, m));
  TLR_TRY(dense_trsm(&c.h, L, ldl, B, ldb, m, n, unit != 0, trans != 0));
  return c.h.sync();
}

tlr_status tlrk_philox(int n, unsigned long long seed, unsigned c1, unsigned c2, unsigned c3,
                       unsigned* out, void* stream) {
  KARG(n >= 0 && out, "invalid argument");
  TLR_HIP(launch_philox_raw(out, n, seed, c1, c2, c3, (hipStream_t)stream));
  TLR_HIP(hipStreamSynchronize((hipStream_t)stream));
  return TLR_OK;
}

tlr_status tlrk_randn(int rows, int cols, unsigned long long seed, unsigned k, unsigned t, unsigned s,
                      double* out, void* stream) {
  KARG(rows >= 0 && cols >= 0 && out, "invalid argument");
  TLR_HIP(launch_randn(out, rows, cols, std::max(rows, 1), seed, k, t, s, (hipStream_t)stream));
  TLR_HIP(hipStreamSynchronize((hipStream_t)stream));
  return TLR_OK;
}

tlr_status tlrk_randn_iters(int rows, int cols0, int cols1, unsigned long long seed, unsigned k,
                            unsigned t0, int nt, unsigned s, double* out, void* stream) {
  KARG(rows >= 0 && cols0 >= 0 && cols1 >= 0 && nt >= 0 && out, "invalid argument");
  const size_t stride = (size_t)rows * std::max(cols0, cols1);
  TLR_HIP(launch_randn_iters(out, rows, stride, cols0, cols1, seed, k, t0, nt, s,
                             (hipStream_t)stream));
  TLR_HIP(hipStreamSynchronize((hipStream_t)stream));
  return TLR_OK;
}

tlr_status tlrk_ara(int m, int count, const double* tiles, double tau, int bs, int r_min,
                    unsigned long long seed, double* Q, double* B, int* ranks, int* iters,
                    void* stream) {
  KARG(m > 0 && count >= 0 && tiles && Q && B && ranks && iters, "invalid argument");
  KARG(orth_block_supported(bs) && r_min >= 1 && r_min <= bs && tau > 0.0, "invalid ARA parameters");
  if (count == 0) return TLR_OK;
  Ctx c;
  TLR_TRY(c.init(stream, m));
  AraConfig cfg;
  cfg.m = m;
  cfg.bs = bs;
  cfg.qcap = m;
  cfg.tau = tau;
  cfg.r_min = r_min;
  cfg.seed = seed;
  cfg.stream_id = 0;
  AraSlots slots;
  TLR_TRY(ara_slots(&c.h, cfg, count, &slots));
  AraSpec spec;
  TLR_TRY(ara_explicit_spec(&c.h, cfg, count, tiles, m, &spec));
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  AraResult res;
  TLR_TRY(ara_run(&c.h, cfg, slots, order, spec, &res, nullptr));
  GemmBatch pb(true, false);
  std::vector<CopyDesc> cd;
  for (int b = 0; b < count; ++b) {
    ranks[b] = res.q[b];
    iters[b] = res.iters[b];
    if (res.q[b] == 0) continue;
    pb.add(m, res.q[b], m, tiles + (size_t)b * m * m, m, slots.qb(b), m, B + (size_t)b * m * m, m, 1.0,
           0.0);
    cd.push_back(CopyDesc{slots.qb(b), Q + (size_t)b * m * m, m, res.q[b], m, m});
  }
  TLR_TRY(pb.run(&c.h));
  if (!cd.empty()) {
    void* d = nullptr;
    TLR_TRY(c.h.stage.upload(&c.h, cd.data(), sizeof(CopyDesc) * cd.size(), &d));
    TLR_HIP(launch_copy_batched((const CopyDesc*)d, (int)cd.size(), m, c.h.stream));
  }
  return c.h.sync();
}

tlr_status tlrk_sort_ranks(int n, const int* ranks, const int* rows, int* order) {
  KARG(n >= 0 && (n == 0 || (ranks && rows && order)), "invalid argument");
  std::vector<int> idx(n);
  sort_ranks(ranks, rows, n, idx.data());
  for (int i = 0; i < n; ++i) order[i] = rows[idx[i]];
  return TLR_OK;
}

tlr_status tlrk_compact(int nslots, int* act, int* count, const int* flags, const int* waiting,
                        int nwaiting, int* cursor, int s_max) {
  KARG(nslots >= 0 && act && count && flags && cursor && nwaiting >= 0 && s_max >= 0,
       "invalid argument");
  KARG(*count >= 0 && *count <= nslots && *cursor >= 0 && *cursor <= nwaiting, "invalid counts");
  KARG(nwaiting == 0 || waiting, "NULL waiting list");
  for (int i = 0; i < *count; ++i) KARG(act[i] >= 0 && act[i] < nslots, "slot out of range");
  Ctx c;
  TLR_TRY(c.init(nullptr, 1));
  const size_t cap = std::max(nslots, 1) + std::max(nwaiting, 1) + std::max(s_max, 1) + 8;
  TLR_TRY(c.h.ws.ints.ensure(c.h.mem, sizeof(int) * cap));
  int* dact = c.h.ws.ints.as<int>();
  int* dcounts = dact + std::max(nslots, s_max) + 2;
  std::vector<int> hdr = {*count, *cursor};
  void* tmp = nullptr;
  if (*count > 0) {
    TLR_TRY(c.h.stage.upload(&c.h, act, sizeof(int) * *count, &tmp));
    TLR_HIP(hipMemcpyAsync(dact, tmp, sizeof(int) * *count, hipMemcpyDeviceToDevice, c.h.stream));
  }
  TLR_TRY(c.h.stage.upload(&c.h, hdr.data(), sizeof(int) * 2, &tmp));
  TLR_HIP(hipMemcpyAsync(dcounts, tmp, sizeof(int) * 2, hipMemcpyDeviceToDevice, c.h.stream));
  void* dflags = nullptr;
  void* dwait = nullptr;
  TLR_TRY(c.h.stage.upload(&c.h, flags, sizeof(int) * std::max(nslots, 1), &dflags));
  if (nwaiting > 0) TLR_TRY(c.h.stage.upload(&c.h, waiting, sizeof(int) * nwaiting, &dwait));
  TLR_HIP(launch_compact(dact, dcounts, (const int*)dflags, (const int*)dwait, nwaiting, s_max,
                         nullptr, c.h.stream));
  TLR_TRY(c.h.sync());
  int back[2];
  TLR_HIP(hipMemcpy(back, dcounts, sizeof back, hipMemcpyDeviceToHost));
  *count = back[0];
  *cursor = back[1];
  if (back[0] > 0) TLR_HIP(hipMemcpy(act, dact, sizeof(int) * back[0], hipMemcpyDeviceToHost));
  return TLR_OK;
}

}  // extern "C"
