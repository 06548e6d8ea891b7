// Batched ARA loop with device-side dynamic batching (see ara_engine.h).
#include "ara_engine.h"

namespace tlr {

static size_t al(size_t n) { return (n + 63) & ~(size_t)63; }

tlr_status ara_slots(Handle* h, const AraConfig& c, int n, AraSlots* s) {
  Work& w = h->ws;
  const int m = c.m, bs = c.bs;
  const int nrb = gram_row_blocks(m);
  s->n = n;
  s->m = m;
  s->bs = bs;
  s->qstride = (size_t)m * (c.qcap + bs);
  const size_t nn = n > 0 ? (size_t)n : 1;
  TLR_TRY(w.Y.ensure(h->mem, sizeof(double) * nn * m * bs));
  TLR_TRY(w.C.ensure(h->mem, sizeof(double) * nn * m * bs));
  const bool fresh_q = w.Q.cap < sizeof(double) * nn * s->qstride;
  TLR_TRY(w.Q.ensure(h->mem, sizeof(double) * nn * s->qstride));
  if (fresh_q) TLR_HIP(hipMemsetAsync(w.Q.p, 0, w.Q.cap, h->stream));
  TLR_TRY(w.part.ensure(h->mem, sizeof(double) * nn * nrb * bs * bs * 2));
  const size_t nint = 4 + 2 * nn + al(nn) + al(nn * (bs + 1)) + al(nn) + 64;
  TLR_TRY(w.ints.ensure(h->mem, sizeof(int) * nint));
  s->Y = w.Y.as<double>();
  s->C = w.C.as<double>();
  s->Q = w.Q.as<double>();
  s->part = w.part.as<double>();
  int* ip = w.ints.as<int>();
  s->counts = ip;
  ip += 4;
  s->act = ip;
  ip += nn;
  s->qv = ip;
  ip += nn;
  s->flag = ip;
  ip += al(nn);
  s->piv = ip;
  ip += al(nn * (bs + 1));
  s->waiting = ip;
  return TLR_OK;
}

tlr_status ara_run(Handle* h, const AraConfig& c, const AraSlots& s, const std::vector<int>& order,
                   const SampleFn& sample, AraResult* res, bool* info_abort) {
  const int n = (int)order.size();
  const int m = c.m, bs = c.bs;
  const int nrb = gram_row_blocks(m);
  const int s_max = c.s_max > 0 ? (c.s_max < n ? c.s_max : n) : n;
  res->q.assign(n, 0);
  res->iters.assign(n, 0);
  res->flops_paper_orth.assign(n, 0.0);
  if (info_abort) *info_abort = false;
  if (n == 0) return TLR_OK;

  Work& w = h->ws;
  TLR_TRY(w.omega.ensure(h->mem, sizeof(double) * (size_t)m * bs));
  double* omega = w.omega.as<double>();

  // initial active list and waiting list (slots in sorted order)
  std::vector<int> act(order.begin(), order.begin() + s_max);
  std::vector<int> waiting(order.begin() + s_max, order.end());
  {
    // q = 0 and flag = 0 for all slots
    TLR_HIP(hipMemsetAsync(s.qv, 0, sizeof(int) * n, h->stream));
    TLR_HIP(hipMemsetAsync(s.flag, 0, sizeof(int) * n, h->stream));
    int hdr[2] = {s_max, 0};
    void* tmp = nullptr;
    TLR_TRY(h->stage.upload(h, act.data(), sizeof(int) * act.size(), &tmp));
    TLR_HIP(hipMemcpyAsync(s.act, tmp, sizeof(int) * act.size(), hipMemcpyDeviceToDevice, h->stream));
    if (!waiting.empty()) {
      TLR_TRY(h->stage.upload(h, waiting.data(), sizeof(int) * waiting.size(), &tmp));
      TLR_HIP(hipMemcpyAsync(s.waiting, tmp, sizeof(int) * waiting.size(), hipMemcpyDeviceToDevice,
                             h->stream));
    }
    TLR_TRY(h->stage.upload(h, hdr, sizeof hdr, &tmp));
    TLR_HIP(hipMemcpyAsync(s.counts, tmp, sizeof hdr, hipMemcpyDeviceToDevice, h->stream));
  }
  std::vector<int>& q = res->q;

  // read-back block: counts[2], status word, pad, act[ns], q[ns], laid out for
  // the slot capacity ns >= n
  const int ns = s.n;
  if (n > ns) {
    set_error("ARA batch of %d tiles exceeds the %d workspace slots", n, ns);
    return TLR_ERR_STATE;
  }
  int* pinned = nullptr;
  TLR_TRY(h->pinned_ints(4 + 2 * (size_t)ns, &pinned));

  unsigned t = 0;
  bool first = true;
  while (!act.empty()) {
    const int na = (int)act.size();
    Plan plan(h);
    const unsigned tt = t;
    plan.launch([=]() { return launch_randn(omega, m, bs, m, c.seed, c.stream_id, tt, 0, h->stream); });
    TLR_TRY(sample(act, omega, plan));

    // block Gram-Schmidt, pass 1: Y -= Q (Q^T Y)
    {
      GemmBatch c1(true, false);
      SegBatch c2;
      for (int sl : act)
        if (q[sl] > 0) {
          c1.add(q[sl], bs, m, s.q(sl), m, s.y(sl), m, s.c(sl), m, -1.0, 0.0);
          c2.add(m, bs, s.q(sl), m, s.c(sl), m, q[sl], nullptr, 1, nullptr, 1, 0, s.y(sl), m, 1.0);
        }
      plan.gemm(c1);
      plan.seg(c2);
    }
    std::vector<OrthDesc> od(na);
    for (int a = 0; a < na; ++a) {
      const int sl = act[a];
      od[a] = OrthDesc{s.y(sl), s.q(sl), q[sl], s.qv + sl, s.flag + sl,
                       s.part + (size_t)sl * nrb * bs * bs * 2, s.piv + (size_t)sl * (bs + 1)};
    }
    const size_t ood = plan.stage(od.data(), sizeof(OrthDesc) * na);
    hipStream_t st = h->stream;
    const double tau2 = c.tau * c.tau;
    const int r_min = c.r_min, qcap = c.qcap;
    plan.launch(ood, [=](const char* p) { return launch_gram_dd((const OrthDesc*)p, na, m, bs, 1, st); });
    plan.launch(ood, [=](const char* p) {
      return launch_orth_step((const OrthDesc*)p, na, m, bs, 1, tau2, r_min, qcap, st);
    });
    // pass 2 on the new columns X = Q[:, qold : qold + bs]
    {
      GemmBatch c1(true, false);
      SegBatch c2;
      for (int sl : act)
        if (q[sl] > 0) {
          double* X = s.q(sl) + (size_t)q[sl] * m;
          c1.add(q[sl], bs, m, s.q(sl), m, X, m, s.c(sl), m, -1.0, 0.0);
          c2.add(m, bs, s.q(sl), m, s.c(sl), m, q[sl], nullptr, 1, nullptr, 1, 0, X, m, 1.0);
        }
      plan.gemm(c1);
      plan.seg(c2);
    }
    plan.launch(ood, [=](const char* p) { return launch_gram_dd((const OrthDesc*)p, na, m, bs, 2, st); });
    plan.launch(ood, [=](const char* p) {
      return launch_orth_step((const OrthDesc*)p, na, m, bs, 2, tau2, r_min, qcap, st);
    });
    // convergence flags -> compaction and refill on the device
    const int nwait = (int)waiting.size(), smax = s_max;
    int* info = h->d_info;
    plan.launch([=]() { return launch_compact(s.act, s.counts, s.flag, s.waiting, nwait, smax, info, st); });
    TLR_TRY(plan.run());
    res->flops += plan.flops;
    for (int sl : act) {
      // two Gram matrices, pivoted factor, two projections and the R^{-1} products
      const double qq = q[sl];
      const double orth = 2.0 * (4.0 * m * qq * bs + 3.0 * m * (double)bs * bs);
      res->flops_paper_orth[sl] += orth;
      res->flops += orth;
      res->iters[sl] += 1;
    }
    TLR_HIP(hipMemcpyAsync(pinned, s.counts, sizeof(int) * (4 + 2 * (size_t)ns),
                           hipMemcpyDeviceToHost, h->stream));
    TLR_TRY(h->sync_main());
    const int cnt = pinned[0];
    if (cnt < 0 || cnt > n) {
      set_error("ARA compaction returned an invalid active count %d", cnt);
      return TLR_ERR_DEVICE;
    }
    if (first && info_abort && pinned[2] != 0) {
      *info_abort = true;
      return TLR_OK;
    }
    first = false;
    act.assign(pinned + 4, pinned + 4 + cnt);
    for (int i = 0; i < n; ++i) q[i] = pinned[4 + ns + i];
    ++t;
    res->launches += 1;
    if ((long long)t > (long long)n * (c.qcap + 1) + 1) {
      set_error("ARA did not converge within %u iterations", t);
      return TLR_ERR_DEVICE;
    }
  }
  return TLR_OK;
}

}  // namespace tlr
