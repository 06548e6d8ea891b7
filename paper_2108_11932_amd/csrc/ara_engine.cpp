// Device-driven batched ARA loop with dynamic batching (see ara_engine.h).
#include "ara_engine.h"

#include <algorithm>
#include <chrono>
#include <cstring>

namespace tlr {

static size_t al(size_t n) { return (n + 63) & ~(size_t)63; }

tlr_status ara_slots(Handle* h, const AraConfig& c, int n, AraSlots* s) {
  Work& w = h->ws;
  const int m = c.m, bs = c.bs_max();
  const int nstrip = (m + 15) / 16;
  s->n = n;
  s->m = m;
  s->bs = bs;
  s->nstrip = nstrip;
  s->qstride = (size_t)m * (c.qcap + bs);
  const size_t nn = n > 0 ? (size_t)n : 1;
  TLR_TRY(w.Y.ensure(h->mem, sizeof(double) * 2 * nn * m * bs));
  TLR_TRY(w.C.ensure(h->mem, sizeof(double) * nn * m * bs));
  const bool fresh_q = w.Q.cap < sizeof(double) * nn * s->qstride;
  TLR_TRY(w.Q.ensure(h->mem, sizeof(double) * nn * s->qstride));
  if (fresh_q) TLR_HIP(hipMemsetAsync(w.Q.p, 0, w.Q.cap, h->stream));
  const size_t pn = nn * nstrip * bs * bs * 2;
  TLR_TRY(w.part.ensure(h->mem, sizeof(double) * 3 * pn));
  const size_t nint = 8 + 13 * al(nn) + al(nn * (bs + 1)) + 64;
  TLR_TRY(w.ints.ensure(h->mem, sizeof(int) * nint));
  s->Y = w.Y.as<double>();
  s->C = w.C.as<double>();
  s->Q = w.Q.as<double>();
  s->part1 = w.part.as<double>();
  s->part2 = s->part1 + 2 * pn;
  s->yalt = (long long)(nn * m * bs);
  s->palt = (long long)pn;
  int* ip = w.ints.as<int>();
  s->counts = ip;
  ip += 8;
  s->act = ip;
  ip += al(nn);
  s->q = ip;   // q, qnew, flag, iters, qsum, ncol, f32 are contiguous (cleared together)
  ip += al(nn);
  s->qnew = ip;
  ip += al(nn);
  s->flag = ip;
  ip += al(nn);
  s->iters = ip;
  ip += al(nn);
  s->qsum = ip;
  ip += al(nn);
  s->ncol = ip;
  ip += al(nn);
  s->f32 = ip;
  ip += al(nn);
  s->qpa = ip;
  ip += al(nn);
  s->qpb = ip;
  ip += al(nn);
  s->counts2 = ip;
  ip += al(nn);
  s->act2 = ip;
  ip += al(nn);
  s->waiting = ip;   // counts .. waiting are written by one upload per run
  ip += al(nn);
  s->piv = ip;
  return TLR_OK;
}

tlr_status ara_omega(Handle* h, const AraConfig& c, double** omega) {
  TLR_TRY(h->ws.omega.ensure(h->mem, sizeof(double) * kOmegaBatch * (size_t)c.m * c.bs_max()));
  *omega = h->ws.omega.as<double>();
  return TLR_OK;
}

tlr_status ara_explicit_spec(Handle* h, const AraConfig& c, int n, const double* tiles, int ld,
                             AraSpec* spec) {
  double* omega = nullptr;
  TLR_TRY(ara_omega(h, c, &omega));
  const int m = c.m;
  spec->slots.assign(n, AraSlotDesc{});
  spec->samp_flops_col.assign(n, 2.0 * m * (double)m);
  spec->samp_bytes.assign(n, 8.0 * (double)m * m);
  spec->samp_bytes_col.assign(n, 16.0 * m);
  for (int t = 0; t < n; ++t) {
    AraSlotDesc& d = spec->slots[t];
    d.a0 = tiles + (size_t)t * ld * m;
    d.lda0 = ld;
    d.k0 = m;
    d.b0 = omega;
    d.ldb0 = m;
    d.lda1 = 1;
    d.ldb1 = 1;
  }
  return TLR_OK;
}

namespace {

// Host-side knowledge of the device state after some iteration.
struct Known {
  int iter = -1;    // the iteration whose end state this is (-1: the start)
  int count = 0;    // active slots
  int cursor = 0;   // waiting-list cursor
  int info = 0;     // status word
  int qmax = 0;     // largest basis width among the active slots
};

}  // namespace

tlr_status ara_run(Handle* h, const AraConfig& c, const AraSlots& s, const std::vector<int>& order,
                   AraSpec& spec, AraResult* res, bool* info_abort,
                   const std::function<tlr_status()>& idle) {
  const int n = (int)order.size();
  const int m = c.m, bs = c.bs_max();
  const int s_max = c.s_max > 0 ? std::min(c.s_max, n) : n;
  res->t_issue = res->t_wait = 0.0;
  res->q.assign(n, 0);
  res->iters.assign(n, 0);
  res->cols.assign(n, 0);
  res->f32.assign(n, 0);
  res->iter_bs.clear();
  res->flops_paper_orth.assign(n, 0.0);
  res->flops_slot.assign(n, 0.0);
  res->samp_bytes_slot.assign(n, 0.0);
  res->samp_flops_slot.assign(n, 0.0);
  if (info_abort) *info_abort = false;
  if (n == 0) return TLR_OK;
  if (n > s.n || (int)spec.slots.size() != n) {
    set_error("ARA batch of %d tiles does not match the %d workspace slots", n, s.n);
    return TLR_ERR_STATE;
  }
  Work& w = h->ws;
  hipStream_t st = h->stream;
  double* omega = nullptr;
  TLR_TRY(ara_omega(h, c, &omega));

  // ---- static slot descriptors, uploaded once for the run
  for (int sl = 0; sl < n; ++sl) {
    AraSlotDesc& d = spec.slots[sl];
    const double tau = spec.tau.empty() ? c.tau : spec.tau[sl];
    d.tau2 = tau * tau;
    d.y = s.y(sl);
    d.q = s.qb(sl);
    d.c = s.c(sl);
    d.part1 = s.p1(sl);
    d.part2 = s.p2(sl);
    d.piv = s.piv + (size_t)sl * (bs + 1);
  }
  // 32-row tiles of the P products of every group
  std::vector<PTile> ptiles;
  for (const PGroup& g : spec.pg)
    for (int r0 = 0; r0 < g.rk; r0 += 32) ptiles.push_back(PTile{g.uk, spec.p + g.roff, g.rk, r0});
  const size_t sbytes = sizeof(AraSlotDesc) * n;
  const size_t zbytes = sizeof(ZSeg) * spec.zseg.size();
  const size_t pbytes = sizeof(PTile) * ptiles.size();
  const size_t gbytes = sizeof(GuardDesc) * spec.guard.size();
  const size_t zoff = (sbytes + 255) & ~(size_t)255;
  const size_t poff = zoff + ((zbytes + 255) & ~(size_t)255);
  const size_t goff = poff + ((pbytes + 255) & ~(size_t)255);
  TLR_TRY(w.orth.ensure(h->mem, goff + gbytes + 256));
  char* dbase = (char*)w.orth.p;
  {
    // slot descriptors, Z pieces, P tiles and precision choices: one copy
    std::vector<char> blob(goff + gbytes);
    std::memcpy(blob.data(), spec.slots.data(), sbytes);
    if (zbytes) std::memcpy(blob.data() + zoff, spec.zseg.data(), zbytes);
    if (pbytes) std::memcpy(blob.data() + poff, ptiles.data(), pbytes);
    if (gbytes) std::memcpy(blob.data() + goff, spec.guard.data(), gbytes);
    TLR_TRY(h->stage.upload_to(h, blob.data(), blob.size(), dbase, st));
  }
  const ZSeg* dzseg = (const ZSeg*)(dbase + zoff);
  bool omega_in_slots = false;
  for (const AraSlotDesc& d : spec.slots)
    omega_in_slots = omega_in_slots || d.b0 == omega || d.b1 == omega;
  const PTile* dptiles = (const PTile*)(dbase + poff);

  // ---- initial state: active list, waiting list, cleared counters
  std::vector<int> act(order.begin(), order.begin() + s_max);
  std::vector<int> waiting(order.begin() + s_max, order.end());
  const int nwait = (int)waiting.size();
  {
    // header, active list, cleared per-slot counters and the waiting list
    // are contiguous: one copy
    const size_t wo = (size_t)(s.waiting - s.counts);
    std::vector<int> blob(wo + nwait, 0);
    blob[0] = s_max;
    std::copy(act.begin(), act.end(), blob.begin() + (s.act - s.counts));
    std::copy(waiting.begin(), waiting.end(), blob.begin() + wo);
    TLR_TRY(h->stage.upload_to(h, blob.data(), sizeof(int) * blob.size(), s.counts, st));
  }
  if (gbytes)
    TLR_HIP(launch_mixed_guard((AraSlotDesc*)dbase, (const GuardDesc*)(dbase + goff), n, s.f32, st));
  int* ring = nullptr;
  TLR_TRY(h->readback_ring(&ring));
  // per-slot results (q, qnew, flag, iters, qsum, ncol, f32: contiguous)
  const size_t stride = (size_t)(s.qnew - s.q);
  const int res_ints = (int)(7 * stride);
  int* pres = nullptr;
  TLR_TRY(h->readback_results((size_t)res_ints, &pres));

  AraDev D;
  D.slots = (const AraSlotDesc*)dbase;
  D.act = s.act;
  D.counts = s.counts;
  D.act_next = s.act2;
  D.counts_next = s.counts2;
  D.qin = s.qpa;
  D.qout = s.qpb;
  D.q = s.q;
  D.qnew = s.qnew;
  D.flag = s.flag;
  D.iters = s.iters;
  D.qsum = s.qsum;
  D.ncol = s.ncol;
  D.m = m;
  D.bs = bs;
  D.qcap = c.qcap;
  D.nstrip = s.nstrip;
  D.yoff = 0;
  D.poff = 0;
  D.skip = nullptr;
  const int p_blocks = (int)ptiles.size();
  const int bps_wa = (spec.a_max + 31) / 32;
  // split-K partial tiles of the TN products
  double* tn_scratch = nullptr;
  {
    const long long tiles = std::max((long long)p_blocks + (long long)n * bps_wa,
                                     (long long)n * ((c.qcap + 31) / 32));
    size_t need = 0;
    ara_tn_scratch(m, bs, tiles, &need);
    TLR_TRY(w.tnpart.ensure(h->mem, sizeof(double) * std::max<size_t>(need, 1)));
    tn_scratch = w.tnpart.as<double>();
  }
  int max_pieces = 0;
  for (const AraSlotDesc& d : spec.slots) max_pieces = std::max(max_pieces, d.nz);
  const int bps_z = (max_pieces + 3) / 4;
  const bool any_z = !spec.zseg.empty() && bps_z > 0 && p_blocks > 0;
  int* info = h->d_info;

  // Sampling lookahead.  Without refills (no waiting list) the active list
  // only shrinks: iteration t + 1 samples the tiles of iteration t less the
  // ones that the pass-1 Cholesky QR step of iteration t flagged as
  // converged.  So, once that step has run, the sampling of t + 1 needs
  // nothing more from iteration t, and it shares the launches of t's second
  // Gram-Schmidt pass (the first blocks of each launch sample, the others
  // orthogonalise): both run at once on one stream, and the host issues one
  // launch for two.  The samples go to the other copy of Y and of its Gram
  // partials.  A slot's samples depend only on the slot, so the result is
  // the same bit for bit as sampling at the start of each iteration.
  const bool fuse = c.overlap && nwait == 0 && !spec.events && fused_block_supported(c.bs) &&
                    (c.bs_tail <= 0 || c.bs_tail == c.bs);
  // the sampling half writes its split-K partials beside the other half's
  double* tn_scratch_s = tn_scratch;
  if (fuse) {
    TLR_TRY(w.tnpart2.ensure(h->mem, w.tnpart.cap));
    tn_scratch_s = w.tnpart2.as<double>();
  }

  Known known;
  known.count = s_max;
  std::vector<int> bs_of;   // samples of every iteration, fixed when it is sampled
  int sampled = -1;         // last iteration whose sampling is enqueued
  // the list a launch of iteration t reads: its own, except for a sampling
  // fused into iteration t - 1, which reads t - 1's (less the flagged tiles)
  auto dev_for = [&](int t, bool sampling) {
    AraDev E = D;
    E.bs = bs_of[t];
    E.yoff = (t & 1) ? s.yalt : 0;
    E.poff = (t & 1) ? s.palt : 0;
    const bool ahead = sampling && fuse && t >= 1;
    E.skip = ahead ? s.flag : nullptr;
    const int lp = (ahead ? t - 1 : t) & 1;
    E.act = lp ? s.act2 : s.act;
    E.counts = lp ? s.counts2 : s.counts;
    E.act_next = lp ? s.act : s.act2;
    E.counts_next = lp ? s.counts : s.counts2;
    E.qin = (t & 1) ? s.qpb : s.qpa;
    E.qout = (t & 1) ? s.qpa : s.qpb;
    return E;
  };
  const size_t ostride = (size_t)m * bs;
  // the test matrix of iteration t: explicit tiles read one buffer through
  // their descriptors (drawn every iteration); the sampling through P and
  // W^A draws the matrices of kOmegaBatch iterations at a time
  auto draw = [&](int t, int bst) -> tlr_status {
    if (omega_in_slots)
      TLR_HIP(launch_randn(omega, m, bst, m, c.seed, c.stream_id, (unsigned)t, 0, st));
    else if (t % kOmegaBatch == 0)
      TLR_HIP(launch_randn_iters(omega, m, ostride, c.bs, bs, c.seed, c.stream_id, (unsigned)t,
                                 kOmegaBatch, 0, st));
    return TLR_OK;
  };
  auto omega_of = [&](int t) {
    return omega_in_slots ? omega : omega + (size_t)(t % kOmegaBatch) * ostride;
  };
  // the sampling of iteration t alone, with launch bounds derived from
  // `known`: the active count can only grow by refills, a basis by at most
  // bs per iteration
  auto enqueue_sampling = [&](int t) -> tlr_status {
    bs_of.push_back(c.bs_for(t, known.count));
    res->iter_bs.push_back(bs_of[t]);
    sampled = t;
    const AraDev E = dev_for(t, true);
    const int cb = (known.cursor >= nwait) ? known.count : s_max;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (spec.events) {
      TLR_HIP(hipEventCreate(&e0));
      TLR_HIP(hipEventCreate(&e1));
      spec.events->push_back({e0, e1});
    }
    TLR_TRY(draw(t, E.bs));
    if (p_blocks > 0 || bps_wa > 0)
      TLR_HIP(launch_ara_tn(E, 0, omega_of(t), dptiles, p_blocks, spec.ldp, cb, bps_wa, tn_scratch,
                            st));
    if (any_z) TLR_HIP(launch_ara_z(E, dzseg, spec.p, spec.ldp, cb, bps_z, st));
    TLR_HIP(launch_ara_seg(E, 0, cb, st, c.strip, e0, e1));
    return TLR_OK;
  };
  // iteration j: its samples (unless drawn with the previous iteration),
  // both Gram-Schmidt passes with the Cholesky QR steps, the compaction;
  // with `fuse`, the sampling of j + 1 inside the second pass
  auto enqueue = [&](int j) -> tlr_status {
    if (spec.pt) TLR_HIP(spec.pt->mark(TLR_PHASE_SAMPLE, st));
    if (sampled < j) TLR_TRY(enqueue_sampling(j));
    const AraDev E = dev_for(j, false);
    const int cb = (known.cursor >= nwait) ? known.count : s_max;
    const int qb = std::min(c.qcap, known.qmax + bs * (j - known.iter - 1));
    const int bps_q = (qb + 31) / 32;
    if (spec.pt) TLR_HIP(spec.pt->mark(TLR_PHASE_ORTH, st));
    if (bps_q > 0) {
      TLR_HIP(launch_ara_tn(E, 1, nullptr, nullptr, 0, 0, cb, bps_q, tn_scratch, st));
      TLR_HIP(launch_ara_seg(E, 1, cb, st));
    }
    TLR_HIP(launch_orth_step(E, 1, c.r_min, cb, st));
    const int bn = c.bs_for(j + 1, known.count);
    bool compacted = false;
    if (fuse && bn == E.bs) {
      bs_of.push_back(bn);
      res->iter_bs.push_back(bn);
      sampled = j + 1;
      const AraDev S = dev_for(j + 1, true);
      TLR_TRY(draw(j + 1, bn));
      TLR_HIP(launch_fused_tn(S, omega_of(j + 1), dptiles, p_blocks, spec.ldp,
                              (p_blocks > 0 || bps_wa > 0) ? cb : 0, bps_wa, tn_scratch_s, E,
                              bps_q > 0 ? cb : 0, bps_q, tn_scratch, s.waiting, nwait, s_max,
                              info, ring + 8 * (j & 1), pres, res_ints, st));
      compacted = true;
      TLR_HIP(launch_fused_z_seg(S, dzseg, spec.p, spec.ldp, any_z ? cb : 0, bps_z, E,
                                 bps_q > 0 ? cb : 0, st));
      TLR_HIP(launch_fused_seg_orth(S, cb, c.strip, E, cb, c.r_min, st));
    } else {
      if (bps_q > 0) {
        TLR_HIP(launch_ara_tn(E, 2, nullptr, nullptr, 0, 0, cb, bps_q, tn_scratch, st));
        TLR_HIP(launch_ara_seg(E, 2, cb, st));
      }
      TLR_HIP(launch_orth_step(E, 2, c.r_min, cb, st));
    }
    if (spec.pt) TLR_HIP(spec.pt->mark(TLR_PHASE_BATCH, st));
    if (!compacted)
      TLR_HIP(launch_ara_compact(E, s.waiting, nwait, s_max, info, ring + 8 * (j & 1), pres,
                                 res_ints, st));
    TLR_HIP(hipEventRecord(h->ev_rb[j & 1], st));
    return TLR_OK;
  };

  const long long limit = (long long)n * (c.qcap + 1) + 1;
  using clk = std::chrono::steady_clock;
  auto ms = [](clk::time_point a, clk::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
  };
  int enq = 0;
  auto t0 = clk::now();
  TLR_TRY(enqueue(0));
  for (;;) {
    // keep one iteration queued ahead of the state being read back
    TLR_TRY(enqueue(enq + 1));
    ++enq;
    auto t1 = clk::now();
    res->t_issue += ms(t0, t1);
    if (idle) TLR_TRY(idle());
    const int j = known.iter + 1;
    t1 = clk::now();
    TLR_HIP(hipEventSynchronize(h->ev_rb[j & 1]));
    t0 = clk::now();
    res->t_wait += ms(t1, t0);
    const int* r = ring + 8 * (j & 1);
    known.iter = j;
    known.count = r[0];
    known.cursor = r[1];
    known.info = r[2];
    known.qmax = r[3];
    if (known.count < 0 || known.count > n) {
      set_error("ARA compaction returned an invalid active count %d", known.count);
      return TLR_ERR_DEVICE;
    }
    if (j == 0 && info_abort && known.info != 0) {
      *info_abort = true;
      break;
    }
    if (known.count == 0) break;
    if (j > limit) {
      set_error("ARA did not converge within %d iterations", j);
      return TLR_ERR_DEVICE;
    }
  }
  res->launches = known.iter + 1;
  // the iteration enqueued past the last active one found nothing to do;
  // its (empty) sampling launch stays in the timed set, as it runs
  // ---- results: basis widths, iteration counts, summed widths
  // the compaction that emptied the active list left the results in pinned
  // memory (its iteration's event has completed); the iteration queued
  // behind it finds nothing to do and is not waited for.  After an abort
  // they are read back from the device.
  std::vector<int> back(7 * stride);
  if (known.count == 0) {
    std::memcpy(back.data(), pres, sizeof(int) * back.size());
  } else {
    TLR_HIP(hipMemcpyAsync(back.data(), s.q, sizeof(int) * back.size(), hipMemcpyDeviceToHost, st));
    TLR_TRY(h->sync_main());
  }
  const int* bq = back.data();
  const int* bit = back.data() + 3 * stride;
  const int* bqs = back.data() + 4 * stride;
  const int* bnc = back.data() + 5 * stride;
  const int* bf32 = back.data() + 6 * stride;
  const double b0 = c.bs, b1 = c.bs_tail > 0 ? c.bs_tail : c.bs;
  for (int sl = 0; sl < n; ++sl) {
    res->q[sl] = bq[sl];
    res->iters[sl] = bit[sl];
    res->cols[sl] = bnc[sl];
    res->f32[sl] = bf32[sl];
    // samples drawn, and the sum of their squares per iteration (every
    // iteration draws b0 or b1 samples)
    const double it = bit[sl], qs = bqs[sl], cols = bnc[sl];
    const double n1 = b1 != b0 ? (cols - b0 * it) / (b1 - b0) : 0.0;
    const double b2 = (it - n1) * b0 * b0 + n1 * b1 * b1;
    // two Gram-Schmidt passes, each a projection and an update, plus the
    // Gram matrices and the triangular solves of the Cholesky QR steps
    // (qs: the sum over iterations of samples times prior basis width)
    const double orth = 8.0 * m * qs + 6.0 * m * b2;
    res->flops_paper_orth[sl] = orth;
    res->flops_slot[sl] = orth + cols * spec.samp_flops_col[sl];
    const double sb = (bf32[sl] == 1 && !spec.samp_bytes32.empty())   ? spec.samp_bytes32[sl]
                      : (bf32[sl] == 2 && !spec.samp_bytes16.empty()) ? spec.samp_bytes16[sl]
                                                                       : spec.samp_bytes[sl];
    res->samp_bytes_slot[sl] = it * sb + cols * spec.samp_bytes_col[sl];
    res->samp_flops_slot[sl] = cols * spec.samp_flops_col[sl];
    res->flops += res->flops_slot[sl];
    res->samp_bytes += res->samp_bytes_slot[sl];
    res->samp_flops += res->samp_flops_slot[sl];
  }
  return TLR_OK;
}

}  // namespace tlr
