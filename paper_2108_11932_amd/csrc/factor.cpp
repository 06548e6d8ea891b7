// Left-looking TLR Cholesky and LDL^T (Algorithms "Left Looking TLR
// Cholesky" and "Left Looking TLR LDL^T" of the paper).
//
// Storage of the factor: block row i of L keeps its low rank factors as two
// m x R_i column-major panels [U_i0 | U_i1 | ...] and [V_i0 | V_i1 | ...]
// that grow by one column block per factorization step (the row-panel
// storage the paper proposes in its conclusions).  With it, the sum over
// j < k of Eq. (1) becomes one long contraction per tile instead of k small
// products and a reduction over parallel buffers.
//
// Sampling of the Schur-complement tile S_ik = A_ik - sum_j L_ij L_kj^T
// (Eq. (2), reassociated, exact algebra):
//   G_ij  = V_ij^T V_kj                      once per column (Eq. (3): V_ij^T D_j V_kj)
//   P     = U_k*^T Omega                     once per ARA iteration (Omega shared)
//   Y_i   = U^A_ik (V^A_ik^T Omega) - U_i* [G_ij P_j]_j
// Projection B_i = S_ik^T Q_i:
//   B_i   = V^A_ik (U^A_ik^T Q_i) - U_k* [G_ij^T (U_ij^T Q_i)]_j
// where the last product is a single m x R_k x (sum_i q_i) GEMM for the whole
// column.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "ara_engine.h"

namespace tlr {

static void release_retired(Handle* h) {
  for (void* p : h->retired) h->mem.put(p);
  h->retired.clear();
}

void free_factor(Handle* h) {
  release_retired(h);
  for (double* p : h->UL) h->mem.put(p);
  for (double* p : h->VL) h->mem.put(p);
  for (float* p : h->UL32) h->mem.put(p);
  for (unsigned short* p : h->UL16) h->mem.put(p);
  h->UL.assign(h->nb, nullptr);
  h->VL.assign(h->nb, nullptr);
  h->UL32.assign(h->nb, nullptr);
  h->UL16.assign(h->nb, nullptr);
  h->R.assign(h->nb, 0);
  h->cap.assign(h->nb, 0);
  h->l_rank.assign((size_t)h->nb * h->nb, 0);
  h->l_off.assign((size_t)h->nb * h->nb, -1);
  h->sort_log.assign(h->nb, std::vector<int>());
  h->fperm.clear();
  h->spos.clear();
  h->mem.put(h->Sd);
  h->Sd = nullptr;
  h->factored = 0;
}

// Make room for `extra` more columns in block row i's panels.  The copy is
// ordered on the main stream after every queued use of the old panels (the
// diagonal-tile stream reads only rows <= k, which are never grown after
// their column); the old panels are retired rather than freed, so the queue
// is not drained.
static tlr_status grow_row(Handle* h, int i, int extra) {
  const int need = h->R[i] + extra;
  if (need <= h->cap[i]) return TLR_OK;
  // capacities in whole 32-column slices, so that the packed copies (slices
  // of 16 and 32 columns over all row blocks, one after another) hold a
  // prefix of whole slices that a larger copy extends
  int nc = std::max(need, h->cap[i] + h->cap[i] / 2 + 16);
  nc = (nc + 31) & ~31;
  const size_t prow = (size_t)16 * ((h->m + 15) / 16);   // rows of a packed copy
  void* u = nullptr;
  void* v = nullptr;
  void* u32 = nullptr;
  void* u16 = nullptr;
  tlr_status st = h->mem.get(&u, sizeof(double) * (size_t)h->m * nc);
  if (st == TLR_OK) st = h->mem.get(&v, sizeof(double) * (size_t)h->m * nc);
  if (st == TLR_OK && h->mixed >= 1) st = h->mem.get(&u32, sizeof(float) * prow * nc);
  if (st == TLR_OK && h->mixed >= 2) st = h->mem.get(&u16, sizeof(unsigned short) * prow * nc);
  if (st != TLR_OK) {
    for (void* p : {u, v, u32, u16}) h->mem.put(p);
    return st;
  }
  if (h->R[i] > 0) {
    const size_t bytes = sizeof(double) * (size_t)h->m * h->R[i];
    TLR_HIP(hipMemcpyAsync(u, h->UL[i], bytes, hipMemcpyDeviceToDevice, h->stream));
    TLR_HIP(hipMemcpyAsync(v, h->VL[i], bytes, hipMemcpyDeviceToDevice, h->stream));
    // the packed copies: every slice that holds a written column
    const size_t cols = (size_t)((h->R[i] + 31) & ~31);
    if (u32)
      TLR_HIP(hipMemcpyAsync(u32, h->UL32[i], sizeof(float) * prow * cols, hipMemcpyDeviceToDevice,
                             h->stream));
    if (u16)
      TLR_HIP(hipMemcpyAsync(u16, h->UL16[i], sizeof(unsigned short) * prow * cols,
                             hipMemcpyDeviceToDevice, h->stream));
  }
  for (void* old : {(void*)h->UL[i], (void*)h->VL[i], (void*)h->UL32[i], (void*)h->UL16[i]})
    if (old) h->retired.push_back(old);
  h->UL[i] = (double*)u;
  h->VL[i] = (double*)v;
  h->UL32[i] = (float*)u32;
  h->UL16[i] = (unsigned short*)u16;
  h->cap[i] = nc;
  return TLR_OK;
}

// ||A_ij||_F of every input tile for the mixed-precision guard: ||V||_F when
// U has orthonormal columns, else the bound ||U||_F ||V||_F.
static tlr_status input_norms(Handle* h) {
  const int nb = h->nb, m = h->m;
  std::vector<NormDesc> nd;
  std::vector<size_t> tile;
  h->a_fro.assign((size_t)nb * nb, 0.0);
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < i; ++j)
      if (h->ar(i, j) > 0) tile.push_back((size_t)i * nb + j);
  if (tile.empty()) return TLR_OK;
  const size_t n = tile.size();
  TLR_TRY(h->ws.fro.ensure(h->mem, sizeof(double) * 2 * n));
  double* out = h->ws.fro.as<double>();
  for (size_t t = 0; t < n; ++t) {
    const int i = (int)(tile[t] / nb), j = (int)(tile[t] % nb), r = h->ar(i, j);
    nd.push_back(NormDesc{h->va(i, j), m, r, m, out + 2 * t});
    nd.push_back(NormDesc{h->ua(i, j), m, r, m, out + 2 * t + 1});
  }
  void* dd = nullptr;
  TLR_TRY(h->stage.upload(h, nd.data(), sizeof(NormDesc) * nd.size(), &dd));
  TLR_HIP(launch_fro_norms((const NormDesc*)dd, (int)nd.size(), h->stream));
  std::vector<double> host(2 * n);
  TLR_TRY(h->sync());
  TLR_HIP(hipMemcpy(host.data(), out, sizeof(double) * 2 * n, hipMemcpyDeviceToHost));
  for (size_t t = 0; t < n; ++t)
    h->a_fro[tile[t]] = h->a_orth ? host[2 * t] : host[2 * t] * host[2 * t + 1];
  return TLR_OK;
}

namespace {

// One problem of a (possibly batched) factorization and its column state.
struct Prob {
  Handle* h = nullptr;
  double tau = 0.0, shift = 0.0;
  double tau_ara = 0.0;   // threshold of the ARA: tau / conv_factor
  double* pin_norm = nullptr;
  bool done = false;
  bool piv = false;   // pivoted Cholesky (Section 5.2)
  // the diagonal tiles' factorization replayed from the handle's captured
  // graph (else launched kernel by kernel)
  DiagGraph* dg = nullptr;
  double mod_delta = 0.0;   // > 0: modified Cholesky of the diagonal tiles (Section 5.1.2)
  bool schur = false;       // Schur compensation of the diagonal updates (Section 5.1.1)
  double* sch = nullptr;    // its buffers (Work::schur)
  double flops = 0.0, flops_paper = 0.0, bytes_alg = 0.0, samp_bytes = 0.0, samp_flops = 0.0;
  long long ara_iters = 0, tile_iters = 0, fp32_tile_iters = 0, bf16_tile_iters = 0;
  double t_issue = 0.0, t_wait = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  std::vector<long long> goff;
  // column k
  int Rk = 0, nrow = 0, base = 0, roff = 0;
  // G_ij of the column: blocks j < k - 1 at G + goff, the blocks of the
  // newest column j = jk = k - 1 at Gk + gkoff[i] (Cholesky), or all of
  // them at G + goff (jk = -1)
  double* G = nullptr;
  double* Gk = nullptr;
  int jk = -1;
  std::vector<long long> gkoff;
  // blocks j < k of column k + 1, formed ahead on the diagonal-tile stream
  int ahead = -1;
  double* Gnext = nullptr;
  std::vector<long long> goff_next;
  std::unique_ptr<Plan> dplan, gplan;
  bool side_pending = false;   // the side worker holds this column's launches
  PhaseTimer* pt = nullptr;    // phase marks of the (shared) main stream
  std::vector<int> order;
  const double* gptr(int i, int j) const {
    if (j == jk) {
      const long long go = gkoff[i];
      return go >= 0 ? Gk + go : Gk;
    }
    const long long go = goff[(size_t)i * h->nb + j];
    return go >= 0 ? G + go : G;
  }
};


// Set-up of one problem: factor storage, streams, thresholds, initial panel
// capacities.
// Steps of the Schur compensation's sign function.  First the odd quintic
// x <- a x + b x^3 + c x^5 (a, b, c = 3.4445, -4.7750, 2.0315: slope 3.44
// at 0, [0, 1] mapped into about [0.68, 1.2]), three products per step,
// which grows an eigenvalue at relative distance delta from the threshold
// 3.44-fold per step; then Newton-Schulz x <- (3 x - x^3) / 2, two products
// per step, converging quadratically from there.  30 + 12 steps resolve
// every eigenvalue farther than ~1e-16 (relative to ||D_k - tau I||_F) from
// tau, as 100 Newton-Schulz steps alone would, with 114 products instead of
// 200.
constexpr int kSchurQuinticIters = 30, kSchurSignIters = 12;
constexpr double kQa = 3.4445, kQb = -4.7750, kQc = 2.0315;

tlr_status prob_init(Prob& p, double eps, const tlr_opts& o, bool ldl) {
  Handle* h = p.h;
  const int m = h->m, nb = h->nb;
  free_factor(h);
  if (!h->Ld) {
    void* q = nullptr;
    TLR_TRY(h->mem.get(&q, sizeof(double) * (size_t)nb * m * m));
    h->Ld = (double*)q;
  }
  if (!h->Li) {
    void* q = nullptr;
    TLR_TRY(h->mem.get(&q, sizeof(double) * (size_t)nb * m * m));
    h->Li = (double*)q;
  }
  TLR_TRY(h->init_streams());
  if (ldl && !h->Dv) {
    void* q = nullptr;
    TLR_TRY(h->mem.get(&q, sizeof(double) * (size_t)nb * m));
    h->Dv = (double*)q;
  }
  p.tau = eps;
  if (o.eps_mode == TLR_EPS_REL) {
    if (h->norm_a <= 0.0) TLR_TRY(estimate_norm(h, &h->norm_a));
    p.tau = eps * h->norm_a;
  }
  p.shift = o.shift < 0.0 ? p.tau : o.shift;
  p.tau_ara = p.tau / o.conv_factor;
  TLR_HIP(hipMemsetAsync(h->d_info, 0, 2 * sizeof(int), h->stream));
  // modified Cholesky: a diagonal tile that lost definiteness has its
  // non-positive pivots raised to the threshold
  p.mod_delta = (!ldl && (o.flags & TLR_FLAG_MODIFIED_CHOL)) ? p.tau : 0.0;
  // Schur compensation: buffers of one column, reused column after column on
  // the diagonal-tile stream
  p.schur = !ldl && !p.piv && (o.flags & TLR_FLAG_SCHUR_COMP);
  if (p.schur) {
    Work& w = h->ws;
    TLR_TRY(w.schur.ensure(h->mem, sizeof(double) * (5 * (size_t)m * m + kPivotTolDoubles)));
    p.sch = w.schur.as<double>();
  }
  p.dg = nullptr;
  if (o.flags & TLR_FLAG_DIAG_GRAPH)
    TLR_TRY(diag_graph(h, m, ldl ? 2 : (p.mod_delta > 0.0 ? 1 : 0), &p.dg));
  // mixed precision: packed FP32 (and BF16) copies of the U panels, used by
  // the tiles whose rounding in that precision stays below tau / 16 (the
  // LDL^T variant samples in FP64 throughout).  The automatic form keeps a
  // BF16 copy when the threshold is at least 1e-3 ||A||_2.
  h->mixed = 0;
  if (!ldl && o.precision == TLR_MIXED_FP32) h->mixed = 1;
  if (!ldl && o.precision == TLR_MIXED_BF16) h->mixed = 2;
  if (!ldl && o.precision == TLR_MIXED_AUTO) {
    if (h->norm_a <= 0.0) TLR_TRY(estimate_norm(h, &h->norm_a));
    h->mixed = p.tau >= 1e-3 * h->norm_a ? 2 : 1;
  }
  if (h->mixed && h->a_fro.empty()) TLR_TRY(input_norms(h));
  h->l_fro.assign((size_t)nb * nb, 0.0);
  if (h->mixed) TLR_TRY(h->pinned_norms((size_t)std::max(nb, 1), &p.pin_norm));
  // initial panel capacities from the input ranks (a large rank in A tends to
  // stay large in L, Section 4.2)
  for (int i = 1; i < nb; ++i) {
    long long sum = 0;
    for (int j = 0; j < i; ++j) sum += h->pr(i, j);
    long long c = (long long)(1.25 * sum) + 32;
    c = std::min(c, (long long)i * m);
    TLR_TRY(grow_row(h, i, (int)c));
  }
  p.goff.assign((size_t)nb * nb, -1);
  p.ahead = -1;
  p.jk = -1;
  if (p.piv) {
    // the updated diagonal tiles start as A_tt + shift I (real rows)
    void* q = nullptr;
    TLR_TRY(h->mem.get(&q, sizeof(double) * (size_t)nb * m * m));
    h->Sd = (double*)q;
    h->fperm.resize(nb);
    h->spos.resize(nb);
    for (int t = 0; t < nb; ++t) {
      h->fperm[t] = t;
      h->spos[t] = t;
      TLR_HIP(launch_copy_shift(h->diagA(t), h->Sd + (size_t)t * m * m, m, h->nreal(t), p.shift,
                                h->stream));
    }
  }
  return TLR_OK;
}

// Pivot choice of column k (Algorithm "Pivoted Left Looking TLR Cholesky",
// Section 5.2).  The updated diagonal tile S_t = A_tt - sum_{j<k} L_tj L_tj^T
// of every position t >= k receives column k - 1's product ("denseUpdates":
// S_t -= U_tj (V_tj^T V_tj) U_tj^T, lower triangle), the pivot is the
// position whose S_t has the largest Frobenius norm, the first of equal
// ones ("selectPivot"), and block rows and columns k and p trade places
// ("pivotRowColumn").  Only bookkeeping moves: the row panels (the columns
// j < k go with their rows), ranks, offsets, the updated tiles and the map
// from positions to the original blocks, through which the input tiles of
// later columns are read.
tlr_status col_pivot(Prob& p, int k) {
  Handle* h = p.h;
  const int m = h->m, nb = h->nb;
  Work& w = h->ws;
  auto S = [&](int t) { return h->Sd + (size_t)h->spos[t] * m * m; };
  Plan plan(h);
  if (k >= 1) {
    const int j = k - 1;
    long long gt = 0, wt = 0;
    std::vector<long long> go(nb, -1), wo(nb, -1);
    for (int t = k; t < nb; ++t) {
      const int r = h->lr(t, j);
      if (r == 0) continue;
      go[t] = gt;
      wo[t] = wt;
      gt += (long long)r * r;
      wt += (long long)m * r;
    }
    if (gt > 0) {
      TLR_TRY(w.Sg.ensure(h->mem, sizeof(double) * (size_t)gt));
      TLR_TRY(w.Sw.ensure(h->mem, sizeof(double) * (size_t)wt));
      double* G = w.Sg.as<double>();
      double* W = w.Sw.as<double>();
      GemmBatch g(true, false), wb(false, false), up(false, true);
      for (int t = k; t < nb; ++t) {
        const int r = h->lr(t, j);
        if (r == 0) continue;
        g.add(r, r, m, h->vl(t, j), m, h->vl(t, j), m, G + go[t], r, 1.0, 0.0);
        wb.add(m, r, r, h->ul(t, j), m, G + go[t], r, W + wo[t], m, 1.0, 0.0);
        up.add(m, m, r, W + wo[t], m, h->ul(t, j), m, S(t), m, -1.0, 1.0, GEMM_LOWER_C);
      }
      plan.gemm(g);
      plan.gemm(wb);
      plan.gemm(up);
      p.flops += g.flops + wb.flops + up.flops / 2;
    }
  }
  const int n = nb - k;
  constexpr int G = 16;
  TLR_TRY(w.Snorm.ensure(h->mem, sizeof(double) * (size_t)n * G));
  double* parts = w.Snorm.as<double>();
  std::vector<const double*> tp(n);
  for (int t = k; t < nb; ++t) tp[t - k] = S(t);
  const size_t off = plan.stage(tp.data(), sizeof(double*) * n);
  hipStream_t st = h->stream;
  plan.launch(off, [=](const char* ptr) {
    return launch_sym_fro_parts((const double* const*)ptr, n, m, m, G, parts, st);
  });
  TLR_TRY(plan.run());
  p.flops += plan.flops;
  double* pin = nullptr;
  TLR_TRY(h->pinned_norms((size_t)nb * G, &pin));
  TLR_HIP(hipMemcpyAsync(pin, parts, sizeof(double) * n * G, hipMemcpyDeviceToHost, st));
  TLR_TRY(h->sync_main());
  int best = k;
  double bmax = -1.0;
  for (int t = k; t < nb; ++t) {
    double v = 0.0;
    for (int g2 = 0; g2 < G; ++g2) v += pin[(size_t)(t - k) * G + g2];
    if (v > bmax) {
      bmax = v;
      best = t;
    }
  }
  if (best != k) {
    const int a = k, b = best;
    std::swap(h->fperm[a], h->fperm[b]);
    std::swap(h->spos[a], h->spos[b]);
    std::swap(h->UL[a], h->UL[b]);
    std::swap(h->VL[a], h->VL[b]);
    std::swap(h->UL32[a], h->UL32[b]);
    std::swap(h->UL16[a], h->UL16[b]);
    std::swap(h->R[a], h->R[b]);
    std::swap(h->cap[a], h->cap[b]);
    for (int j = 0; j < k; ++j) {
      std::swap(h->l_rank[(size_t)a * nb + j], h->l_rank[(size_t)b * nb + j]);
      std::swap(h->l_off[(size_t)a * nb + j], h->l_off[(size_t)b * nb + j]);
    }
  }
  return TLR_OK;
}

// Column k, before the ARA: G_ij = V_ij^T (D_j) V_kj, the fork of the
// diagonal-tile stream, and the sortRanks order of the column's tiles.
tlr_status col_begin(Prob& p, int k, bool ldl) {
  Handle* h = p.h;
  const int m = h->m, nb = h->nb;
  Work& w = h->ws;
  TLR_HIP(p.pt->mark(TLR_PHASE_GBLOCKS, h->stream));
  if (p.piv) TLR_TRY(col_pivot(p, k));
  p.Rk = h->R[k];
  const int Rk = p.Rk;
  // ---------------------------------------------- G_ij = V_ij^T (D_j) V_kj
  // Blocks j < k - 1 are formed ahead on the diagonal-tile stream during the
  // previous column (their panels and pivots were final), else here; the
  // blocks of the newest column j = k - 1 are formed here.  LDL^T multiplies
  // by V_kj D_j, the row panel scaled block by block.
  const bool ahead = p.ahead == k;
  p.ahead = -1;
  const double* Vk = h->VL[k];
  if (ldl && Rk > 0) {
    TLR_TRY(w.W.ensure(h->mem, sizeof(double) * (size_t)m * Rk));
    // the columns to scale: the newest block only when the others were
    // formed ahead, else the whole panel
    const int c0 = (ahead && k >= 1 && h->lr(k, k - 1) > 0) ? (int)h->lo(k, k - 1) : (ahead ? Rk : 0);
    if (c0 < Rk) {
      std::vector<int> colj;
      for (int j = 0; j < k; ++j)
        for (int c = 0; c < h->lr(k, j); ++c)
          if (h->lo(k, j) + c >= c0) colj.push_back(j);
      void* dcol = nullptr;
      TLR_TRY(h->stage.upload(h, colj.data(), sizeof(int) * colj.size(), &dcol));
      TLR_HIP(launch_scale_panel(h->VL[k] + (size_t)c0 * m, m, w.W.as<double>() + (size_t)c0 * m,
                                 m, m, (int)colj.size(), (const int*)dcol, h->Dv, h->stream));
    }
    Vk = w.W.as<double>();
  }
  DevBuf& gbuf = (k & 1) ? w.G2 : w.G;
  if (ahead) {
    for (int i = k; i < nb; ++i)
      for (int j = 0; j < k - 1; ++j) p.goff[(size_t)i * nb + j] = p.goff_next[(size_t)i * nb + j];
    p.G = p.Gnext;
    TLR_HIP(hipStreamWaitEvent(h->stream, h->ev_gnext, 0));
  } else {
    long long gtot = 0;
    for (int i = k; i < nb; ++i)
      for (int j = 0; j < k - 1; ++j) {
        const int a = h->lr(i, j), b = h->lr(k, j);
        p.goff[(size_t)i * nb + j] = (a > 0 && b > 0) ? gtot : -1;
        if (a > 0 && b > 0) gtot += (long long)a * b;
      }
    TLR_TRY(gbuf.ensure(h->mem, sizeof(double) * (size_t)std::max(gtot, 1LL)));
    p.G = gbuf.as<double>();
    GemmBatch g(true, false);
    for (int i = k; i < nb; ++i)
      for (int j = 0; j < k - 1; ++j) {
        const long long go = p.goff[(size_t)i * nb + j];
        if (go < 0) continue;
        const int a = h->lr(i, j), b = h->lr(k, j);
        g.add(a, b, m, h->vl(i, j), m, Vk + h->lo(k, j) * m, m, p.G + go, a, 1.0, 0.0);
      }
    TLR_TRY(g.run(h));
    p.flops += g.flops;
  }
  p.jk = k - 1;
  p.gkoff.assign(nb, -1);
  if (k >= 1) {
    const int j = k - 1;
    long long gk = 0;
    for (int i = k; i < nb; ++i) {
      const int a = h->lr(i, j), b = h->lr(k, j);
      p.gkoff[i] = (a > 0 && b > 0) ? gk : -1;
      if (a > 0 && b > 0) gk += (long long)a * b;
    }
    TLR_TRY(w.Gk.ensure(h->mem, sizeof(double) * (size_t)std::max(gk, 1LL)));
    p.Gk = w.Gk.as<double>();
    GemmBatch g(true, false);
    for (int i = k; i < nb; ++i) {
      if (p.gkoff[i] < 0) continue;
      const int a = h->lr(i, j), b = h->lr(k, j);
      g.add(a, b, m, h->vl(i, j), m, Vk + h->lo(k, j) * m, m, p.Gk + p.gkoff[i], a, 1.0, 0.0);
    }
    TLR_TRY(g.run(h));
    p.flops += g.flops;
  }
  // ---------------------------------------------- updateDense + chol / ldl
  // on the diagonal-tile stream: they need only the G blocks and row k's
  // panels, and the column's ARA needs L_kk only at the triangular solve
  TLR_HIP(hipEventRecord(h->ev_fork, h->stream));
  TLR_HIP(hipStreamWaitEvent(h->side, h->ev_fork, 0));
  p.flops_paper += 2.0 * m * (double)m * Rk + (double)m * m * m / 3.0;
  p.flops += (double)m * m * m / 3.0 + (double)m * m * m / 3.0;
  p.nrow = nb - k - 1;
  // ---------------------------------------------- sortRanks
  // The order (descending input rank, ties by row) needs only the input
  // ranks: it is taken on the host and the device queue is not drained
  // (the mixed form's precision choice is made on the device).
  p.order.assign(p.nrow, 0);
  if (p.nrow > 0) {
    std::vector<int> rk(p.nrow), rows(p.nrow);
    for (int s = 0; s < p.nrow; ++s) {
      rows[s] = k + 1 + s;
      rk[s] = h->pr(k + 1 + s, k);
    }
    sort_ranks(rk.data(), rows.data(), p.nrow, p.order.data());
  }
  std::vector<int>& log = h->sort_log[k];
  log.resize(p.nrow);
  for (int s = 0; s < p.nrow; ++s) log[s] = k + 1 + p.order[s];
  return TLR_OK;
}

// The launches of column k's diagonal tile (dense update, factorization,
// inverse) on the diagonal-tile stream, which waits for the fork recorded by
// col_begin.  The host builds them in the first wait of the column's
// iterations (the main stream then holds two iterations of work); the
// column's iterations need L_kk only at the triangular solve.
tlr_status col_diag(Prob& p, int k, bool ldl) {
  Handle* h = p.h;
  const int m = h->m;
  const int Rk = p.Rk;
  Work& w = h->ws;
  double* Lkk = h->diagL(k);
  hipStream_t ds = h->side;
  if (Rk > 0 && w.Wd.cap < sizeof(double) * (size_t)m * Rk) {
    TLR_HIP(hipStreamSynchronize(ds));
    TLR_TRY(w.Wd.ensure(h->mem, sizeof(double) * (size_t)m * Rk));
  }
  p.dplan.reset(new Plan(h, ds));
  Plan& dplan = *p.dplan;
  dplan.persist = &w.sideblob;
  {
    // pivoting: the updated tile S_k already holds the shift and every
    // low rank product of the columns j < k.  The updated tile is formed in
    // place of the factor, or in the captured factorization's buffer.
    const double* Akk = p.piv ? h->Sd + (size_t)h->spos[k] * m * m : h->diagA(k);
    const int nr = h->nreal(k);
    const double shift = p.piv ? 0.0 : p.shift;
    double* Tk = p.dg ? p.dg->A.as<double>() : Lkk;
    dplan.launch([=]() { return launch_copy_shift(Akk, Tk, m, nr, shift, ds); });
    if (Rk > 0 && !p.piv) {
      double* Wd = w.Wd.as<double>();
      GemmBatch wb(false, false);
      for (int j = 0; j < k; ++j) {
        const int r = h->lr(k, j);
        if (r == 0) continue;
        wb.add(m, r, r, h->ul(k, j), m, p.gptr(k, j), r, Wd + h->lo(k, j) * m, m, 1.0, 0.0);
      }
      dplan.gemm(wb);
      GemmBatch up(false, true);
      up.add(m, m, Rk, Wd, m, h->UL[k], m, Tk, m, -1.0, 1.0, GEMM_LOWER_C);
      dplan.gemm(up);
      p.flops += wb.flops + up.flops / 2;
      if (p.schur) {
        // Schur compensation (Section 5.1.1): the update D_k = W U_k*^T in
        // full; the part its compression to tau drops is D_k P, P the
        // spectral projector on the eigenvalues <= tau,
        // P = (I - sign(D_k - tau I)) / 2; the sign function from
        // X_0 = (D_k - tau I) / ||D_k - tau I||_F (eigenvalues in [-1, 1])
        // by the quintic and then the Newton-Schulz steps, matrix products
        // only; then the absolute row sums of E = (D_k - D_k X) / 2 onto
        // the diagonal of the updated tile
        const size_t mm = (size_t)m * m;
        double* D = p.sch;
        double* X = p.sch + mm;
        double* Xn = p.sch + 2 * mm;
        double* Y = p.sch + 3 * mm;
        double* E = p.sch + 4 * mm;
        double* parts = p.sch + 5 * mm;
        double* nrm = parts + (kPivotTolDoubles - 32);
        const double tau = p.tau;
        GemmBatch db(false, true);
        db.add(m, m, Rk, Wd, m, h->UL[k], m, D, m, 1.0, 0.0);
        dplan.gemm(db);
        p.flops += db.flops;
        dplan.launch([=]() { return launch_schur_shift(D, m, tau, X, ds); });
        dplan.launch([=]() { return launch_norm2(X, (long long)mm, nrm, parts, ds); });
        dplan.launch([=]() { return launch_scale_by(X, (long long)mm, nrm, X, ds); });
        auto copy = [&](const double* src, double* dst) {
          dplan.launch([=]() {
            return hipMemcpyAsync(dst, src, sizeof(double) * mm, hipMemcpyDeviceToDevice, ds);
          });
        };
        for (int it = 0; it < kSchurQuinticIters + kSchurSignIters; ++it) {
          GemmBatch sq(false, false);
          sq.add(m, m, m, X, m, X, m, Y, m, 1.0, 0.0);   // Y = X^2
          dplan.gemm(sq);
          p.flops += sq.flops;
          copy(X, Xn);
          GemmBatch st(false, false);
          if (it < kSchurQuinticIters) {
            // E (scratch) = c Y^2 + b Y, then X' = X E + a X
            copy(Y, E);
            GemmBatch q4(false, false);
            q4.add(m, m, m, Y, m, Y, m, E, m, kQc, kQb);
            dplan.gemm(q4);
            p.flops += q4.flops;
            st.add(m, m, m, X, m, E, m, Xn, m, 1.0, kQa);
          } else {
            st.add(m, m, m, X, m, Y, m, Xn, m, -0.5, 1.5);   // X' = (3 X - X^3) / 2
          }
          dplan.gemm(st);
          p.flops += st.flops;
          std::swap(X, Xn);
        }
        copy(D, E);
        GemmBatch eb(false, false);
        eb.add(m, m, m, D, m, X, m, E, m, -0.5, 0.5);
        dplan.gemm(eb);
        dplan.launch([=]() { return launch_schur_diag(E, m, Tk, m, nr, ds); });
        p.flops += eb.flops;
      }
    }
    if (DiagGraph* g = p.dg) {
      // the updated tile went to the graph's buffer (above); one replay,
      // then the results to their places
      double* tol = g->tol.as<double>();
      const double md = p.mod_delta;
      if (md > 0.0) dplan.launch([=]() { return launch_fill(tol, 1, md, ds); });
      hipGraphExec_t ex = g->exec;
      dplan.launch([=]() { return hipGraphLaunch(ex, ds); });
      const double* gA = g->A.as<double>();
      const double* gL = g->Linv.as<double>();
      const double* gD = ldl ? g->D.as<double>() : nullptr;
      double* dv = ldl ? h->Dv + (size_t)k * m : nullptr;
      double* Li = h->invL(k);
      int* gi = g->info.as<int>();
      int* info = h->d_info;
      const int rb = k * m;
      dplan.launch([=]() {
        return launch_diag_out(gA, Lkk, gL, Li, gD, dv, m, gi, info, rb, ds);
      });
    } else {
      TLR_TRY(dense_factor(h, dplan, !ldl, Lkk, m, m, ldl ? h->Dv + (size_t)k * m : nullptr,
                           k * m, h->invL(k), p.mod_delta));
    }
    // the staged descriptors go up from this thread; the launches are
    // issued by the handle's side worker, which also records the join
    TLR_TRY(dplan.run_some(0));
    if (!h->worker) h->worker.reset(new SideWorker(h->dev));
    std::shared_ptr<Plan> plan(p.dplan.release());
    hipEvent_t ej = h->ev_join;
    PhaseTimer* pts = &h->pt_side;
    h->worker->submit([plan, ej, ds, pts]() -> tlr_status {
      TLR_HIP(pts->mark(TLR_PHASE_DIAG, ds));
      TLR_TRY(plan->run());
      TLR_HIP(pts->mark(-1, ds));
      TLR_HIP(hipEventRecord(ej, ds));
      return TLR_OK;
    });
    p.side_pending = true;
  }
  return TLR_OK;
}

// Lookahead: the blocks j < k of column k + 1's G read only panels (and,
// for LDL^T, pivots) that are final, so they are formed on the diagonal-tile
// stream after column k's diagonal tile, while the main stream runs column
// k's iterations; the host builds the batch in the first wait of those
// iterations.  Their buffer was last read by column k - 1, whose launches
// precede column k's fork to that stream.
tlr_status col_lookahead(Prob& p, int k, bool ldl) {
  Handle* h = p.h;
  const int m = h->m, nb = h->nb;
  Work& w = h->ws;
  hipStream_t ds = h->side;
  if (k + 1 < nb && k >= 1 && !p.piv) {
    const int kn = k + 1;
    p.goff_next.assign((size_t)nb * nb, -1);
    long long gt = 0;
    for (int i = kn; i < nb; ++i)
      for (int j = 0; j < k; ++j) {
        const int a = h->lr(i, j), b = h->lr(kn, j);
        p.goff_next[(size_t)i * nb + j] = (a > 0 && b > 0) ? gt : -1;
        if (a > 0 && b > 0) gt += (long long)a * b;
      }
    DevBuf& nbuf = (kn & 1) ? w.G2 : w.G;
    TLR_TRY(nbuf.ensure(h->mem, sizeof(double) * (size_t)std::max(gt, 1LL)));
    p.Gnext = nbuf.as<double>();
    p.gplan.reset(new Plan(h, ds));
    p.gplan->persist = &w.sideblob2;
    // LDL^T: the blocks j < k of row k + 1's panel scaled by D_j (D_k is
    // being formed on this stream, before these launches)
    const double* Vn = h->VL[kn];
    if (ldl) {
      std::vector<int> colj;
      for (int j = 0; j < k; ++j)
        for (int c = 0; c < h->lr(kn, j); ++c) colj.push_back(j);
      if (!colj.empty()) {
        TLR_TRY(w.Wn.ensure(h->mem, sizeof(double) * (size_t)m * colj.size()));
        double* Wn = w.Wn.as<double>();
        const double* src = h->VL[kn];
        const double* Dv = h->Dv;
        const int nc = (int)colj.size();
        const size_t off = p.gplan->stage(colj.data(), sizeof(int) * colj.size());
        p.gplan->launch(off, [=](const char* ptr) {
          return launch_scale_panel(src, m, Wn, m, m, nc, (const int*)ptr, Dv, ds);
        });
        Vn = Wn;
      }
    }
    GemmBatch g(true, false);
    for (int i = kn; i < nb; ++i)
      for (int j = 0; j < k; ++j) {
        const long long go = p.goff_next[(size_t)i * nb + j];
        if (go < 0) continue;
        const int a = h->lr(i, j), b = h->lr(kn, j);
        g.add(a, b, m, h->vl(i, j), m, Vn + h->lo(kn, j) * m, m, p.Gnext + go, a, 1.0, 0.0);
      }
    p.gplan->gemm(g);
    TLR_TRY(p.gplan->run_some(0));
    p.flops += g.flops;
    p.ahead = kn;
    std::shared_ptr<Plan> gplan(p.gplan.release());
    hipEvent_t eg = h->ev_gnext;
    PhaseTimer* pts = &h->pt_side;
    h->worker->submit([gplan, eg, ds, pts]() -> tlr_status {
      TLR_HIP(pts->mark(TLR_PHASE_DIAG, ds));
      TLR_TRY(gplan->run());
      TLR_HIP(pts->mark(-1, ds));
      TLR_HIP(hipEventRecord(eg, ds));
      return TLR_OK;
    });
  }
  return TLR_OK;
}

tlr_status side_done(Prob& p) {
  if (!p.side_pending) return TLR_OK;
  p.side_pending = false;
  return p.h->worker->wait();
}


// The sampling description of problem p's tiles of column k, appended to the
// pooled spec at slots [p.base, p.base + p.nrow) and P rows [p.roff, ...).
tlr_status col_spec(Prob& p, int k, int bsm, AraSpec& spec) {
  Handle* h = p.h;
  const int m = h->m, nrow = p.nrow, Rk = p.Rk;
  Work& w = h->ws;
  TLR_TRY(w.Wa.ensure(h->mem, sizeof(double) * (size_t)nrow * m * bsm));
  {
    long long zt = 0;
    for (int s = 0; s < nrow; ++s) zt += h->R[k + 1 + s];
    TLR_TRY(w.Z.ensure(h->mem, sizeof(double) * (size_t)std::max(zt, 1LL) * bsm));
  }
  double* Wa = w.Wa.as<double>();
  double* Z = w.Z.as<double>();
  // static sampling description of every tile of the column:
  //   Y_i = U^A_ik W^A_i + U_i* Z_i,  W^A_i = V^A_ik^T Omega,
  //   Z_i = -[G_ij P_j]_j,  P = U_k*^T Omega
  if (Rk > 0) spec.pg.push_back(PGroup{h->UL[k], Rk, p.roff});
  long long zo = 0;
  for (int s = 0; s < nrow; ++s) {
    const int i = k + 1 + s;
    const int a = h->pr(i, k), Ri = h->R[i];
    AraSlotDesc& d = spec.slots[p.base + s];
    double* wa_s = Wa + (size_t)s * m * bsm;
    d.a0 = h->pu(i, k);
    d.lda0 = m;
    d.k0 = a;
    d.b0 = wa_s;
    d.ldb0 = std::max(a, 1);
    d.va = h->pv(i, k);
    d.wa = wa_s;
    d.a = a;
    spec.a_max = std::max(spec.a_max, a);
    d.lda1 = m;
    d.ldb1 = 1;
    if (Rk > 0 && Ri > 0) {
      double* zs = Z + zo;
      zo += (long long)Ri * bsm;
      d.a1 = (const void*)h->UL[i];
      d.a1_prec = 0;
      d.k1 = Ri;
      d.b1 = zs;
      d.ldb1 = Ri;
      d.z = zs;
      d.R = Ri;
      d.zseg = (int)spec.zseg.size();
      for (int j = 0; j < k; ++j) {
        const int rij = h->lr(i, j);
        for (int r0 = 0; r0 < rij; r0 += 16)
          spec.zseg.push_back(ZSeg{p.gptr(i, j) + r0, rij, std::min(16, rij - r0), h->lr(k, j),
                                   (int)h->lo(i, j) + r0, p.roff + (int)h->lo(k, j)});
      }
      d.nz = (int)spec.zseg.size() - d.zseg;
      spec.r_max = std::max(spec.r_max, Ri);
    }
    const double kk = (double)a + d.k1;
    spec.samp_flops_col[p.base + s] = 2.0 * m * kk;
    spec.samp_bytes[p.base + s] = 8.0 * m * a + 8.0 * m * d.k1;
    if (h->mixed && d.k1 > 0) {
      // a low-precision panel term when its rounding, (2 u_p + sqrt(R_i)
      // u32) nu_ik with nu_ik = ||A_ik||_F + sum_j ||L_ij||_F ||L_kj||_F,
      // stays below tau / 16 (both operands rounded once, FP32 accumulation
      // over R_i terms); the newest column's term of nu is added on the
      // device, where its norms were formed
      const int nb = h->nb;
      double nu = h->a_fro[(size_t)i * nb + k];
      for (int j = 0; j + 1 < k; ++j)
        nu += h->l_fro[(size_t)i * nb + j] * h->l_fro[(size_t)k * nb + j];
      const double u32 = 5.9604644775390625e-08, u16 = 3.90625e-03;
      const double acc = std::sqrt((double)d.k1) * u32;
      spec.samp_bytes32[p.base + s] = 8.0 * m * a + 4.0 * m * d.k1;
      spec.samp_bytes16[p.base + s] = 8.0 * m * a + 2.0 * m * d.k1;
      spec.guard[p.base + s] =
          GuardDesc{(const void*)h->UL32[i], h->mixed >= 2 ? (const void*)h->UL16[i] : nullptr,
                    h->ws.fro.as<double>(), nu, p.tau_ara / (16.0 * (2.0 * u32 + acc)),
                    p.tau_ara / (16.0 * (2.0 * u16 + acc)), k >= 1 ? i - k : -1, (m + 15) / 16};
    }
    spec.samp_bytes_col[p.base + s] = 8.0 * (kk + m);
    spec.tau[p.base + s] = p.tau_ara;
  }
  return TLR_OK;
}

// Column k, after the ARA: projection B_i = S_ik^T Q_i, batched triangular
// solve with L_kk, and the append of U_ik = Q_i, V_ik to the row panels.
tlr_status col_finish(Prob& p, int k, bool ldl, const AraConfig& cfg, const AraSlots& slots,
                      const AraResult& res) {
  // the norms of column k - 1's factor tiles, read back by the previous
  // projection (complete: this column's iterations ran after it)
  if (p.h->mixed && k > 0)
    for (int s = 0; s < p.h->nb - k; ++s)
      p.h->l_fro[(size_t)(k + s) * p.h->nb + (k - 1)] = p.pin_norm[s];
  Handle* h = p.h;
  const int m = h->m, nb = h->nb, nrow = p.nrow, Rk = p.Rk;
  Work& w = h->ws;
  // W^A, Z and P products of the iterations (P counted for the problem's
  // share of the launches: the iterations its tiles took part in)
  int launches = 0;
  for (int s = 0; s < nrow; ++s) launches = std::max(launches, res.iters[p.base + s]);
  double cols_launched = 0.0;
  for (int j = 0; j < launches && j < (int)res.iter_bs.size(); ++j) cols_launched += res.iter_bs[j];
  p.flops += 2.0 * Rk * m * cols_launched;
  std::vector<int> q(nrow), it(nrow);
  for (int s = 0; s < nrow; ++s) {
    const int i = k + 1 + s, sl = p.base + s;
    q[s] = res.q[sl];
    it[s] = res.iters[sl];
    double zf = 0.0;
    for (int j = 0; j < k; ++j) zf += (double)h->lr(i, j) * h->lr(k, j);
    const double cols = res.cols[sl];
    p.flops += cols * 2.0 * ((double)h->pr(i, k) * m + zf);
    if (res.f32[sl] == 1) p.fp32_tile_iters += it[s];
    if (res.f32[sl] == 2) p.bf16_tile_iters += it[s];
    p.flops += res.flops_slot[sl];
    p.samp_bytes += res.samp_bytes_slot[sl];
    p.samp_flops += res.samp_flops_slot[sl];
  }
  p.ara_iters += launches;
  p.t_issue += res.t_issue;
  p.t_wait += res.t_wait;

  // ---------------------------------------------- projection  B_i = S_ik^T Q_i
  std::vector<long long> boff(nrow), toff(nrow), taoff(nrow);
  long long sq = 0, st_ = 0, sta = 0;
  for (int s = 0; s < nrow; ++s) {
    const int i = k + 1 + s;
    boff[s] = sq;
    toff[s] = st_;
    taoff[s] = sta;
    sq += q[s];
    st_ += (long long)h->R[i] * q[s];
    sta += (long long)h->pr(i, k) * q[s];
  }
  TLR_TRY(w.T.ensure(h->mem, sizeof(double) * (size_t)std::max(st_, 1LL)));
  TLR_TRY(w.Ta.ensure(h->mem, sizeof(double) * (size_t)std::max(sta, 1LL)));
  TLR_TRY(w.H.ensure(h->mem, sizeof(double) * (size_t)std::max((long long)Rk * sq, 1LL)));
  TLR_TRY(w.Ball.ensure(h->mem, sizeof(double) * (size_t)std::max((long long)m * sq, 1LL)));
  double* T = w.T.as<double>();
  double* Ta = w.Ta.as<double>();
  double* H = w.H.as<double>();
  double* Ball = w.Ball.as<double>();
  TLR_TRY(w.Bt.ensure(h->mem, sizeof(double) * (size_t)std::max((long long)m * sq, 1LL)));
  double* Bt = w.Bt.as<double>();
  for (int s = 0; s < nrow; ++s)
    if (q[s] > 0) TLR_TRY(grow_row(h, k + 1 + s, q[s]));
  // partial products of the split long products (at most 8 slices of
  // m x sq); growing it waits for both streams, whose queued work may read
  // the old buffer (the diagonal-tile stream has no launches left to issue)
  {
    const size_t need = sizeof(double) * 8 * (size_t)m * (size_t)std::max(sq, 1LL);
    if (w.splitk.cap < need) {
      TLR_TRY(h->sync());
      TLR_TRY(w.splitk.ensure(h->mem, need));
    }
  }
  // The products that need only the bases go out first, so the GPU works on
  // them while the host builds the per-block batch of the update term.
  TLR_HIP(p.pt->mark(TLR_PHASE_PROJECT, h->stream));
  {
    Plan first(h);
    GemmBatch t1(true, false), t2(true, false), b1(false, false);
    for (int s = 0; s < nrow; ++s) {
      const int i = k + 1 + s, qs = q[s];
      if (qs == 0) continue;
      const int a = h->pr(i, k), Ri = h->R[i];
      const double* Qs = slots.qb(p.base + s);
      if (Ri > 0) t1.add(Ri, qs, m, h->UL[i], m, Qs, m, T + toff[s], Ri, 1.0, 0.0);
      if (a > 0) t2.add(a, qs, m, h->pu(i, k), m, Qs, m, Ta + taoff[s], a, 1.0, 0.0);
      b1.add(m, qs, a, h->pv(i, k), m, Ta + taoff[s], std::max(a, 1), Ball + boff[s] * m, m, 1.0,
             0.0);
    }
    // t1 and t2 stream the same basis blocks Q_i: one batch
    for (const GemmDesc& d : t2.d) t1.d.push_back(d);
    t1.flops += t2.flops;
    first.gemm(t1);
    first.gemm(b1);
    TLR_TRY(first.run());
    p.flops += first.flops;
  }
  Plan plan(h);
  plan.splitk = &w.splitk;
  {
    GemmBatch hb(true, false), b2(false, false);
    if (Rk > 0) {
      for (int s = 0; s < nrow; ++s) {
        const int i = k + 1 + s, qs = q[s];
        if (qs == 0) continue;
        const int Ri = h->R[i];
        for (int j = 0; j < k; ++j) {
          const int rkj = h->lr(k, j);
          if (rkj == 0) continue;
          const int rij = h->lr(i, j);
          hb.add(rkj, qs, rij, p.gptr(i, j), rij, T + toff[s] + (rij > 0 ? h->lo(i, j) : 0),
                 std::max(Ri, 1), H + boff[s] * Rk + h->lo(k, j), Rk, 1.0, 0.0);
        }
      }
    }
    if (Rk > 0 && sq > 0) b2.add(m, (int)sq, Rk, h->UL[k], m, H, Rk, Ball, m, -1.0, 1.0);
    plan.gemm(hb);
    plan.gemm(b2);
  }
  // ---------------------------------------------- batchTrsm (+ batchIDMult)
  // V = L_kk^{-1} B for every tile of the column: one triangular product
  PhaseTimer* pt = p.pt;
  {
    hipStream_t st = h->stream;
    hipEvent_t ej = h->ev_join;
    plan.launch([=]() { return pt->mark(TLR_PHASE_TRSM, st); });
    plan.launch([=]() { return hipStreamWaitEvent(st, ej, 0); });
    GemmBatch tb(false, false);
    tb.add(m, (int)sq, m, h->invL(k), m, Ball, m, Bt, m, 1.0, 0.0, GEMM_TRIL_A);
    plan.gemm(tb);
    if (ldl && sq > 0) {
      const double* dk = h->Dv + (size_t)k * m;
      const int n = (int)sq;
      plan.launch([=]() { return launch_scale_rows(Bt, m, Bt, m, dk, m, n, true, st); });
    }
  }
  p.flops += (double)m * m * sq;
  // ---------------------------------------------- updateTiles
  {
    hipStream_t st = h->stream;
    plan.launch([=]() { return pt->mark(TLR_PHASE_APPEND, st); });
    std::vector<CopyDesc> cd;
    int maxc = 0;
    for (int s = 0; s < nrow; ++s) {
      const int i = k + 1 + s, qs = q[s];
      if (qs == 0) continue;
      CopyDesc c{slots.qb(p.base + s), h->UL[i] + (size_t)h->R[i] * m, m, qs, m, m};
      if (h->mixed) {
        c.dst32 = h->UL32[i];
        c.dst16 = h->UL16[i];
        c.pcol = h->R[i];
      }
      cd.push_back(c);
      cd.push_back(CopyDesc{Bt + boff[s] * m, h->VL[i] + (size_t)h->R[i] * m, m, qs, m, m});
      maxc = std::max(maxc, qs);
    }
    if (!cd.empty()) {
      const size_t off = plan.stage(cd.data(), sizeof(CopyDesc) * cd.size());
      const int n = (int)cd.size();
      hipStream_t st = h->stream;
      plan.launch(off, [=](const char* ptr) {
        return launch_copy_batched((const CopyDesc*)ptr, n, maxc, st);
      });
    }
  }
  if (h->mixed) {
    // ||L_ik||_F = ||V_ik||_F (U_ik orthonormal): read on the device by the
    // next column's precision choice, and stored by the same kernel to the
    // host's pinned copy for the later columns' sums
    TLR_TRY(w.fro.ensure(h->mem, sizeof(double) * (size_t)std::max(nrow, 1)));
    double* fro = w.fro.as<double>();
    std::vector<NormDesc> nd;
    for (int s = 0; s < nrow; ++s)
      nd.push_back(NormDesc{Bt + boff[s] * m, m, q[s], m, fro + s, p.pin_norm + s});
    const size_t off = plan.stage(nd.data(), sizeof(NormDesc) * nd.size());
    const int n = nrow;
    hipStream_t st = h->stream;
    plan.launch(off, [=](const char* ptr) { return launch_fro_norms((const NormDesc*)ptr, n, st); });
  }
  TLR_TRY(plan.run());
  p.flops += plan.flops;
  for (int s = 0; s < nrow; ++s) {
    const int i = k + 1 + s;
    h->l_rank[(size_t)i * nb + k] = q[s];
    h->l_off[(size_t)i * nb + k] = h->R[i];
    h->R[i] += q[s];
    // operation count of the paper's formulation (four-product sampling of
    // Eq. (2) per iteration, the same for the projection, orthogonalisation,
    // triangular solve)
    const double ext = (double)h->R[i] - q[s] + Rk + h->pr(i, k);
    const double cols = res.cols[p.base + s];
    p.flops_paper += cols * 4.0 * m * ext + 4.0 * m * q[s] * ext +
                     res.flops_paper_orth[p.base + s] + (double)m * m * q[s];
    p.bytes_alg += it[s] * 8.0 * m * ((double)h->R[i] - q[s] + h->pr(i, k));
    p.tile_iters += it[s];
  }
  return TLR_OK;
}

// Statistics and status of a finished problem.
tlr_status prob_finish(Prob& p, const tlr_opts& o, bool ldl, tlr_stats* st,
                       const double* t_main) {
  Handle* h = p.h;
  const int m = h->m, nb = h->nb;
  double samp_ms = 0.0;
  for (auto& ev : p.events) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) samp_ms += ms;
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  const long long nev = (long long)p.events.size();
  p.events.clear();
  int iw[2] = {0, 0};
  TLR_HIP(hipMemcpy(iw, h->d_info, sizeof iw, hipMemcpyDeviceToHost));
  const int info = iw[0];
  if (st) {
    std::memset(st, 0, sizeof *st);
    st->info = info;
    st->tau = p.tau;
    st->norm_a = o.eps_mode == TLR_EPS_REL ? h->norm_a : 0.0;
    st->flops = p.flops;
    st->flops_paper = p.flops_paper;
    st->bytes_alg = p.bytes_alg;
    st->ara_iters = p.ara_iters;
    st->tile_iters = p.tile_iters;
    st->fp32_tile_iters = p.fp32_tile_iters;
    st->bf16_tile_iters = p.bf16_tile_iters;
    st->modified_pivots = iw[1];
    st->t_host_issue = p.t_issue;
    st->t_host_wait = p.t_wait;
    long long cnt = 0, tot = 0, full = 0;
    int mx = 0;
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < i; ++j) {
        const int r = h->lr(i, j);
        tot += r;
        ++cnt;
        mx = std::max(mx, r);
        if (r >= m) ++full;
      }
    st->max_rank = mx;
    st->mean_rank = cnt ? (double)tot / cnt : 0.0;
    st->full_rank_tiles = full;
    st->factor_bytes = 8.0 * ((double)nb * m * m + 2.0 * m * (double)tot);
    st->sample_launches = nev;
    st->sample_ms = samp_ms;
    st->sample_bytes = p.samp_bytes;
    st->sample_flops = p.samp_flops;
    st->shift = p.shift;
    if (h->pt_side.on) {
      for (int f = 0; f < TLR_NPHASE; ++f) st->t_phase[f] = t_main[f];
      TLR_TRY(h->pt_side.collect(st->t_phase));
    }
  }
  if (info != 0) {
    h->factored = 0;
    set_error("diagonal tile %d lost %s at global row %d", (info - 1) / m,
              ldl ? "a nonzero pivot" : "positive definiteness", info);
    return ldl ? TLR_ERR_ZERO_PIVOT : TLR_ERR_NOT_SPD;
  }
  h->factored = ldl ? 2 : 1;
  return TLR_OK;
}

// Problems of one tile size, stepped through the columns together: at step
// k every problem with more than k block columns does its column k, and the
// ARA of all their Schur-complement tiles is one pooled run (the union of
// the active tiles of every problem in each launch).  Everything runs on
// the first problem's (shared) main stream; each problem keeps its own
// diagonal-tile stream.
tlr_status factorize_group(std::vector<Prob>& ps, const double* eps, const tlr_opts& o,
                           bool ldl, tlr_stats* stats, const std::vector<int>& idx) {
  Handle* lead = ps[idx[0]].h;
  const int m = lead->m, bs = o.bs;
  int nbmax = 0, slots_max = 1;
  const bool phases = (o.flags & TLR_FLAG_PHASE_TIMING) != 0;
  lead->pt_main.reset(phases);
  for (int pi : idx) {
    ps[pi].pt = &lead->pt_main;
    ps[pi].h->pt_side.reset(phases);
    TLR_TRY(prob_init(ps[pi], eps[pi], o, ldl));
    nbmax = std::max(nbmax, ps[pi].h->nb);
  }
  for (int k = 0; k < nbmax; ++k) {
    int tot = 0;
    for (int pi : idx)
      if (k < ps[pi].h->nb) tot += ps[pi].h->nb - k - 1;
    slots_max = std::max(slots_max, tot);
  }
  AraConfig cfg;
  cfg.m = m;
  cfg.bs = bs;
  cfg.bs_tail = o.bs_tail;
  cfg.tail_active = o.tail_active;
  cfg.qcap = m;
  cfg.tau = ps[idx[0]].tau;
  cfg.r_min = o.r_min;
  cfg.s_max = o.max_active;
  cfg.seed = o.seed;
  cfg.strip = o.sample_strip;
  cfg.overlap = (o.flags & TLR_FLAG_SERIAL_SAMPLING) == 0;
  AraSlots slots;
  TLR_TRY(ara_slots(lead, cfg, slots_max, &slots));
  const bool timing = (o.flags & TLR_FLAG_KERNEL_TIMING) != 0;
  const bool single = idx.size() == 1;

  for (int k = 0; k < nbmax; ++k) {
    std::vector<int> live;
    for (int pi : idx)
      if (!ps[pi].done && k < ps[pi].h->nb) live.push_back(pi);
    if (live.empty()) break;
    // ---- G, diagonal-tile stream, device sortRanks of every problem
    int base = 0;
    for (int pi : live) {
      Prob& p = ps[pi];
      p.base = base;
      TLR_TRY(col_begin(p, k, ldl));
      base += p.nrow;
    }
    const int total = base;
    std::vector<int> order;
    {
      // pooled sortRanks: descending input rank; ties by problem, then by
      // each problem's own order (one problem: its device order unchanged)
      std::vector<std::pair<int, int>> key;   // (rank, global slot)
      for (int pi : live) {
        Prob& p = ps[pi];
        for (int s : p.order) key.push_back({p.h->pr(k + 1 + s, k), p.base + s});
      }
      std::stable_sort(key.begin(), key.end(),
                       [](const std::pair<int, int>& a, const std::pair<int, int>& b) {
                         return a.first > b.first;
                       });
      for (auto& kv : key) order.push_back(kv.second);
    }
    // a problem at its last column has only its diagonal tile left
    for (int pi : live)
      if (ps[pi].nrow == 0) {
        TLR_TRY(col_diag(ps[pi], k, ldl));
        TLR_TRY(side_done(ps[pi]));
        ps[pi].done = true;
      }
    if (total == 0) continue;
    // ---- pooled ARA of every problem's column-k tiles
    const int bsm = cfg.bs_max();
    AraSpec spec;
    spec.slots.assign(total, AraSlotDesc{});
    spec.samp_bytes.assign(total, 0.0);
    spec.samp_bytes_col.assign(total, 0.0);
    spec.samp_flops_col.assign(total, 0.0);
    spec.tau.assign(total, 0.0);
    if (lead->mixed) {
      GuardDesc none{};
      none.irow = -1;
      spec.guard.assign(total, none);
      spec.samp_bytes32.assign(total, 0.0);
      spec.samp_bytes16.assign(total, 0.0);
    }
    int prow = 0;
    for (int pi : live) {
      Prob& p = ps[pi];
      if (p.nrow == 0) continue;
      p.roff = prow;
      prow += p.Rk;
    }
    Work& lw = lead->ws;
    TLR_TRY(lw.P.ensure(lead->mem, sizeof(double) * (size_t)std::max(prow, 1) * bsm));
    spec.p = lw.P.as<double>();
    spec.ldp = std::max(prow, 1);
    spec.events = timing ? &ps[idx[0]].events : nullptr;
    spec.pt = phases ? &lead->pt_main : nullptr;
    for (int pi : live) {
      Prob& p = ps[pi];
      if (p.nrow > 0) TLR_TRY(col_spec(p, k, bsm, spec));
    }
    AraResult res;
    cfg.stream_id = (unsigned)k;
    bool abort = false;
    // the first wait of the iterations builds the next column's lookahead
    bool looked = false;
    auto lookahead = [&]() -> tlr_status {
      if (looked) return TLR_OK;
      looked = true;
      for (int pi : live)
        if (!ps[pi].done) {
          TLR_TRY(col_diag(ps[pi], k, ldl));
          TLR_TRY(col_lookahead(ps[pi], k, ldl));
        }
      return TLR_OK;
    };
    TLR_TRY(ara_run(lead, cfg, slots, order, spec, &res, single ? &abort : nullptr, lookahead));
    TLR_TRY(lookahead());
    for (int pi : live) TLR_TRY(side_done(ps[pi]));
    if (abort) {
      ps[idx[0]].done = true;
      break;
    }
    for (int pi : live) {
      Prob& p = ps[pi];
      if (p.nrow == 0) continue;
      TLR_TRY(col_finish(p, k, ldl, cfg, slots, res));
    }
  }
  for (int pi : idx) {
    Handle* h = ps[pi].h;
    TLR_HIP(hipEventRecord(h->ev_join, h->side));
    TLR_HIP(hipStreamWaitEvent(h->stream, h->ev_join, 0));
  }
  TLR_HIP(lead->pt_main.mark(-1, lead->stream));
  for (int pi : idx) TLR_TRY(ps[pi].h->sync());
  for (int pi : idx) {
    Handle* h = ps[pi].h;
    release_retired(h);
    // the updated diagonal tiles of the pivoted form are spent (the
    // permutation stays with the factor)
    h->mem.put(h->Sd);
    h->Sd = nullptr;
    h->spos.clear();
  }
  double t_main[TLR_NPHASE] = {0.0};
  if (phases) TLR_TRY(lead->pt_main.collect(t_main));
  tlr_status first = TLR_OK;
  for (int pi : idx) {
    const tlr_status s = prob_finish(ps[pi], o, ldl, stats ? stats + pi : nullptr, t_main);
    if (first == TLR_OK && s != TLR_OK) first = s;
  }
  return first;
}

}  // namespace

tlr_status factorize_batch(Handle* const* hs, int count, const double* eps, const tlr_opts& o,
                           tlr_stats* st, bool ldl, bool piv) {
  std::vector<Prob> ps(count);
  for (int i = 0; i < count; ++i) {
    ps[i].h = hs[i];
    ps[i].piv = piv;
  }
  // problems of one tile size run together (the ARA kernels take one m)
  std::vector<int> ms;
  for (int i = 0; i < count; ++i)
    if (std::find(ms.begin(), ms.end(), hs[i]->m) == ms.end()) ms.push_back(hs[i]->m);
  tlr_status first = TLR_OK;
  for (int m : ms) {
    std::vector<int> idx;
    for (int i = 0; i < count; ++i)
      if (hs[i]->m == m) idx.push_back(i);
    const tlr_status s = factorize_group(ps, eps, o, ldl, st, idx);
    if (s < 0) {
      // a failure part way (allocation, launch): let the queued work of
      // both streams and of the side worker finish before the handles are
      // touched again, and leave them without a factor
      for (int i : idx) {
        Handle* h = hs[i];
        if (h->worker) (void)h->worker->wait();
        (void)hipStreamSynchronize(h->stream);
        if (h->side) (void)hipStreamSynchronize(h->side);
        release_retired(h);
        h->stage.used = 0;
        h->factored = 0;
      }
      return s;
    }
    if (first == TLR_OK && s != TLR_OK) first = s;
  }
  return first;
}

tlr_status factorize(Handle* h, double eps, const tlr_opts& o, tlr_stats* st, bool ldl, bool piv) {
  return factorize_batch(&h, 1, &eps, o, st, ldl, piv);
}

}  // namespace tlr
