// Products and solves with TLR matrices (Section 4.4): the TLR matrix-vector
// product of the input matrix, the 2-norm estimate it serves, and the
// triangular solves with the factor (Algorithm "TLR Triangular Solve" and
// its transpose).
#include <algorithm>
#include <cmath>

#include "host.h"

namespace tlr {

// Copy N x nrhs (ld) into the padded nb*m x nrhs work vector (zero padding),
// or back.
static tlr_status pad_in(Handle* h, const double* X, long long ldx, int nrhs, double* Xp) {
  const long long np = (long long)h->nb * h->m;
  TLR_HIP(launch_fill(Xp, np * nrhs, 0.0, h->stream));
  CopyDesc cd{X, Xp, (int)h->N, nrhs, (int)ldx, (int)np};
  void* d = nullptr;
  TLR_TRY(h->stage.upload(h, &cd, sizeof cd, &d));
  TLR_HIP(launch_copy_batched((const CopyDesc*)d, 1, nrhs, h->stream));
  return TLR_OK;
}

static tlr_status pad_out(Handle* h, const double* Xp, int nrhs, double* Y, long long ldy) {
  const long long np = (long long)h->nb * h->m;
  CopyDesc cd{Xp, Y, (int)h->N, nrhs, (int)np, (int)ldy};
  void* d = nullptr;
  TLR_TRY(h->stage.upload(h, &cd, sizeof cd, &d));
  TLR_HIP(launch_copy_batched((const CopyDesc*)d, 1, nrhs, h->stream));
  return TLR_OK;
}

tlr_status matvec(Handle* h, int nrhs, const double* X, long long ldx, double* Y, long long ldy) {
  const int m = h->m, nb = h->nb;
  const long long np = (long long)nb * m;
  Work& w = h->ws;
  TLR_TRY(w.omega.ensure(h->mem, sizeof(double) * np * nrhs * 2));
  TLR_TRY(w.T.ensure(h->mem, sizeof(double) * (size_t)std::max(h->a_cols, 1LL) * nrhs * 2));
  double* Xp = w.omega.as<double>();
  double* Yp = Xp + np * nrhs;
  double* Tl = w.T.as<double>();
  double* Tu = Tl + (size_t)std::max(h->a_cols, 1LL) * nrhs;
  const int ldt = (int)std::max(h->a_cols, 1LL);
  TLR_TRY(pad_in(h, X, ldx, nrhs, Xp));
  {
    GemmBatch dg(false, false);
    for (int i = 0; i < nb; ++i)
      dg.add(m, nrhs, m, h->diagA(i), m, Xp + (size_t)i * m, (int)np, Yp + (size_t)i * m, (int)np,
             1.0, 0.0);
    TLR_TRY(dg.run(h));
  }
  if (h->a_cols > 0) {
    GemmBatch tl(true, false), tu(true, false);
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < i; ++j) {
        const int a = h->ar(i, j);
        if (a == 0) continue;
        const long long off = h->a_off[(size_t)i * nb + j];
        tl.add(a, nrhs, m, h->va(i, j), m, Xp + (size_t)j * m, (int)np, Tl + off, ldt, 1.0, 0.0);
        tu.add(a, nrhs, m, h->ua(i, j), m, Xp + (size_t)i * m, (int)np, Tu + off, ldt, 1.0, 0.0);
      }
    TLR_TRY(tl.run(h));
    TLR_TRY(tu.run(h));
    // lower part: row i's tiles are adjacent in the arena -> one product per row
    GemmBatch lo(false, false);
    for (int i = 1; i < nb; ++i) {
      long long K = 0;
      for (int j = 0; j < i; ++j) K += h->ar(i, j);
      if (K == 0) continue;
      const long long off = h->a_off[(size_t)i * nb + 0];
      lo.add(m, nrhs, (int)K, h->UA + (size_t)off * m, m, Tl + off, ldt, Yp + (size_t)i * m, (int)np,
             1.0, 1.0);
    }
    TLR_TRY(lo.run(h));
    // upper part: tiles (j + d, j) of one sub-diagonal d update distinct rows
    for (int d = 1; d < nb; ++d) {
      GemmBatch up(false, false);
      for (int j = 0; j + d < nb; ++j) {
        const int i = j + d, a = h->ar(i, j);
        if (a == 0) continue;
        const long long off = h->a_off[(size_t)i * nb + j];
        up.add(m, nrhs, a, h->va(i, j), m, Tu + off, ldt, Yp + (size_t)j * m, (int)np, 1.0, 1.0);
      }
      TLR_TRY(up.run(h));
    }
  }
  TLR_TRY(pad_out(h, Yp, nrhs, Y, ldy));
  return TLR_OK;
}

tlr_status estimate_norm(Handle* h, double* out) {
  // power iteration on the TLR input (20 steps from a Gaussian start), the
  // norms and the normalisation on the device; one read-back at the end
  const long long n = h->N;
  void* xv = nullptr;
  TLR_TRY(h->mem.get(&xv, sizeof(double) * (n * 2 + 2 + 256)));
  double* x = (double*)xv;
  double* y = x + n;
  double* nrm = y + n;          // [0] ||x_0||, [1] ||A x|| of the last step
  double* parts = nrm + 2;
  tlr_status st = TLR_OK;
  double host[2] = {0.0, 0.0};
  const int steps = 20;
  auto body = [&]() -> tlr_status {
    TLR_HIP(launch_randn(x, (int)n, 1, (int)n, 0x4e6f726dULL, 0, 0, 0, h->stream));
    TLR_HIP(launch_norm2(x, n, nrm, parts, h->stream));
    for (int it = 0; it < steps; ++it) {
      TLR_TRY(matvec(h, 1, x, n, y, n));
      TLR_HIP(launch_norm2(y, n, nrm + 1, parts, h->stream));
      TLR_HIP(launch_scale_by(y, n, nrm + 1, x, h->stream));
    }
    TLR_HIP(hipMemcpyAsync(host, nrm, sizeof(double) * 2, hipMemcpyDeviceToHost, h->stream));
    return h->sync();
  };
  st = body();
  h->mem.put(xv);
  // after the first step x is normalised, so the last ||A x|| is the estimate
  // (the start vector's norm enters only when a single step ran)
  *out = steps > 1 ? host[1] : (host[0] > 0.0 ? host[1] / host[0] : 0.0);
  return st;
}

// Rows of the per-column products V^T x (forward sweep, the tiles of one
// column) and U^T x (backward sweep, one block row's panel).
static long long solve_tcap(const Handle* h) {
  const int nb = h->nb;
  long long tcap = 0;
  for (int k = 0; k < nb; ++k) {
    long long s = 0;
    for (int i = k + 1; i < nb; ++i) s += h->lr(i, k);
    tcap = std::max(tcap, std::max(s, (long long)h->R[k]));
  }
  return std::max(tcap, 1LL);
}

size_t solve_workspace(const Handle* h, int nrhs) {
  const long long np = (long long)h->nb * h->m;
  // a pivoted factor also needs the right-hand sides in its block order
  const long long perm = h->fperm.empty() ? 0 : np;
  return (size_t)(np + perm + h->m + solve_tcap(h)) * (size_t)std::max(nrhs, 0);
}

// Block rows of the padded right-hand sides between the original order
// (X) and the pivoted factor's order (Xq, position t = block perm[t]).
static tlr_status permute_blocks(Handle* h, double* X, double* Xq, int nrhs, bool to_factor) {
  const int m = h->m, nb = h->nb;
  const int ld = nb * m;
  std::vector<CopyDesc> cd;
  for (int t = 0; t < nb; ++t) {
    double* orig = X + (size_t)h->fperm[t] * m;
    double* pos = Xq + (size_t)t * m;
    cd.push_back(CopyDesc{to_factor ? orig : pos, to_factor ? pos : orig, m, nrhs, ld, ld});
  }
  void* d = nullptr;
  TLR_TRY(h->stage.upload(h, cd.data(), sizeof(CopyDesc) * cd.size(), &d));
  TLR_HIP(launch_copy_batched((const CopyDesc*)d, nb, nrhs, h->stream));
  return TLR_OK;
}

tlr_status solve(Handle* h, int nrhs, double* B, long long ldb) {
  TLR_TRY(h->ws.omega.ensure(h->mem, sizeof(double) * std::max<size_t>(solve_workspace(h, nrhs), 1)));
  return solve_in(h, nrhs, B, ldb, h->ws.omega.as<double>());
}

tlr_status solve_in(Handle* h, int nrhs, double* B, long long ldb, double* work) {
  const int m = h->m, nb = h->nb;
  const long long np = (long long)nb * m;
  const bool ldl = h->factored == 2;
  const long long tcap = solve_tcap(h);
  const bool piv = !h->fperm.empty();
  double* Xo = work;                    // padded N x nrhs, original block order
  double* Xp = piv ? Xo + np * nrhs : Xo;   // the factor's block order
  double* tk = Xp + np * nrhs;          // m x nrhs
  double* T = tk + (size_t)m * nrhs;    // tcap x nrhs
  const int ldx = (int)np;
  TLR_TRY(pad_in(h, B, ldb, nrhs, Xo));
  if (piv) TLR_TRY(permute_blocks(h, Xo, Xp, nrhs, true));
  auto apply_inv = [&](int k, bool trans) -> tlr_status {
    double* xk = Xp + (size_t)k * m;
    GemmBatch g(trans, false);
    g.add(m, nrhs, m, h->invL(k), m, xk, ldx, tk, m, 1.0, 0.0, trans ? GEMM_TRIU_A : GEMM_TRIL_A);
    TLR_TRY(g.run(h));
    CopyDesc cd{tk, xk, m, nrhs, m, ldx};
    void* d = nullptr;
    TLR_TRY(h->stage.upload(h, &cd, sizeof cd, &d));
    TLR_HIP(launch_copy_batched((const CopyDesc*)d, 1, nrhs, h->stream));
    return TLR_OK;
  };
  // forward sweep: x_k = L_kk^{-1} x_k, then x_i -= U_ik (V_ik^T x_k) for i > k
  for (int k = 0; k < nb; ++k) {
    double* xk = Xp + (size_t)k * m;
    TLR_TRY(apply_inv(k, false));
    GemmBatch t(true, false), u(false, false);
    long long off = 0;
    for (int i = k + 1; i < nb; ++i) {
      const int r = h->lr(i, k);
      if (r == 0) continue;
      t.add(r, nrhs, m, h->vl(i, k), m, xk, ldx, T + off, (int)tcap, 1.0, 0.0);
      u.add(m, nrhs, r, h->ul(i, k), m, T + off, (int)tcap, Xp + (size_t)i * m, ldx, -1.0, 1.0);
      off += r;
    }
    TLR_TRY(t.run(h));
    TLR_TRY(u.run(h));
  }
  if (ldl) TLR_HIP(launch_scale_rows(Xp, ldx, Xp, ldx, h->Dv, (int)np, nrhs, true, h->stream));
  // backward sweep with L^T: x_k = L_kk^{-T} x_k, then x_j -= V_kj (U_kj^T x_k)
  for (int k = nb - 1; k >= 0; --k) {
    double* xk = Xp + (size_t)k * m;
    TLR_TRY(apply_inv(k, true));
    const int Rk = h->R[k];
    if (Rk == 0) continue;
    GemmBatch t(true, false), v(false, false);
    t.add(Rk, nrhs, m, h->UL[k], m, xk, ldx, T, (int)tcap, 1.0, 0.0);
    for (int j = 0; j < k; ++j) {
      const int r = h->lr(k, j);
      if (r == 0) continue;
      v.add(m, nrhs, r, h->vl(k, j), m, T + h->lo(k, j), (int)tcap, Xp + (size_t)j * m, ldx, -1.0,
            1.0);
    }
    TLR_TRY(t.run(h));
    TLR_TRY(v.run(h));
  }
  if (piv) TLR_TRY(permute_blocks(h, Xo, Xp, nrhs, false));
  TLR_TRY(pad_out(h, Xo, nrhs, B, ldb));
  return h->sync();
}

}  // namespace tlr
