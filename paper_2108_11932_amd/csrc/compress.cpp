// Construction of the TLR representation (Section 1): dense diagonal tiles
// and off-diagonal tiles compressed by adaptive randomized approximation
// (Algorithm "Adaptive Randomized Approximation", Section 3.1).  Tiles are
// produced on the device -- generated from the covariance kernel of the
// Section 6 test problems, or copied from a dense matrix -- in batches, and
// the batch is compressed by the same batched ARA with dynamic batching as
// the factorization.  Results are appended to the U/V arenas in row-major
// lower order, which yields the arena offsets of the format directly.
#include <algorithm>

#include "ara_engine.h"

namespace tlr {

static tlr_status grow_arena(Handle* h, long long need_cols, long long* cap_cols) {
  if (need_cols <= *cap_cols) return TLR_OK;
  long long nc = std::max(need_cols, *cap_cols + *cap_cols / 2 + 256);
  void* u = nullptr;
  void* v = nullptr;
  TLR_TRY(h->mem.get(&u, sizeof(double) * (size_t)h->m * nc));
  tlr_status st = h->mem.get(&v, sizeof(double) * (size_t)h->m * nc);
  if (st != TLR_OK) {
    h->mem.put(u);
    return st;
  }
  if (h->a_cols > 0) {
    const size_t bytes = sizeof(double) * (size_t)h->m * h->a_cols;
    TLR_HIP(hipMemcpyAsync(u, h->UA, bytes, hipMemcpyDeviceToDevice, h->stream));
    TLR_HIP(hipMemcpyAsync(v, h->VA, bytes, hipMemcpyDeviceToDevice, h->stream));
  }
  TLR_TRY(h->sync());
  h->mem.put(h->UA);
  h->mem.put(h->VA);
  h->UA = (double*)u;
  h->VA = (double*)v;
  *cap_cols = nc;
  return TLR_OK;
}

tlr_status compress(Handle* h, const double* A, long long lda, const double* pts, int dim,
                    int kernel, double ell, double diag_add, double eps, const tlr_opts& o) {
  const int m = h->m, nb = h->nb, bs = o.bs;
  const int kern = A ? -1 : kernel;
  // diagonal tiles
  {
    std::vector<GenDesc> gd(nb);
    for (int k = 0; k < nb; ++k) gd[k] = GenDesc{h->diagA(k), m, (long long)k * m, (long long)k * m};
    void* dg = nullptr;
    TLR_TRY(h->stage.upload(h, gd.data(), sizeof(GenDesc) * nb, &dg));
    TLR_HIP(launch_gen_tiles((const GenDesc*)dg, nb, pts, dim, h->N, m, kern, ell, diag_add, A, lda,
                             h->stream));
  }
  h->a_rank.assign((size_t)nb * nb, 0);
  h->a_off.assign((size_t)nb * nb, -1);
  h->a_cols = 0;
  h->a_orth = true;   // every tile becomes Q B^T with orthonormal Q
  h->a_fro.clear();
  h->mem.put(h->UA);
  h->mem.put(h->VA);
  h->UA = h->VA = nullptr;
  long long cap_cols = 0;
  TLR_TRY(grow_arena(h, std::max(64LL, (long long)nb * (nb - 1) / 2 * 8), &cap_cols));

  // tiles in row-major lower order, batches bounded by a workspace budget
  std::vector<std::pair<int, int>> tiles;
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < i; ++j) tiles.emplace_back(i, j);
  const size_t per_tile = sizeof(double) * (size_t)m * (2 * (size_t)m + 4 * bs);
  const size_t budget = (size_t)4 << 30;
  int batch = (int)std::max<size_t>(1, budget / per_tile);
  batch = std::min<int>(batch, 4096);
  batch = std::min<int>(batch, std::max<int>(1, (int)tiles.size()));

  AraConfig cfg;
  cfg.m = m;
  cfg.bs = bs;
  cfg.bs_tail = o.bs_tail;
  cfg.tail_active = o.tail_active;
  cfg.qcap = m;
  cfg.tau = eps / o.conv_factor;
  cfg.r_min = o.r_min;
  cfg.strip = o.sample_strip;
  cfg.overlap = (o.flags & TLR_FLAG_SERIAL_SAMPLING) == 0;
  cfg.s_max = 0;
  cfg.seed = o.seed ^ 0xC0FFEEULL;
  AraSlots slots;
  TLR_TRY(ara_slots(h, cfg, batch, &slots));
  Work& w = h->ws;
  TLR_TRY(w.T.ensure(h->mem, sizeof(double) * (size_t)batch * m * m));

  for (size_t b0 = 0, bid = 0; b0 < tiles.size(); b0 += batch, ++bid) {
    const int nt = (int)std::min<size_t>(batch, tiles.size() - b0);
    double* Tt = w.T.as<double>();
    std::vector<GenDesc> gd(nt);
    for (int t = 0; t < nt; ++t) {
      const auto ij = tiles[b0 + t];
      gd[t] = GenDesc{Tt + (size_t)t * m * m, m, (long long)ij.first * m, (long long)ij.second * m};
    }
    void* dg = nullptr;
    TLR_TRY(h->stage.upload(h, gd.data(), sizeof(GenDesc) * nt, &dg));
    TLR_HIP(launch_gen_tiles((const GenDesc*)dg, nt, pts, dim, h->N, m, kern, ell, diag_add, A, lda,
                             h->stream));
    AraSpec spec;
    TLR_TRY(ara_explicit_spec(h, cfg, nt, Tt, m, &spec));
    std::vector<int> order(nt);
    for (int t = 0; t < nt; ++t) order[t] = t;
    AraResult res;
    cfg.stream_id = 0x80000000u + (unsigned)bid;
    TLR_TRY(ara_run(h, cfg, slots, order, spec, &res, nullptr));
    // B = T^T Q for every tile, then append Q and B to the arenas
    long long add = 0;
    for (int t = 0; t < nt; ++t) add += res.q[t];
    TLR_TRY(grow_arena(h, h->a_cols + add, &cap_cols));
    GemmBatch pb(true, false);
    std::vector<CopyDesc> cd;
    int maxc = 0;
    long long col = h->a_cols;
    for (int t = 0; t < nt; ++t) {
      const auto ij = tiles[b0 + t];
      const int q = res.q[t];
      h->a_rank[(size_t)ij.first * nb + ij.second] = q;
      h->a_off[(size_t)ij.first * nb + ij.second] = col;
      if (q > 0) {
        pb.add(m, q, m, Tt + (size_t)t * m * m, m, slots.qb(t), m, h->VA + (size_t)col * m, m, 1.0, 0.0);
        cd.push_back(CopyDesc{slots.qb(t), h->UA + (size_t)col * m, m, q, m, m});
        maxc = std::max(maxc, q);
      }
      col += q;
    }
    TLR_TRY(pb.run(h));
    if (!cd.empty()) {
      void* dcd = nullptr;
      TLR_TRY(h->stage.upload(h, cd.data(), sizeof(CopyDesc) * cd.size(), &dcd));
      TLR_HIP(launch_copy_batched((const CopyDesc*)dcd, (int)cd.size(), maxc, h->stream));
    }
    h->a_cols = col;
    TLR_TRY(h->sync());
  }
  // the tile and basis buffers are sized for the compression batches
  w.T.release(h->mem);
  w.Q.release(h->mem);
  return TLR_OK;
}

}  // namespace tlr
