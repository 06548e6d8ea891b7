// SVD post-recompression of the low rank tiles of the input or of the
// factor (Section 6.2): every tile U V^T (U with orthonormal columns) is
// replaced by its truncated SVD at an absolute 2-norm threshold, which
// lowers its rank to the smallest one that threshold allows.
//
// Per tile, with batched GEMMs and the batched Jacobi eigensolver of
// recompress.hip: G_1 = V^T V and its eigenvectors W_1; V_1 = V W_1 and the
// eigenvectors W_2 of G_2 = V_1^T V_1 in descending order, which resolve
// the singular values to full relative accuracy (the second pass works on
// columns that are already orthogonal); r = #{sqrt(lambda_j) > tau};
// W = W_1 W_2(:, 1:r); U' = U W and V' = V W into a staging buffer; a copy
// to the tile's new place.  Tiles are visited in storage order (block
// row by block row, each row's tiles in the order of their columns), a new
// offset never exceeds the old one and a tile's new columns end before the
// next tile's old ones begin, so the panels are compacted in place.  A last
// pass moves every panel into storage of its new width.
#include <algorithm>
#include <cmath>

#include "host.h"

namespace tlr {

namespace {

struct RTile {
  int i, j, q;
  const double* u;    // old columns (m x q)
  const double* v;
  long long off;      // old offset (sort key)
};

// Bytes of the per-chunk buffers a tile needs: G_1, G_2, the combined W,
// the solver's workspace (global-memory class only), two result doubles and
// its products (at most q columns of U and V).
size_t tile_bytes(int m, int q) {
  const size_t qq = (size_t)q * q;
  return sizeof(double) * (3 * qq + (q > kEigLdsLarge ? qq : 0) + 2 + 2 * (size_t)m * q);
}

// Absolute rotation threshold of the first pass, relative to the largest
// diagonal entry: the Gram matrix's own rounding level.
constexpr double kPass1Abs = 1e-14;

}  // namespace

tlr_status recompress(Handle* h, int which, double tau) {
  const int m = h->m, nb = h->nb;
  const bool fac = which == TLR_FACTOR;
  std::vector<RTile> tiles;
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < i; ++j) {
      const int q = fac ? h->lr(i, j) : h->ar(i, j);
      const long long off = fac ? h->lo(i, j) : h->a_off[(size_t)i * nb + j];
      tiles.push_back(RTile{i, j, q, q > 0 ? (fac ? h->ul(i, j) : h->ua(i, j)) : nullptr,
                            q > 0 ? (fac ? h->vl(i, j) : h->va(i, j)) : nullptr, off});
    }
  // storage order: the factor's panels are per block row, the input's arena
  // is one row-major sequence, so both are ordered by block row and then by
  // offset; ties (rank-0 tiles) by column
  std::stable_sort(tiles.begin(), tiles.end(), [](const RTile& a, const RTile& b) {
    if (a.i != b.i) return a.i < b.i;
    if (a.off != b.off) return a.off < b.off;
    return a.j < b.j;
  });

  // chunks of tiles whose buffers fit the budget (at least one tile each):
  // every chunk costs two solver launches as long as its slowest tile, so
  // the budget is generous (N = 131072 with ranks near 14 fits one chunk)
  const size_t budget = (size_t)4 << 30;
  std::vector<size_t> cuts{0};
  size_t acc = 0, chunk_max = 0;
  for (size_t t = 0; t < tiles.size(); ++t) {
    const size_t b = tile_bytes(m, tiles[t].q);
    if (acc > 0 && acc + b > budget) {
      cuts.push_back(t);
      chunk_max = std::max(chunk_max, acc);
      acc = 0;
    }
    acc += b;
  }
  chunk_max = std::max(chunk_max, acc);
  cuts.push_back(tiles.size());

  TLR_TRY(h->init_streams());
  // every buffer is allocated before the first tile changes
  void* work = nullptr;
  TLR_TRY(h->mem.get(&work, std::max<size_t>(chunk_max, 64)));
  std::vector<double> res_host;
  std::vector<int> nrank((size_t)nb * nb, 0);
  std::vector<long long> noff((size_t)nb * nb, -1);
  std::vector<double> nfro((size_t)nb * nb, 0.0);
  std::vector<long long> roff(nb, 0);   // factor: running offset per block row
  long long acol = 0;                   // input: running arena column
  tlr_status st = TLR_OK;

  for (size_t c = 0; c + 1 < cuts.size() && st == TLR_OK; ++c) {
    const size_t t0 = cuts[c], t1 = cuts[c + 1], nt = t1 - t0;
    // buffer layout of the chunk: results, then per tile G_1, G_2, W, the
    // solver's workspace, U', V'
    double* res = static_cast<double*>(work);
    double* p = res + 2 * nt;
    std::vector<double*> G(nt, nullptr), G2(nt, nullptr), WC(nt, nullptr), W(nt, nullptr),
        PU(nt, nullptr), PV(nt, nullptr);
    for (size_t t = 0; t < nt; ++t) {
      const int q = tiles[t0 + t].q;
      G[t] = p;
      p += (size_t)q * q;
      G2[t] = p;
      p += (size_t)q * q;
      WC[t] = p;
      p += (size_t)q * q;
      if (q > kEigLdsLarge) {
        W[t] = p;
        p += (size_t)q * q;
      }
      PU[t] = p;
      p += (size_t)m * q;
      PV[t] = p;
      p += (size_t)m * q;
    }
    GemmBatch gram(true, false), rot(false, false), gram2(true, false);
    std::vector<EigDesc> ed[4], ed2[4];
    std::vector<CopyDesc> keep;   // tiles above the solver's rank limit
    for (size_t t = 0; t < nt; ++t) {
      const RTile& r = tiles[t0 + t];
      const int cls = eig_class(r.q);
      if (r.q == 0) continue;
      if (cls < 0) {
        keep.push_back(CopyDesc{r.u, PU[t], m, r.q, m, m});
        keep.push_back(CopyDesc{r.v, PV[t], m, r.q, m, m});
        continue;
      }
      gram.add(r.q, r.q, m, r.v, m, r.v, m, G[t], r.q, 1.0, 0.0);
      ed[cls].push_back(EigDesc{G[t], W[t], res + 2 * t, r.q});
      rot.add(m, r.q, r.q, r.v, m, G[t], r.q, PV[t], m, 1.0, 0.0);        // V_1 = V W_1
      gram2.add(r.q, r.q, m, PV[t], m, PV[t], m, G2[t], r.q, 1.0, 0.0);   // G_2 = V_1^T V_1
      ed2[cls].push_back(EigDesc{G2[t], W[t], res + 2 * t, r.q});
    }
    // the solver classes of a pass: the large ones (a few hundred tiles next
    // to the diagonal, one workgroup per CU) on the second stream, beside
    // the small ones on the caller's stream, then joined
    auto eig = [&](std::vector<EigDesc>* sets, double abs_scale) -> tlr_status {
      const bool fork = !sets[2].empty() || !sets[3].empty();
      if (fork) {
        TLR_HIP(hipEventRecord(h->ev_fork, h->stream));
        TLR_HIP(hipStreamWaitEvent(h->side, h->ev_fork, 0));
      }
      for (int cls = 3; cls >= 0; --cls) {
        if (sets[cls].empty()) continue;
        hipStream_t s = cls >= 2 ? h->side : h->stream;
        void* d = nullptr;
        TLR_TRY(h->stage.upload(h, sets[cls].data(), sizeof(EigDesc) * sets[cls].size(), &d, s));
        const hipError_t e = launch_sym_eig((const EigDesc*)d, (int)sets[cls].size(), cls, tau,
                                            abs_scale, s);
        if (e != hipSuccess) {
          set_error("launch_sym_eig: %s", hipGetErrorString(e));
          return TLR_ERR_DEVICE;
        }
      }
      if (fork) {
        TLR_HIP(hipEventRecord(h->ev_join, h->side));
        TLR_HIP(hipStreamWaitEvent(h->stream, h->ev_join, 0));
      }
      return TLR_OK;
    };
    if ((st = gram.run(h)) != TLR_OK) break;
    if ((st = eig(ed, kPass1Abs)) != TLR_OK) break;
    if ((st = rot.run(h)) != TLR_OK) break;
    if ((st = gram2.run(h)) != TLR_OK) break;
    if ((st = eig(ed2, 0.0)) != TLR_OK) break;
    res_host.assign(2 * nt, 0.0);
    if (hipMemcpyAsync(res_host.data(), res, sizeof(double) * 2 * nt, hipMemcpyDeviceToHost,
                       h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
      set_error("recompress: result read-back failed");
      st = TLR_ERR_DEVICE;
      break;
    }
    // W = W_1 W_2(:, 1:r), U' = U W, V' = V W, then every tile to its new place
    GemmBatch comb(false, false), prod(false, false);
    std::vector<CopyDesc> place;
    int maxc = 1;
    for (size_t t = 0; t < nt; ++t) {
      const RTile& r = tiles[t0 + t];
      const size_t ij = (size_t)r.i * nb + r.j;
      int nr = 0;
      double fro2 = 0.0;
      if (r.q > 0 && eig_class(r.q) < 0) {
        nr = r.q;
        fro2 = -1.0;   // unknown: kept from before
      } else if (r.q > 0) {
        nr = (int)res_host[2 * t];
        fro2 = res_host[2 * t + 1];
        comb.add(r.q, nr, r.q, G[t], r.q, G2[t], r.q, WC[t], r.q, 1.0, 0.0);
        prod.add(m, nr, r.q, r.u, m, WC[t], r.q, PU[t], m, 1.0, 0.0);
        prod.add(m, nr, r.q, r.v, m, WC[t], r.q, PV[t], m, 1.0, 0.0);
      }
      long long& run = fac ? roff[r.i] : acol;
      nrank[ij] = nr;
      noff[ij] = run;
      nfro[ij] = fro2 >= 0.0 ? std::sqrt(fro2) : (fac && !h->l_fro.empty() ? h->l_fro[ij] : 0.0);
      if (nr > 0) {
        double* base_u = fac ? h->UL[r.i] : h->UA;
        double* base_v = fac ? h->VL[r.i] : h->VA;
        place.push_back(CopyDesc{PU[t], base_u + (size_t)run * m, m, nr, m, m});
        place.push_back(CopyDesc{PV[t], base_v + (size_t)run * m, m, nr, m, m});
        maxc = std::max(maxc, nr);
      }
      run += nr;
    }
    if (!keep.empty()) {
      void* d = nullptr;
      if ((st = h->stage.upload(h, keep.data(), sizeof(CopyDesc) * keep.size(), &d)) != TLR_OK) break;
      int kc = 1;
      for (const CopyDesc& k : keep) kc = std::max(kc, k.cols);
      if (launch_copy_batched((const CopyDesc*)d, (int)keep.size(), kc, h->stream) != hipSuccess) {
        st = TLR_ERR_DEVICE;
        break;
      }
    }
    if ((st = comb.run(h)) != TLR_OK) break;
    if ((st = prod.run(h)) != TLR_OK) break;
    if (!place.empty()) {
      void* d = nullptr;
      if ((st = h->stage.upload(h, place.data(), sizeof(CopyDesc) * place.size(), &d)) != TLR_OK)
        break;
      if (launch_copy_batched((const CopyDesc*)d, (int)place.size(), maxc, h->stream) != hipSuccess) {
        set_error("recompress: panel copy launch failed");
        st = TLR_ERR_DEVICE;
        break;
      }
    }
    // the chunk's buffers are reused by the next chunk
    if ((st = h->sync()) != TLR_OK) break;
  }
  h->mem.put(work);
  if (st != TLR_OK) {
    // tiles of finished chunks have moved: the representation is undefined
    if (fac) free_factor(h);
    return st;
  }

  // storage of the new widths (kept as it is when the allocation fails: the
  // compacted content is valid either way)
  if (fac) {
    for (int i = 0; i < nb; ++i) {
      const long long w = roff[i];
      const int nc = (int)((std::max<long long>(w, 1) + 31) & ~31LL);
      if (nc >= h->cap[i]) continue;
      void* u = nullptr;
      void* v = nullptr;
      if (h->mem.get(&u, sizeof(double) * (size_t)m * nc) != TLR_OK) continue;
      if (h->mem.get(&v, sizeof(double) * (size_t)m * nc) != TLR_OK) {
        h->mem.put(u);
        continue;
      }
      if (w > 0) {
        TLR_HIP(hipMemcpyAsync(u, h->UL[i], sizeof(double) * (size_t)m * w, hipMemcpyDeviceToDevice,
                               h->stream));
        TLR_HIP(hipMemcpyAsync(v, h->VL[i], sizeof(double) * (size_t)m * w, hipMemcpyDeviceToDevice,
                               h->stream));
      }
      TLR_TRY(h->sync());
      h->mem.put(h->UL[i]);
      h->mem.put(h->VL[i]);
      h->UL[i] = (double*)u;
      h->VL[i] = (double*)v;
      h->cap[i] = nc;
    }
    // the low-precision panel copies serve the factorization's sampling only
    for (float* q : h->UL32) h->mem.put(q);
    for (unsigned short* q : h->UL16) h->mem.put(q);
    h->UL32.assign(nb, nullptr);
    h->UL16.assign(nb, nullptr);
    for (int i = 0; i < nb; ++i) h->R[i] = (int)roff[i];
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < i; ++j) {
        const size_t ij = (size_t)i * nb + j;
        h->l_rank[ij] = nrank[ij];
        h->l_off[ij] = noff[ij];
      }
    h->l_fro = nfro;
  } else {
    if (acol < h->a_cols) {
      void* u = nullptr;
      void* v = nullptr;
      const size_t cols = (size_t)std::max<long long>(acol, 1);
      if (h->mem.get(&u, sizeof(double) * cols * m) == TLR_OK) {
        if (h->mem.get(&v, sizeof(double) * cols * m) == TLR_OK) {
          if (acol > 0) {
            TLR_HIP(hipMemcpyAsync(u, h->UA, sizeof(double) * (size_t)acol * m,
                                   hipMemcpyDeviceToDevice, h->stream));
            TLR_HIP(hipMemcpyAsync(v, h->VA, sizeof(double) * (size_t)acol * m,
                                   hipMemcpyDeviceToDevice, h->stream));
          }
          TLR_TRY(h->sync());
          h->mem.put(h->UA);
          h->mem.put(h->VA);
          h->UA = (double*)u;
          h->VA = (double*)v;
        } else {
          h->mem.put(u);
        }
      }
    }
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < i; ++j) {
        const size_t ij = (size_t)i * nb + j;
        h->a_rank[ij] = nrank[ij];
        h->a_off[ij] = noff[ij];
      }
    h->a_cols = acol;
    h->a_fro.clear();
  }
  return h->sync();
}

}  // namespace tlr
