// Data-movement and elementwise kernels of the TLR library: batched panel
// copies ("updateTiles": appending the new column of low rank factors to the
// block-row panels), the diagonal tile set-up with the optional shift
// (Section 5.1), row scaling by a diagonal (the D factors of LDL^T,
// Section 5.3), zeroing of a strict triangle, and the covariance tile
// generator of the Section 6 test matrices.
#include "mfma_tiles.h"
#include "tlr_internal.h"

namespace tlr {

namespace {

// One workgroup per (descriptor, 8-column slab); each thread copies rows.
// The packed FP32 / BF16 copies take the layout of pack_index.
__global__ __launch_bounds__(256) void k_copy_batched(const CopyDesc* __restrict__ descs) {
  const CopyDesc d = descs[blockIdx.y];
  const int c0 = blockIdx.x * 8;
  if (c0 >= d.cols) return;
  const int c1 = min(d.cols, c0 + 8);
  const int nrb = (d.rows + 15) / 16;
  for (int c = c0; c < c1; ++c)
    for (int r = threadIdx.x; r < d.rows; r += blockDim.x) {
      const double v = d.src[r + (size_t)c * d.lds];
      d.dst[r + (size_t)c * d.ldd] = v;
      if (d.dst32) d.dst32[pack_index(r, d.pcol + c, nrb, Pack<1>::K, Pack<1>::V)] = (float)v;
      if (d.dst16) d.dst16[pack_index(r, d.pcol + c, nrb, Pack<2>::K, Pack<2>::V)] = bf16_bits(v);
    }
}

// Frobenius norms: one workgroup per block, a fixed-order tree reduction.
// Thread t takes the entries t, t + 256, ... of the block in column-major
// order (32-bit indices: a block has at most 2^31 entries), eight loads in
// flight before their squares are added; the norm also goes to pinned host
// memory when the descriptor names it (stores at system scope).
__global__ __launch_bounds__(256) void k_fro_norms(const NormDesc* __restrict__ descs) {
  __shared__ double red[256];
  const NormDesc d = descs[blockIdx.x];
  const int n = d.rows * d.cols;
  constexpr int U = 8;
  double s = 0.0;
  for (int e0 = threadIdx.x; e0 < n; e0 += 256 * U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + 256 * u;
      v[u] = (e < n) ? d.p[(e % d.rows) + (size_t)(e / d.rows) * d.ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) s = fma(v[u], v[u], s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double f = sqrt(red[0]);
    *d.out = f;
    if (d.host)
      __hip_atomic_store((unsigned long long*)d.host, (unsigned long long)__double_as_longlong(f),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Partial sums of the squared Frobenius norms of symmetric m x m tiles held
// by their lower triangle: workgroup (t, g) adds columns g, g + G, g + 2G, ...
// of tile t (every entry below the diagonal twice) and stores the sum at
// out[t G + g]; the caller adds the G partials of a tile in order.
__global__ __launch_bounds__(256) void k_sym_fro_parts(const double* const* __restrict__ tiles,
                                                       int m, int ld, int G, double* out) {
  __shared__ double red[256];
  const double* p = tiles[blockIdx.x / G];
  const int g = blockIdx.x % G;
  double s = 0.0;
  for (int c = g; c < m; c += G) {
    const double* col = p + (size_t)c * ld;
    for (int r = c + (int)threadIdx.x; r < m; r += 256) {
      const double v = col[r];
      s += (r == c ? 1.0 : 2.0) * (v * v);
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ void k_copy_shift(const double* src, double* dst, int m, int nreal, double shift) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)m * m) return;
  const int r = (int)(e % m), c = (int)(e / m);
  double v = src[e];
  if (r == c && r < nreal) v += shift;
  dst[e] = v;
}

__global__ void k_scale_rows(const double* in, int ldi, double* out, int ldo, const double* dg,
                             int rows, int cols, int inverse) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)rows * cols) return;
  const int r = (int)(e % rows), c = (int)(e / rows);
  const double v = in[r + (size_t)c * ldi];
  out[r + (size_t)c * ldo] = inverse ? v / dg[r] : v * dg[r];
}

// W(:, c) = V(:, c) * D_{colj[c]} (rows scaled by the pivots of the column's
// block: the V_kj D_j of a whole LDL^T row panel in one launch).
__global__ void k_scale_panel(const double* __restrict__ V, int ldv, double* __restrict__ W,
                              int ldw, int m, int ncols, const int* __restrict__ colj,
                              const double* __restrict__ Dv) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)m * ncols) return;
  const int r = (int)(e % m), c = (int)(e / m);
  W[r + (size_t)c * ldw] = V[r + (size_t)c * ldv] * Dv[(size_t)colj[c] * m + r];
}

// p[0 .. n) = v (a fill kernel rather than a memset, so the stream holds
// only kernel launches)
__global__ void k_fill(double* p, long long n, double v) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

// 64 * u * ||A||_F (the LDL^T zero-pivot tolerance) for an m x m tile held
// by its lower triangle (the strict upper part may be stale), in two
// launches: workgroup g of kPivotParts adds columns g, g + kPivotParts, ...
// (entries below the diagonal twice) into parts[g]; one workgroup then adds
// the partials in a fixed tree order.
constexpr int kPivotParts = 256;

__global__ __launch_bounds__(256) void k_pivot_tol_parts(const double* A, int lda, int m,
                                                         double* parts) {
  __shared__ double red[256];
  double s = 0.0;
  for (int c = blockIdx.x; c < m; c += kPivotParts) {
    const double* col = A + (size_t)c * lda;
    for (int r = c + (int)threadIdx.x; r < m; r += 256) {
      const double v = col[r];
      s += (r == c ? 1.0 : 2.0) * (v * v);
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kPivotParts) void k_pivot_tol_final(const double* parts,
                                                                 double* tol) {
  __shared__ double red[kPivotParts];
  red[threadIdx.x] = parts[threadIdx.x];
  __syncthreads();
  for (int o = kPivotParts / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *tol = 64.0 * 1.1102230246251565e-16 * sqrt(red[0]);
}

// Covariance tiles: out(r, c) = k(|x_{r0+r} - x_{c0+c}|) (+ diag_add on the
// global diagonal); identity where the row or column lies in the padding.
__global__ __launch_bounds__(256) void k_gen_tiles(const GenDesc* __restrict__ descs,
                                                   const double* __restrict__ pts, int dim,
                                                   long long n, int m, int kernel, double ell,
                                                   double diag_add, const double* __restrict__ src,
                                                   long long lds) {
  const GenDesc d = descs[blockIdx.y];
  const int c = blockIdx.x;          // one column per workgroup x
  const long long gc = d.c0 + c;
  double xc[3] = {0.0, 0.0, 0.0};
  if (gc < n && kernel >= 0)
    for (int t = 0; t < dim; ++t) xc[t] = pts[gc * dim + t];
  const double inv_ell = 1.0 / ell;
  const double s3 = 1.7320508075688772935274463415059;
  for (int r = threadIdx.x; r < m; r += blockDim.x) {
    const long long gr = d.r0 + r;
    double v;
    if (gr >= n || gc >= n) {
      v = (gr == gc) ? 1.0 : 0.0;
    } else if (kernel < 0) {
      // lower triangle of the dense input, mirrored above the diagonal
      v = (gr >= gc) ? src[gr + gc * lds] : src[gc + gr * lds];
    } else {
      double s = 0.0;
      for (int t = 0; t < dim; ++t) {
        const double df = pts[gr * dim + t] - xc[t];
        s += df * df;
      }
      const double dist = sqrt(s);
      if (kernel == 0) {
        v = exp(-dist * inv_ell);
      } else {
        const double q = s3 * dist * inv_ell;
        v = (1.0 + q) * exp(-q);
      }
      if (gr == gc) v += diag_add;
    }
    d.out[r + (size_t)c * d.ld] = v;
  }
}

}  // namespace

hipError_t launch_copy_batched(const CopyDesc* d, int n, int max_cols, hipStream_t s) {
  if (n <= 0 || max_cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_batched, dim3((max_cols + 7) / 8, n), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_fro_norms(const NormDesc* d, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fro_norms, dim3(n), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_sym_fro_parts(const double* const* tiles, int n, int m, int ld, int G,
                                double* out, hipStream_t s) {
  if (n <= 0 || G <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sym_fro_parts, dim3((unsigned)(n * G)), dim3(256), 0, s, tiles, m, ld, G,
                     out);
  return hipGetLastError();
}

hipError_t launch_copy_shift(const double* src, double* dst, int m, int nreal, double shift,
                             hipStream_t s) {
  const long long n = (long long)m * m;
  hipLaunchKernelGGL(k_copy_shift, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, m,
                     nreal, shift);
  return hipGetLastError();
}

hipError_t launch_scale_rows(const double* in, int ldi, double* out, int ldo, const double* dg,
                             int rows, int cols, bool inverse, hipStream_t s) {
  const long long n = (long long)rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, ldi, out,
                     ldo, dg, rows, cols, inverse ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_scale_panel(const double* V, int ldv, double* W, int ldw, int m, int ncols,
                              const int* colj, const double* Dv, hipStream_t s) {
  const long long n = (long long)m * ncols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_panel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, V, ldv, W,
                     ldw, m, ncols, colj, Dv);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, long long n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// ||x||_2 of a vector: kPivotParts grid-stride partial sums of squares,
// then one workgroup adds them in a fixed tree order (*out on the device).
__global__ __launch_bounds__(256) void k_sumsq_parts(const double* __restrict__ x, long long n,
                                                     double* parts) {
  __shared__ double red[256];
  double s = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * kPivotParts)
    s = fma(x[i], x[i], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kPivotParts) void k_norm_final(const double* parts, double* out) {
  __shared__ double red[kPivotParts];
  red[threadIdx.x] = parts[threadIdx.x];
  __syncthreads();
  for (int o = kPivotParts / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt(red[0]);
}

// x = y / *s (x = y when *s is zero)
__global__ void k_scale_by(const double* __restrict__ y, long long n, const double* s,
                           double* __restrict__ x) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  const double d = *s;
  x[i] = d > 0.0 ? y[i] / d : y[i];
}

hipError_t launch_norm2(const double* x, long long n, double* out, double* parts, hipStream_t s) {
  if (n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sumsq_parts, dim3(kPivotParts), dim3(256), 0, s, x, n, parts);
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kPivotParts), 0, s, parts, out);
  return hipGetLastError();
}

hipError_t launch_scale_by(const double* y, long long n, const double* sc, double* x,
                           hipStream_t s) {
  if (n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scale_by, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, n, sc, x);
  return hipGetLastError();
}

hipError_t launch_pivot_tol(const double* A, int lda, int m, double* tol, hipStream_t s) {
  double* parts = tol + 32;
  hipLaunchKernelGGL(k_pivot_tol_parts, dim3(kPivotParts), dim3(256), 0, s, A, lda, m, parts);
  hipLaunchKernelGGL(k_pivot_tol_final, dim3(1), dim3(kPivotParts), 0, s, parts, tol);
  return hipGetLastError();
}

hipError_t launch_gen_tiles(const GenDesc* d, int ntiles, const double* pts, int dim, long long n,
                            int m, int kernel, double ell, double diag_add, const double* src,
                            long long lds, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (kernel >= 0 && (dim < 1 || dim > 3)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gen_tiles, dim3(m, ntiles), dim3(256), 0, s, d, pts, dim, n, m, kernel, ell,
                     diag_add, src, lds);
  return hipGetLastError();
}

}  // namespace tlr
