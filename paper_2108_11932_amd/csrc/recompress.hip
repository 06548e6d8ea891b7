// SVD post-recompression of low rank tiles (Section 6.2): the ARA stops at
// ranks a few percent above the smallest ones its threshold allows, and a
// post-processing pass with the SVD of every low rank tile brings them down
// to that minimum.
//
// A tile U V^T whose U has orthonormal columns has the singular values
// sigma_j = sqrt(lambda_j) of the Gram matrix V^T V = W diag(lambda) W^T,
// and U V^T = (U W) (V W)^T with U W orthonormal and the columns of V W
// orthogonal with norms sigma_j.  Keeping the eigenpairs with sigma_j > tau
// gives the truncated SVD, error sigma_{r+1} <= tau.  The Gram matrices and
// the products with W are batched GEMMs; this file holds the batched
// symmetric eigensolver: cyclic two-sided Jacobi (Golub and Van Loan,
// "Matrix Computations", Section 8.5) with the rotations of one round of a
// round-robin ordering applied in parallel, one workgroup per tile.
//
// The Gram matrix squares the spread of the singular values: from V^T V
// alone, sigma_j carries a relative error near u (sigma_1 / sigma_j)^2.
// The caller therefore runs two passes: the first (an absolute rotation
// threshold, abs_scale > 0) gives W_1, the second diagonalises the Gram
// matrix of V W_1 (whose columns are already orthogonal to working
// accuracy, so its entries carry errors relative to the column norms) with
// the relative threshold, which resolves every sigma_j to a relative error
// near m u, as one-sided Jacobi on V would.
#include "tlr_internal.h"

namespace tlr {

namespace {

constexpr int kSweeps = 40;          // every tile stops after this many sweeps
constexpr double kJacTol = 2.220446049250313e-16;   // 2^-52

// Pair k of round t of a round-robin tournament on n (even) indices: index
// 0 stays, indices 1 .. n-1 sit on a circle that turns one step per round,
// and positions k - 1 and n - 2 - k meet (position n - 2 meets index 0).
// Over the n - 1 rounds every pair meets once.
__device__ __forceinline__ void jac_pair(int n, int t, int k, int& a, int& b) {
  const int c = n - 1;
  if (k == 0) {
    a = 0;
    b = (n - 2 + t) % c + 1;
  } else {
    a = (k - 1 + t) % c + 1;
    b = (n - 2 - k + t) % c + 1;
  }
  if (a > b) {
    const int x = a;
    a = b;
    b = x;
  }
}

struct JacShared {
  double* cs;
  double* sn;
  int* pa;
  int* pb;
  int* flag;
  double* atol;
};

// Diagonalise the symmetric q x q matrix G (ld lg) in place, accumulating
// the rotations in W (ld lw): G_out = W^T G_in W.  A sweep visits every
// pair once; a pair (a, b) is rotated when |g_ab| > 2^-52 sqrt(g_aa g_bb)
// and |g_ab| > abs_scale max_j g_jj, with the rotation of Golub and Van
// Loan's symmetric Schur decomposition of the 2 x 2 block
// (t = sign(theta) / (|theta| + sqrt(1 + theta^2)),
// theta = (g_bb - g_aa) / (2 g_ab)), which zeroes g_ab.  The pairs of a
// round are disjoint, so the round's transformation J^T G J acts on the
// 2 x 2 blocks (pair k1's rows, pair k2's columns) independently:
// block <- R_k1^T block R_k2, one block per work item, together with the
// column pairs of W.  The run ends after a sweep without rotations or
// after kSweeps sweeps; the decision is the workgroup's, so every wave
// leaves the loop together.
// Element (i, j) of G: column-major with leading dimension lg, or (PACKED)
// the upper triangle stored by columns, (i, j) and (j, i) at one place.
template <bool PACKED>
__device__ __forceinline__ size_t gidx(int i, int j, int lg) {
  if (!PACKED) return i + (size_t)j * lg;
  if (i > j) {
    const int x = i;
    i = j;
    j = x;
  }
  return (size_t)j * (j + 1) / 2 + i;
}

template <int NT, bool PACKED = false>
__device__ void jacobi(double* G, int lg, double* W, int lw, int q, double abs_scale,
                       const JacShared& sh) {
  const int tid = threadIdx.x;
  const int n = q + (q & 1), half = n / 2;
  for (int e = tid; e < q * q; e += NT) {
    const int i = e % q, j = e / q;
    W[i + (size_t)j * lw] = i == j ? 1.0 : 0.0;
  }
  if (tid == 0) {
    double g = 0.0;
    for (int j = 0; j < q; ++j) g = fmax(g, fabs(G[gidx<PACKED>(j, j, lg)]));
    *sh.atol = abs_scale * g;
  }
  __syncthreads();
  const double atol = *sh.atol;
  // packed storage holds each block pair once: the blocks k1 <= k2
  const int nblk = PACKED ? half * (half + 1) / 2 : half * half;
  for (int sweep = 0; sweep < kSweeps; ++sweep) {
    if (tid == 0) *sh.flag = 0;
    __syncthreads();
    for (int t = 0; t < n - 1; ++t) {
      for (int k = tid; k < half; k += NT) {
        int a, b;
        jac_pair(n, t, k, a, b);
        double c = 1.0, s = 0.0;
        if (b < q) {
          const double gaa = G[gidx<PACKED>(a, a, lg)], gbb = G[gidx<PACKED>(b, b, lg)];
          const double gab = G[gidx<PACKED>(a, b, lg)];
          if (fabs(gab) > fmax(kJacTol * sqrt(fabs(gaa)) * sqrt(fabs(gbb)), atol)) {
            const double th = (gbb - gaa) / (2.0 * gab);
            const double at = fabs(th);
            // for |theta| beyond 1e150, theta^2 would overflow: t = 1 / (2 theta)
            double tt = at > 1e150 ? 0.5 / at : 1.0 / (at + sqrt(1.0 + th * th));
            if (th < 0.0) tt = -tt;
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            *sh.flag = 1;
          }
        }
        sh.cs[k] = c;
        sh.sn[k] = s;
        sh.pa[k] = a;
        sh.pb[k] = b;
      }
      __syncthreads();
      // blocks of G (k2 fastest: consecutive items share pair k1's rows)
      for (int e = tid; e < nblk; e += NT) {
        int k1, k2;
        if (PACKED) {
          // e = k2 (k2 + 1) / 2 + k1, k1 <= k2
          k2 = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
          while ((k2 + 1) * (k2 + 2) / 2 <= e) ++k2;
          while (k2 * (k2 + 1) / 2 > e) --k2;
          k1 = e - k2 * (k2 + 1) / 2;
        } else {
          k1 = e / half;
          k2 = e - k1 * half;
        }
        const double s1 = sh.sn[k1], s2 = sh.sn[k2];
        if (s1 == 0.0 && s2 == 0.0) continue;
        const double c1 = sh.cs[k1], c2 = sh.cs[k2];
        const int a1 = sh.pa[k1], b1 = sh.pb[k1], a2 = sh.pa[k2], b2 = sh.pb[k2];
        // a pair holding the padding index (b = q) has s = 0 and no row b
        const bool hb1 = b1 < q, hb2 = b2 < q;
        if (PACKED && k1 == k2) {
          // diagonal block of a symmetric matrix: R^T X R with X = [xaa xab; xab xbb]
          if (!hb1) continue;
          double* paa = G + gidx<true>(a1, a1, lg);
          double* pab = G + gidx<true>(a1, b1, lg);
          double* pbb = G + gidx<true>(b1, b1, lg);
          const double xaa = *paa, xab = *pab, xbb = *pbb;
          const double yaa = c1 * xaa - s1 * xab, yab = c1 * xab - s1 * xbb;
          const double yba = s1 * xaa + c1 * xab, ybb = s1 * xab + c1 * xbb;
          *paa = c1 * yaa - s1 * yab;
          *pab = s1 * yaa + c1 * yab;
          *pbb = s1 * yba + c1 * ybb;
          continue;
        }
        double* paa = G + gidx<PACKED>(a1, a2, lg);
        double* pab = G + gidx<PACKED>(a1, b2, lg);
        double* pba = G + gidx<PACKED>(b1, a2, lg);
        double* pbb = G + gidx<PACKED>(b1, b2, lg);
        const double xaa = *paa;
        const double xab = hb2 ? *pab : 0.0;
        const double xba = hb1 ? *pba : 0.0;
        const double xbb = hb1 && hb2 ? *pbb : 0.0;
        // rows: R1^T X
        const double yaa = c1 * xaa - s1 * xba, yab = c1 * xab - s1 * xbb;
        const double yba = s1 * xaa + c1 * xba, ybb = s1 * xab + c1 * xbb;
        // columns: Y R2
        *paa = c2 * yaa - s2 * yab;
        if (hb2) *pab = s2 * yaa + c2 * yab;
        if (hb1) *pba = c2 * yba - s2 * ybb;
        if (hb1 && hb2) *pbb = s2 * yba + c2 * ybb;
      }
      // column pairs of W
      for (int e = tid; e < half * q; e += NT) {
        const int k = e / q, i = e - k * q;
        const double s = sh.sn[k];
        if (s == 0.0) continue;
        const double c = sh.cs[k];
        double* wa = W + i + (size_t)sh.pa[k] * lw;
        double* wb = W + i + (size_t)sh.pb[k] * lw;
        const double u = *wa, v = *wb;
        *wa = c * u - s * v;
        *wb = s * u + c * v;
      }
      __syncthreads();
    }
    const int go = *sh.flag;
    __syncthreads();
    if (!go) break;
  }
}

// Eigenvalues (the diagonal of G) in descending order, ties by index; the
// eigenvectors (columns of W) to `out` (q x q, ld q) in that order; res[0]
// = r, the number of leading eigenvalues with sqrt(max(lambda, 0)) > tau,
// res[1] = their sum (the squared Frobenius norm of the kept part).  `out`
// may be G's own storage: G is only read before the barrier.
template <int NT, bool PACKED = false>
__device__ void finish(const double* G, int lg, const double* W, int lw, int q, double tau,
                       double* out, double* res, double* lam, int* pos) {
  const int tid = threadIdx.x;
  for (int j = tid; j < q; j += NT) {
    const double lj = G[gidx<PACKED>(j, j, lg)];
    int p = 0;
    for (int i = 0; i < q; ++i) {
      const double li = G[gidx<PACKED>(i, i, lg)];
      p += (li > lj) || (li == lj && i < j);
    }
    pos[j] = p;
    lam[p] = lj;
  }
  __syncthreads();
  for (int e = tid; e < q * q; e += NT) {
    const int i = e % q, j = e / q;
    out[i + (size_t)pos[j] * q] = W[i + (size_t)j * lw];
  }
  if (tid == 0) {
    int r = 0;
    double sum = 0.0;
    for (; r < q; ++r) {
      const double l = lam[r];
      if (!(sqrt(fmax(l, 0.0)) > tau)) break;
      sum += l;
    }
    res[0] = (double)r;
    res[1] = sum;
  }
}

// Tiles of rank q <= QMAX: G and W in LDS (G with an odd leading dimension,
// so that the strided row updates spread over the banks).
template <int QMAX, int NT>
__global__ __launch_bounds__(NT) void k_sym_eig_lds(const EigDesc* __restrict__ descs, double tau,
                                                   double abs_scale) {
  constexpr int LG = QMAX + 1;
  __shared__ double sG[QMAX * LG];
  __shared__ double sW[QMAX * QMAX];
  __shared__ double cs[QMAX / 2], sn[QMAX / 2], lam[QMAX];
  __shared__ int pa[QMAX / 2], pb[QMAX / 2], pos[QMAX], flag;
  __shared__ double atol;
  const EigDesc d = descs[blockIdx.x];
  const int q = d.q;
  if (q <= 0 || q > QMAX) return;   // uniform over the workgroup
  for (int e = threadIdx.x; e < q * q; e += NT) {
    const int i = e % q, j = e / q;
    sG[i + j * LG] = d.G[i + (size_t)j * q];
  }
  __syncthreads();
  jacobi<NT>(sG, LG, sW, q, q, abs_scale, JacShared{cs, sn, pa, pb, &flag, &atol});
  finish<NT>(sG, LG, sW, q, q, tau, d.G, d.res, lam, pos);
}

// Tiles of rank q <= QMAX: G packed (upper triangle) in LDS, W in the
// descriptor's workspace in global memory (column pairs: coalesced).
template <int QMAX, int NT>
__global__ __launch_bounds__(NT) void k_sym_eig_packed(const EigDesc* __restrict__ descs,
                                                      double tau, double abs_scale) {
  __shared__ double sG[QMAX * (QMAX + 1) / 2];
  __shared__ double cs[QMAX / 2], sn[QMAX / 2], lam[QMAX];
  __shared__ int pa[QMAX / 2], pb[QMAX / 2], pos[QMAX], flag;
  __shared__ double atol;
  const EigDesc d = descs[blockIdx.x];
  const int q = d.q;
  if (q <= 0 || q > QMAX) return;
  const int np = q * (q + 1) / 2;
  for (int e = threadIdx.x; e < np; e += NT) {
    int j = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while ((j + 1) * (j + 2) / 2 <= e) ++j;
    while (j * (j + 1) / 2 > e) --j;
    const int i = e - j * (j + 1) / 2;
    sG[e] = d.G[i + (size_t)j * q];
  }
  __syncthreads();
  jacobi<NT, true>(sG, 0, d.W, q, q, abs_scale, JacShared{cs, sn, pa, pb, &flag, &atol});
  finish<NT, true>(sG, 0, d.W, q, q, tau, d.G, d.res, lam, pos);
}

// Tiles of rank up to kEigMaxRank: G in place and W in the descriptor's
// workspace, both q x q in global memory (L2-resident for the ranks met),
// 1024 threads to keep many accesses in flight.
__global__ __launch_bounds__(1024) void k_sym_eig_glb(const EigDesc* __restrict__ descs, double tau,
                                                     double abs_scale) {
  __shared__ double cs[kEigMaxRank / 2], sn[kEigMaxRank / 2], lam[kEigMaxRank];
  __shared__ int pa[kEigMaxRank / 2], pb[kEigMaxRank / 2], pos[kEigMaxRank], flag;
  __shared__ double atol;
  const EigDesc d = descs[blockIdx.x];
  const int q = d.q;
  if (q <= 0 || q > kEigMaxRank) return;
  jacobi<1024>(d.G, q, d.W, q, q, abs_scale, JacShared{cs, sn, pa, pb, &flag, &atol});
  finish<1024>(d.G, q, d.W, q, q, tau, d.G, d.res, lam, pos);
}

__global__ __launch_bounds__(256) void k_schur_shift(const double* __restrict__ D, int m,
                                                    double tau, double* __restrict__ X) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)m * m) return;
  X[e] = D[e] - (e % m == e / m ? tau : 0.0);
}

__global__ __launch_bounds__(256) void k_schur_diag(const double* __restrict__ E, int m,
                                                   double* __restrict__ T, int ldt, int nreal) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) acc += fabs(E[i + (size_t)j * m]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && j < nreal) T[j + (size_t)j * ldt] += red[0];
}

}  // namespace

hipError_t launch_schur_shift(const double* D, int m, double tau, double* X, hipStream_t s) {
  const size_t n = (size_t)m * m;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_schur_shift, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, D, m, tau,
                     X);
  return hipGetLastError();
}

hipError_t launch_schur_diag(const double* E, int m, double* T, int ldt, int nreal, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_schur_diag, dim3(m), dim3(256), 0, s, E, m, T, ldt, nreal);
  return hipGetLastError();
}

hipError_t launch_sym_eig(const EigDesc* d, int n, int cls, double tau, double abs_scale,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (cls) {
    case 0:
      hipLaunchKernelGGL((k_sym_eig_lds<kEigLdsSmall, 64>), dim3(n), dim3(64), 0, s, d, tau,
                         abs_scale);
      break;
    case 1:
      hipLaunchKernelGGL((k_sym_eig_lds<kEigLdsLarge, 512>), dim3(n), dim3(512), 0, s, d, tau,
                         abs_scale);
      break;
    case 2:
      hipLaunchKernelGGL((k_sym_eig_packed<kEigPacked, 1024>), dim3(n), dim3(1024), 0, s, d, tau,
                         abs_scale);
      break;
    case 3:
      hipLaunchKernelGGL(k_sym_eig_glb, dim3(n), dim3(1024), 0, s, d, tau, abs_scale);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tlr
