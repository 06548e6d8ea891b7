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
// theta = (g_bb - g_aa) / (2 g_ab)), which zeroes g_ab.  The rounds' pairs
// are disjoint, so the row updates of all of them and then the column
// updates run in parallel.  The run ends after a sweep without rotations
// or after kSweeps sweeps; the decision is the workgroup's, so every wave
// leaves the loop together.
template <int NT>
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
    for (int j = 0; j < q; ++j) g = fmax(g, fabs(G[j + (size_t)j * lg]));
    *sh.atol = abs_scale * g;
  }
  __syncthreads();
  const double atol = *sh.atol;
  for (int sweep = 0; sweep < kSweeps; ++sweep) {
    if (tid == 0) *sh.flag = 0;
    __syncthreads();
    for (int t = 0; t < n - 1; ++t) {
      for (int k = tid; k < half; k += NT) {
        int a, b;
        jac_pair(n, t, k, a, b);
        double c = 1.0, s = 0.0;
        if (b < q) {
          const double gaa = G[a + (size_t)a * lg], gbb = G[b + (size_t)b * lg];
          const double gab = G[a + (size_t)b * lg];
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
      // rows a and b of G: G <- J^T G
      for (int e = tid; e < half * q; e += NT) {
        const int k = e / q, j = e - k * q;
        const double s = sh.sn[k];
        if (s == 0.0) continue;
        const double c = sh.cs[k];
        double* ra = G + sh.pa[k] + (size_t)j * lg;
        double* rb = G + sh.pb[k] + (size_t)j * lg;
        const double x = *ra, y = *rb;
        *ra = c * x - s * y;
        *rb = s * x + c * y;
      }
      __syncthreads();
      // columns a and b of G and W: G <- G J, W <- W J
      for (int e = tid; e < half * q; e += NT) {
        const int k = e / q, i = e - k * q;
        const double s = sh.sn[k];
        if (s == 0.0) continue;
        const double c = sh.cs[k];
        double* ca = G + i + (size_t)sh.pa[k] * lg;
        double* cb = G + i + (size_t)sh.pb[k] * lg;
        const double x = *ca, y = *cb;
        *ca = c * x - s * y;
        *cb = s * x + c * y;
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
template <int NT>
__device__ void finish(const double* G, int lg, const double* W, int lw, int q, double tau,
                       double* out, double* res, double* lam, int* pos) {
  const int tid = threadIdx.x;
  for (int j = tid; j < q; j += NT) {
    const double lj = G[j + (size_t)j * lg];
    int p = 0;
    for (int i = 0; i < q; ++i) {
      const double li = G[i + (size_t)i * lg];
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

// Tiles of rank up to kEigMaxRank: G in place and W in the descriptor's
// workspace, both q x q in global memory (L2-resident for the ranks met).
__global__ __launch_bounds__(256) void k_sym_eig_glb(const EigDesc* __restrict__ descs, double tau,
                                                     double abs_scale) {
  __shared__ double cs[kEigMaxRank / 2], sn[kEigMaxRank / 2], lam[kEigMaxRank];
  __shared__ int pa[kEigMaxRank / 2], pb[kEigMaxRank / 2], pos[kEigMaxRank], flag;
  __shared__ double atol;
  const EigDesc d = descs[blockIdx.x];
  const int q = d.q;
  if (q <= 0 || q > kEigMaxRank) return;
  jacobi<256>(d.G, q, d.W, q, q, abs_scale, JacShared{cs, sn, pa, pb, &flag, &atol});
  finish<256>(d.G, q, d.W, q, q, tau, d.G, d.res, lam, pos);
}

}  // namespace

hipError_t launch_sym_eig(const EigDesc* d, int n, int cls, double tau, double abs_scale,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (cls) {
    case 0:
      hipLaunchKernelGGL((k_sym_eig_lds<kEigLdsSmall, 64>), dim3(n), dim3(64), 0, s, d, tau,
                         abs_scale);
      break;
    case 1:
      hipLaunchKernelGGL((k_sym_eig_lds<kEigLdsLarge, 256>), dim3(n), dim3(256), 0, s, d, tau,
                         abs_scale);
      break;
    case 2:
      hipLaunchKernelGGL(k_sym_eig_glb, dim3(n), dim3(256), 0, s, d, tau, abs_scale);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tlr
