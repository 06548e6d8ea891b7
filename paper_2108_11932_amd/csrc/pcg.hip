// Preconditioned conjugate gradients with a TLR factorization as the
// preconditioner (the use of the factorizations in Section 6: a loosely
// compressed factor preconditions the accurately compressed operator).
//
// The operator is the input matrix of one handle (tlr_matvec), the
// preconditioner the factor of another (tlr_solve).  The vector kernels are
// plain streaming kernels; the two inner products of an iteration are
// reduced in a fixed order (per-workgroup partial sums, then one workgroup
// over them), so a run is reproducible, and read back to the host, which
// forms the step lengths.
#include <cmath>

#include "host.h"

namespace tlr {

namespace {

constexpr int kDotBlocks = 256;

// partial[b] = sum over the grid-stride range of block b of x_i y_i
__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ x,
                                                     const double* __restrict__ y, long long n,
                                                     double* partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x)
    s = fma(x[i], y[i], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out[slot] = sum of the kDotBlocks partials, in order of a fixed tree
__global__ __launch_bounds__(256) void k_dot_final(const double* partial, double* out) {
  __shared__ double red[kDotBlocks];
  red[threadIdx.x] = partial[threadIdx.x];
  __syncthreads();
  for (int w = kDotBlocks / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// y += a x
__global__ void k_axpy(double a, const double* __restrict__ x, double* __restrict__ y, long long n) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i < n) y[i] = fma(a, x[i], y[i]);
}

// p = z + b p
__global__ void k_xpby(const double* __restrict__ z, double b, double* __restrict__ p, long long n) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i < n) p[i] = fma(b, p[i], z[i]);
}

// r = b - r (r holds A x on entry)
__global__ void k_residual(const double* __restrict__ b, double* __restrict__ r, long long n) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i < n) r[i] = b[i] - r[i];
}

unsigned grid_for(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

}  // namespace tlr

extern "C" {

tlr_status tlr_pcg(tlr_matrix_t A, tlr_matrix_t F, const double* b, double* x, double rtol,
                   int maxit, int* iters, double* relres, void* stream) {
  using namespace tlr;
  if (!A || !b || !x || !iters || !relres) {
    set_error("NULL argument");
    return TLR_ERR_ARG;
  }
  if (!(rtol > 0.0) || maxit < 0) {
    set_error("rtol must be positive and maxit non-negative");
    return TLR_ERR_ARG;
  }
  if (F && (F->N != A->N || !F->factored)) {
    set_error(F->N != A->N ? "the preconditioner's size differs from the operator's"
                           : "the preconditioner handle holds no factor");
    return F->N != A->N ? TLR_ERR_ARG : TLR_ERR_STATE;
  }
  const long long n = A->N;
  hipStream_t s = (hipStream_t)stream;
  A->stream = A->mem.stream = s;
  // r, z, p, q, partial sums and the two reduced scalars
  void* wk = nullptr;
  const size_t nv = (size_t)n;
  TLR_TRY(A->mem.get(&wk, sizeof(double) * (4 * nv + kDotBlocks + 8)));
  double* r = (double*)wk;
  double* z = r + nv;
  double* p = z + nv;
  double* q = p + nv;
  double* part = q + nv;
  double* dsc = part + kDotBlocks;
  tlr_status st = TLR_OK;
  auto dot = [&](const double* u, const double* v, double* out) -> tlr_status {
    hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, s, u, v, n, part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kDotBlocks), 0, s, part, dsc);
    TLR_HIP(hipGetLastError());
    TLR_HIP(hipMemcpyAsync(out, dsc, sizeof(double), hipMemcpyDeviceToHost, s));
    TLR_HIP(hipStreamSynchronize(s));
    return TLR_OK;
  };
  auto precond = [&]() -> tlr_status {
    TLR_HIP(hipMemcpyAsync(z, r, sizeof(double) * nv, hipMemcpyDeviceToDevice, s));
    if (F) TLR_TRY(tlr_solve(F, 1, z, n, stream));
    return TLR_OK;
  };
  auto body = [&]() -> tlr_status {
    double bb = 0.0, rr = 0.0, rz = 0.0, pq = 0.0;
    TLR_TRY(dot(b, b, &bb));
    const double bnorm = std::sqrt(bb);
    // r = b - A x
    TLR_TRY(tlr_matvec(A, 1, x, n, r, n, stream));
    hipLaunchKernelGGL(k_residual, dim3(grid_for(n)), dim3(256), 0, s, b, r, n);
    TLR_HIP(hipGetLastError());
    TLR_TRY(dot(r, r, &rr));
    *iters = 0;
    *relres = bnorm > 0.0 ? std::sqrt(rr) / bnorm : 0.0;
    if (bnorm == 0.0 || *relres <= rtol) return TLR_OK;
    TLR_TRY(precond());
    TLR_HIP(hipMemcpyAsync(p, z, sizeof(double) * nv, hipMemcpyDeviceToDevice, s));
    TLR_TRY(dot(r, z, &rz));
    for (int it = 1; it <= maxit; ++it) {
      TLR_TRY(tlr_matvec(A, 1, p, n, q, n, stream));
      TLR_TRY(dot(p, q, &pq));
      if (!(pq > 0.0)) {
        set_error("PCG: the operator is not positive definite along the search direction");
        return TLR_ERR_NOT_SPD;
      }
      const double alpha = rz / pq;
      hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(256), 0, s, alpha, p, x, n);
      hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(256), 0, s, -alpha, q, r, n);
      TLR_HIP(hipGetLastError());
      TLR_TRY(dot(r, r, &rr));
      *iters = it;
      *relres = std::sqrt(rr) / bnorm;
      if (*relres <= rtol) break;
      TLR_TRY(precond());
      double rz_new = 0.0;
      TLR_TRY(dot(r, z, &rz_new));
      const double beta = rz_new / rz;
      rz = rz_new;
      hipLaunchKernelGGL(k_xpby, dim3(grid_for(n)), dim3(256), 0, s, z, beta, p, n);
      TLR_HIP(hipGetLastError());
    }
    return TLR_OK;
  };
  st = body();
  (void)hipStreamSynchronize(s);
  A->mem.put(wk);
  return st;
}

}  // extern "C"
