// Kernels of the batched adaptive randomized approximation (Section 3.1 and
// Algorithm "Left Looking Cholesky TLR ARA Update", Section 4.2):
//
//  * batchRandn      -- Philox4x32-10 + Box-Muller Gaussian test matrices
//  * batchOrthog     -- block Gram-Schmidt, the QR of each block done by a
//                       Cholesky QR whose Gram matrix and Cholesky factor are
//                       carried in double-double (the paper's mixed-precision
//                       Cholesky QR), with diagonal pivoting and a threshold
//                       so that the rank is found column by column
//  * getConvergedTiles / updateSubset -- convergence flags and the stable
//                       compaction + refill of the active subset
//  * sortRanks       -- order of the tiles of a column by input rank
#include "dd.h"
#include "mfma_tiles.h"
#include "tlr_internal.h"

// The double-double arithmetic below relies on error-free transformations
// that must see every product and sum rounded separately: no contraction of
// a*b + c into fused multiply-adds in this file (explicit fma() calls stay).
#pragma clang fp contract(off)

#include "ara_compact.h"
#include "ara_orth.h"

namespace tlr {

namespace {

// ------------------------------------------------------------------ Philox
constexpr unsigned PH_M0 = 0xD2511F53u, PH_M1 = 0xCD9E8D57u;
constexpr unsigned PH_W0 = 0x9E3779B9u, PH_W1 = 0xBB67AE85u;

__device__ inline uint4 philox10(uint4 c, unsigned k0, unsigned k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += PH_W0; k1 += PH_W1; }
    const unsigned hi0 = __umulhi(PH_M0, c.x), lo0 = PH_M0 * c.x;
    const unsigned hi1 = __umulhi(PH_M1, c.z), lo1 = PH_M1 * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

__device__ inline double u53(unsigned hi, unsigned lo) {
  return ((double)(hi >> 5) * 67108864.0 + (double)(lo >> 6)) * (1.0 / 9007199254740992.0);
}

__global__ void k_randn(double* out, int rows, int cols, int ld, unsigned k0, unsigned k1,
                        unsigned k, unsigned t, unsigned strm) {
  const long long n = (long long)rows * cols;
  const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (2 * c >= n) return;
  const uint4 w = philox10(make_uint4((unsigned)c, t, k, strm), k0, k1);
  const double u1 = 1.0 - u53(w.x, w.y);
  const double u2 = u53(w.z, w.w);
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos(6.283185307179586476925286766559 * u2, &sn, &cs);
  long long e = 2 * c;
  out[(e % rows) + (e / rows) * (long long)ld] = rad * cs;
  if (e + 1 < n) {
    e += 1;
    out[(e % rows) + (e / rows) * (long long)ld] = rad * sn;
  }
}

// The test matrices of iterations t0 .. t0 + nt - 1 (blockIdx.y = t - t0),
// each rows x cols_t with cols_t = cols0 for t = 0 and cols1 after, the
// same values as k_randn with that t; matrix t - t0 at out + (t - t0) * stride.
__global__ void k_randn_iters(double* out, int rows, size_t stride, int cols0, int cols1,
                              unsigned k0, unsigned k1, unsigned k, unsigned t0, unsigned strm) {
  const unsigned t = t0 + blockIdx.y;
  const int cols = t == 0 ? cols0 : cols1;
  const long long n = (long long)rows * cols;
  const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (2 * c >= n) return;
  const uint4 w = philox10(make_uint4((unsigned)c, t, k, strm), k0, k1);
  const double u1 = 1.0 - u53(w.x, w.y);
  const double u2 = u53(w.z, w.w);
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos(6.283185307179586476925286766559 * u2, &sn, &cs);
  double* o = out + (size_t)blockIdx.y * stride;
  o[2 * c] = rad * cs;
  if (2 * c + 1 < n) o[2 * c + 1] = rad * sn;
}

__global__ void k_philox_raw(unsigned* out, int n, unsigned k0, unsigned k1, unsigned c1,
                             unsigned c2, unsigned c3) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const uint4 w = philox10(make_uint4((unsigned)c, c1, c2, c3), k0, k1);
  out[4 * c + 0] = w.x;
  out[4 * c + 1] = w.y;
  out[4 * c + 2] = w.z;
  out[4 * c + 3] = w.w;
}

template <int BS, bool PIV>
__global__ __launch_bounds__(APPLY_ROWS) void k_orth_step(AraDev D, int r_min) {
  orth_body<BS, PIV>(D, r_min, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void k_compact(int* act, int* counts, const int* flag,
                                                 const int* waiting, int nwaiting, int s_max,
                                                 const int* info) {
  __shared__ int wsum[8];
  compact_active(act, act, counts, counts, flag, waiting, nwaiting, s_max, nullptr, nullptr, wsum);
  if (threadIdx.x == 0 && info) counts[2] = *info;
}

__global__ __launch_bounds__(256) void k_ara_compact(AraDev D, const int* waiting, int nwaiting,
                                                     int s_max, const int* info, int* host_out,
                                                     int* host_res, int res_ints) {
  ara_compact_body(D, waiting, nwaiting, s_max, info, host_out, host_res, res_ints);
}

}  // namespace

hipError_t launch_randn(double* out, int rows, int cols, int ld, unsigned long long seed, unsigned k,
                        unsigned t, unsigned stream, hipStream_t s) {
  const long long pairs = ((long long)rows * cols + 1) / 2;
  if (pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_randn, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, out, rows,
                     cols, ld, (unsigned)(seed & 0xffffffffu), (unsigned)(seed >> 32), k, t,
                     stream);
  return hipGetLastError();
}

hipError_t launch_randn_iters(double* out, int rows, size_t stride, int cols0, int cols1,
                              unsigned long long seed, unsigned k, unsigned t0, int nt,
                              unsigned stream, hipStream_t s) {
  const long long pairs = ((long long)rows * (cols0 > cols1 ? cols0 : cols1) + 1) / 2;
  if (pairs <= 0 || nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_randn_iters, dim3((unsigned)((pairs + 255) / 256), (unsigned)nt), dim3(256),
                     0, s, out, rows, stride, cols0, cols1, (unsigned)(seed & 0xffffffffu),
                     (unsigned)(seed >> 32), k, t0, stream);
  return hipGetLastError();
}

hipError_t launch_philox_raw(unsigned* out, int n, unsigned long long seed, unsigned c1,
                             unsigned c2, unsigned c3, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox_raw, dim3((n + 255) / 256), dim3(256), 0, s, out, n,
                     (unsigned)(seed & 0xffffffffu), (unsigned)(seed >> 32), c1, c2, c3);
  return hipGetLastError();
}

namespace {
__global__ void k_mixed_guard(AraSlotDesc* slots, const GuardDesc* __restrict__ g, int n,
                              int* prec) {
#pragma clang fp contract(off)
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= n) return;
  const GuardDesc d = g[sl];
  double nu = d.nu;
  if (d.irow >= 0) {
    const double prod = d.fro[d.irow] * d.fro[0];
    nu = nu + prod;
  }
  int use = 0;
  if (d.a1_16 != nullptr && nu <= d.lim16)
    use = 2;
  else if (d.a1_32 != nullptr && nu <= d.lim32)
    use = 1;
  if (use) {
    slots[sl].a1 = use == 2 ? d.a1_16 : d.a1_32;
    slots[sl].lda1 = d.nrb;
    slots[sl].a1_prec = use;
  }
  prec[sl] = use;
}
}  // namespace

hipError_t launch_mixed_guard(AraSlotDesc* slots, const GuardDesc* g, int n, int* prec,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mixed_guard, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, slots, g, n,
                     prec);
  return hipGetLastError();
}

// KERNEL is a template-id whose block-size argument is spelled BS_ARG.
#define TLR_BS_CASE(v, KERNEL, ...)                    \
  case v: {                                            \
    constexpr int BS_ARG = v;                          \
    hipLaunchKernelGGL(KERNEL, __VA_ARGS__);           \
    break;                                             \
  }
#define TLR_BS_DISPATCH(bs, KERNEL, ...)               \
  switch (bs) {                                        \
    TLR_BS_CASE(16, KERNEL, __VA_ARGS__)               \
    TLR_BS_CASE(32, KERNEL, __VA_ARGS__)               \
    TLR_BS_CASE(8, KERNEL, __VA_ARGS__)                \
    TLR_BS_CASE(24, KERNEL, __VA_ARGS__)               \
    TLR_BS_CASE(4, KERNEL, __VA_ARGS__)                \
    TLR_BS_CASE(2, KERNEL, __VA_ARGS__)                \
    TLR_BS_CASE(1, KERNEL, __VA_ARGS__)                \
    default: return hipErrorInvalidValue;              \
  }

bool orth_block_supported(int bs) {
  return bs == 1 || bs == 2 || bs == 4 || bs == 8 || bs == 16 || bs == 24 || bs == 32;
}

hipError_t launch_orth_step(const AraDev& D, int pass, int r_min, int count_bound, hipStream_t s) {
  if (count_bound <= 0) return hipSuccess;
  const dim3 grid((D.m + APPLY_ROWS - 1) / APPLY_ROWS, count_bound);
  if (pass == 1) {
    TLR_BS_DISPATCH(D.bs, (k_orth_step<BS_ARG, true>), grid, dim3(APPLY_ROWS), 0, s, D, r_min);
  } else {
    TLR_BS_DISPATCH(D.bs, (k_orth_step<BS_ARG, false>), grid, dim3(APPLY_ROWS), 0, s, D, r_min);
  }
  return hipGetLastError();
}

hipError_t launch_ara_compact(const AraDev& D, const int* waiting, int nwaiting, int s_max,
                              const int* info, int* host_out, int* host_res, int res_ints,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_ara_compact, dim3(1), dim3(256), 0, s, D, waiting, nwaiting, s_max, info,
                     host_out, host_res, res_ints);
  return hipGetLastError();
}

hipError_t launch_compact(int* act, int* counts, const int* flag, const int* waiting, int nwaiting,
                          int s_max, const int* info, hipStream_t s) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(256), 0, s, act, counts, flag, waiting, nwaiting,
                     s_max, info);
  return hipGetLastError();
}

}  // namespace tlr
