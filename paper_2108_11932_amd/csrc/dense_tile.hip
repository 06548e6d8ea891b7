// Dense tile kernels: the blocked Cholesky and unpivoted LDL^T of the
// diagonal tiles, and the diagonal-block step of the blocked triangular solve.
//
// The diagonal tile factorization is the "chol" (Algorithm "Left Looking TLR
// Cholesky") and "ldl" (Algorithm "Left Looking TLR LDL^T", unpivoted with
// scalar pivots) step of the paper.  The tile is factored right-looking by
// panels of 32 columns with one launch per panel: the launch for panel p
// solves the panel below its diagonal block with the block's explicit
// inverse (L21 = A21 L11^{-T}, one MFMA product), applies the rank-32
// trailing update on MFMA, and the workgroup that owns the next diagonal
// block then factors that block and inverts it in the same pass (Gauss-
// Jordan elimination beside the factorization), so that the next launch
// finds L11 and L11^{-1} ready.  The diagonal-block inverses also seed the
// assembly of L_kk^{-1}, by which the batched triangular solve of a column
// ("batchTrsm", one triangle shared by every tile) becomes one product.
#include "mfma_tiles.h"
#include "tlr_internal.h"

namespace tlr {

namespace {

constexpr int NB = 64;   // block size of the blocked triangular solve
constexpr int ND = 32;   // diagonal block of the blocked factorizations
constexpr int TT = 64;   // trailing-update tile

// A workgroup of FT = 256 threads factors the w x w (w <= 32) symmetric
// block S (LDS, lower triangle read, ld ND + 1) whose top-left entry sits at
// (b0, b0) of the tile A: Cholesky S = L L^T, or unit LDL^T S = L D L^T with
// scalar pivots.  L goes to A (zeros above its diagonal); L^{-1} (the unit
// inverse for LDL^T) to Inv at (b0, b0) (zeros above); the pivots to
// dvec[b0..] (LDL^T).
//
// Thread t holds row r = t % 32, columns 4 g .. 4 g + 3 (g = t / 32), of S
// and of X in registers (rows and columns beyond w are the identity, which
// leaves the real part unchanged).  At step j the threads holding column j
// put it into LDS, and by symmetry that column is also row j, so each
// thread reads d = S(j, j), its own S(r, j) and the S(c, j) of its columns
// as LDS broadcasts and subtracts l_rj S(j, c) from S(r, c), l_rj =
// S(r, j) / d.  The same row operation applied to X, which starts as the
// identity, leaves X = L_unit^{-1} after the last step (Gauss-Jordan
// elimination: the product of the elimination matrices), with row j of X
// read from the threads that hold it; L^{-1} = D^{-1/2} X for Cholesky.
// Two LDS buffers alternate, so one barrier per step suffices.
//
// info receives the 1-based row (row_base + b0 + j + 1) of the first
// failing pivot (the pivot is then taken as 1 so that the factor stays
// finite).  LDL^T: a pivot fails when |d| <= *tolp.  Cholesky: when d <= 0,
// or, with tolp set (modified Cholesky), d becomes max(|d|, *tolp) and is
// counted in info[1] instead.  Every thread of the workgroup calls it.
constexpr int FT = 256;
template <bool CHOL>
__device__ __forceinline__ void factor_block(const double (*S)[ND + 1], int w, double* A, int lda,
                                             int b0, double* Inv, int ldi, double* dvec, int* info,
                                             int row_base, const double* tolp) {
  constexpr int CW = ND * ND / FT;   // columns per thread (4)
  __shared__ double colb[2][ND];
  __shared__ double xrow[2][ND];
  __shared__ double Ls[ND][ND + 1];   // Ls[r][j] = L(r, j)
  const int t = threadIdx.x;
  const int r = t % ND, g = t / ND, c0 = CW * g;
  double sv[CW], xr[CW];
#pragma unroll
  for (int i = 0; i < CW; ++i) {
    const int c = c0 + i;
    double v = (r == c) ? 1.0 : 0.0;
    if (r < w && c < w && c <= r) v = S[r][c];
    sv[i] = v;
    xr[i] = (r == c) ? 1.0 : 0.0;
  }
  const bool modify = CHOL && tolp != nullptr;
  const double tol = CHOL ? (modify ? *tolp : 0.0) : *tolp;
  int bad_row = 0, nmod = 0;
  double my_rs = 1.0, my_d = 1.0;
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    double* cb = colb[j & 1];
    double* xb = xrow[j & 1];
    if (g == j / CW) cb[r] = sv[j % CW];
    if (r == j) {
#pragma unroll
      for (int i = 0; i < CW; ++i) xb[c0 + i] = xr[i];
    }
    __syncthreads();
    double d = cb[j];
    const double a = cb[r];   // S(r, j)
    double cv[CW], xv[CW];
#pragma unroll
    for (int i = 0; i < CW; ++i) {
      cv[i] = cb[c0 + i];
      xv[i] = xb[c0 + i];
    }
    const bool bad = CHOL ? !(d > 0.0) : !(fabs(d) > tol);
    if (bad && modify) {
      if (j < w) ++nmod;
      d = fmax(fabs(d), tol);
    } else if (bad) {
      if (j < w && bad_row == 0) bad_row = row_base + b0 + j + 1;
      d = 1.0;
    }
    // 1/sqrt(d) (Cholesky) or 1/d from the hardware estimate and two Newton
    // steps: a handful of FMAs instead of the division and square-root
    // sequences on the step's dependency chain
    double rs = 0.0, rd;
    if (CHOL) {
      rs = __builtin_amdgcn_rsq(d);
#pragma unroll
      for (int it = 0; it < 2; ++it) rs = fma(0.5 * rs, fma(-d * rs, rs, 1.0), rs);
      rd = rs * rs;
    } else {
      rd = __builtin_amdgcn_rcp(d);
#pragma unroll
      for (int it = 0; it < 2; ++it) rd = fma(rd, fma(-d, rd, 1.0), rd);
    }
    const double mr = a * rd;   // l_rj of the unit factor (r > j)
    // every column of S (finished columns and the upper triangle only
    // collect values that are never read again); X only on the rows below j
    const double xm = (r > j) ? mr : 0.0;
#pragma unroll
    for (int i = 0; i < CW; ++i) {
      sv[i] = fma(-mr, cv[i], sv[i]);
      xr[i] = fma(-xm, xv[i], xr[i]);
    }
    if (r == j) {
      my_rs = rs;
      my_d = d;
    }
    if (g == 0) {
      double lv;
      if (CHOL)
        lv = (r == j) ? d * rs : (r > j ? a * rs : 0.0);
      else
        lv = (r == j) ? 1.0 : (r > j ? mr : 0.0);
      Ls[r][j] = lv;
    }
  }
  __syncthreads();
  if (bad_row && t == 0) atomicCAS(info, 0, bad_row);
  if (nmod && t == 0) atomicAdd(info + 1, nmod);
  if (!CHOL && g == 0 && r < w) gmem(dvec)[b0 + r] = my_d;
  gdouble* Ag = gmem(A);
  gdouble* Ig = gmem(Inv);
#pragma unroll
  for (int i = 0; i < CW; ++i) {
    const int c = c0 + i;
    if (r < w && c < w) {
      Ag[(b0 + r) + (size_t)(b0 + c) * lda] = Ls[r][c];
      Ig[(b0 + r) + (size_t)(b0 + c) * ldi] = (c <= r) ? (CHOL ? my_rs * xr[i] : xr[i]) : 0.0;
    }
  }
}

// The first diagonal block of the tile: factor and invert.
template <bool CHOL>
__global__ __launch_bounds__(FT) void k_potrf_first(double* A, int lda, int m, double* Inv, int ldi,
                                                    double* dvec, int* info, int row_base,
                                                    const double* tolp) {
  __shared__ double S[ND][ND + 1];
  const int w = min(ND, m);
#pragma unroll
  for (int u = 0; u < ND * ND / FT; ++u) {
    const int e = threadIdx.x + FT * u;
    const int r = e % ND, c = e / ND;
    S[r][c] = (r < w && c < w && c <= r) ? gmem(A)[r + (size_t)c * lda] : 0.0;
  }
  __syncthreads();
  factor_block<CHOL>(S, w, A, lda, 0, Inv, ldi, dvec, info, row_base, tolp);
}

// Panel p (columns [p0, p0 + 32), its diagonal block already factored with
// L11^{-1} at (p0, p0) of Inv) of the blocked factorization.  The trailing
// matrix T = rows and columns [p0 + 32, m) is cut into 64 x 64 tiles; one
// workgroup (four waves) per tile (I, J), I >= J, of its lower triangle:
//   W(I) = A21(I) L11^{-T}           (Cholesky: L21(I) = W(I))
//   L21(J) = W(J) D^{-1}             (LDL^T; Cholesky: L21(J) = W(J))
//   T(I, J) -= W(I) L21(J)^T         (diagonal tiles: lower triangle stored)
// on the FP64 matrix cores (a 16-row slice of the tile per wave).  The
// workgroups with J = 0 write L21(I) into Lp (ld ldp, at the rows and
// columns it has in A: A's panel columns are still being read by the other
// workgroups); the workgroup of tile (0, 0), which holds the next diagonal
// block updated, then factors and inverts it (factor_block).
template <bool CHOL>
__global__ __launch_bounds__(256) void k_potrf_step(double* A, int lda, int m, int p0, double* Lp,
                                                    int ldp, double* Inv, int ldi, double* dvec,
                                                    int* info, int row_base, const double* tolp) {
  __shared__ double Lv[ND][ND + 1];   // L11^{-1}(c, q)
  __shared__ double Ai[TT][ND + 1];   // A21 rows of tile row I, then W(I)
  __shared__ double Aj[TT][ND + 1];   // A21 rows of tile column J, then L21(J)
  __shared__ double Sb[ND][ND + 1];   // the next diagonal block, updated (tile (0, 0))
  __shared__ double Dp[ND];
  const int t0 = p0 + ND;
  // tile (I, J) of the lower triangle from the workgroup index
  const int t = blockIdx.x;
  int bi = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while (bi * (bi + 1) / 2 > t) --bi;
  while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
  const int bj = t - bi * (bi + 1) / 2;
  const int r0 = t0 + TT * bi, c0 = t0 + TT * bj;
  const int nr = min(TT, m - r0), nc = min(TT, m - c0);
  const bool diag = bi == bj;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const gdouble* Ag = gmem((const double*)A);
  // every load of the launch in flight at once: L11^{-1}, the panel rows
  // of tile row I and column J, the pivots, and this wave's slice of the
  // trailing tile in the accumulator layout (register r of lane l: row
  // l / 16 + 4 r, column l % 16 of a 16 x 16 block)
  constexpr int NL = ND * ND / 256, NA = TT * ND / 256;
  double lvv[NL], aiv[NA], ajv[NA];
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int e = tid + 256 * u, r = e % ND, c = e / ND;
    lvv[u] = gmem((const double*)Inv)[(p0 + r) + (size_t)(p0 + c) * ldi];
  }
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const int e = tid + 256 * u, r = e % TT, q = e / TT;
    aiv[u] = Ag[(r0 + min(r, nr - 1)) + (size_t)(p0 + q) * lda];
    ajv[u] = diag ? 0.0 : Ag[(c0 + min(r, nc - 1)) + (size_t)(p0 + q) * lda];
  }
  const double dp = (!CHOL && tid < ND) ? gmem((const double*)dvec)[p0 + tid] : 1.0;
  d4 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int lr = 16 * wv + g + 4 * rr, lc = 16 * ct + li;
      acc[ct][rr] = Ag[(r0 + min(lr, nr - 1)) + (size_t)(c0 + min(lc, nc - 1)) * lda];
    }
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int e = tid + 256 * u;
    Lv[e % ND][e / ND] = lvv[u];
  }
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const int e = tid + 256 * u, r = e % TT, q = e / TT;
    Ai[r][q] = (r < nr) ? aiv[u] : 0.0;
    if (!diag) Aj[r][q] = (r < nc) ? ajv[u] : 0.0;
  }
  if (!CHOL && tid < ND) Dp[tid] = dp;
  __syncthreads();
  // W = A21 L11^{-T} for the 16-row slice wv of tile row I (and of tile
  // column J): D(i, n) = sum_q A21(i, q) L11^{-1}(n, q)
  d4 wi[2], wj[2];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    wi[ct] = d4{0.0, 0.0, 0.0, 0.0};
    wj[ct] = d4{0.0, 0.0, 0.0, 0.0};
  }
#pragma unroll
  for (int k0 = 0; k0 < ND; k0 += 4) {
    const double ai = Ai[16 * wv + li][k0 + g];
    const double aj = diag ? 0.0 : Aj[16 * wv + li][k0 + g];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const double b = Lv[16 * ct + li][k0 + g];
      wi[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, b, wi[ct], 0, 0, 0);
      if (!diag) wj[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(aj, b, wj[ct], 0, 0, 0);
    }
  }
  __syncthreads();   // every read of A21 done
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int lr = 16 * wv + g + 4 * rr, lc = 16 * ct + li;
      const double vi = wi[ct][rr];
      Ai[lr][lc] = vi;
      if (diag) {
        if (!CHOL) Aj[lr][lc] = vi / Dp[lc];
      } else {
        Aj[lr][lc] = CHOL ? wj[ct][rr] : wj[ct][rr] / Dp[lc];
      }
      if (bj == 0 && lr < nr) gmem(Lp)[(r0 + lr) + (size_t)(p0 + lc) * ldp] = CHOL ? vi : vi / Dp[lc];
    }
  __syncthreads();
  const double (*Lj)[ND + 1] = (CHOL && diag) ? Ai : Aj;
  // T(I, J) -= W(I) L21(J)^T: rows 16 wv .. 16 wv + 15 of the tile, all 64
  // columns
  gdouble* Tg = gmem(A);
#pragma unroll
  for (int k0 = 0; k0 < ND; k0 += 4) {
    const double a = -Ai[16 * wv + li][k0 + g];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Lj[16 * ct + li][k0 + g], acc[ct], 0, 0, 0);
  }
  const bool first = bi == 0 && bj == 0;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int lr = 16 * wv + g + 4 * rr, lc = 16 * ct + li;
      // the next diagonal block goes to A factored (below), not updated
      if (first && lr < ND && lc < ND)
        Sb[lr][lc] = acc[ct][rr];
      else if (lr < nr && lc < nc && (!diag || lr >= lc))
        Tg[(r0 + lr) + (size_t)(c0 + lc) * lda] = acc[ct][rr];
    }
  if (!first) return;
  __syncthreads();
  factor_block<CHOL>(Sb, min(ND, m - t0), A, lda, t0, Inv, ldi, dvec, info, row_base, tolp);
}

// A's final form after the panel steps: the panels below the diagonal
// blocks from Lp, the diagonal blocks as factored, zeros above the
// diagonal.
__global__ void k_tri_finish(double* A, int lda, const double* Lp, int ldp, int m) {
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)m * m) return;
  const int r = (int)(e % m), c = (int)(e / m);
  if (c > r)
    gmem(A)[r + (size_t)c * lda] = 0.0;
  else if (r / ND != c / ND)
    gmem(A)[r + (size_t)c * lda] = gmem(Lp)[r + (size_t)c * ldp];
}

// After a replay of the captured factorization: copy the results out of
// its fixed buffers and merge its status word (see launch_diag_out).
__global__ void k_diag_out(const double* __restrict__ A, double* __restrict__ Adst,
                           const double* __restrict__ Linv, double* __restrict__ Ldst,
                           const double* __restrict__ D, double* __restrict__ Ddst, int m,
                           int* ginfo, int* info, int row_base) {
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  const long long n = (long long)m * m;
  if (e < n) {
    gmem(Adst)[e] = gmem((const double*)A)[e];
    gmem(Ldst)[e] = gmem((const double*)Linv)[e];
  }
  if (D && e < m) gmem(Ddst)[e] = gmem((const double*)D)[e];
  if (e == 0) {
    const int bad = ginfo[0], nmod = ginfo[1];
    if (bad) atomicCAS(info, 0, row_base + bad);
    if (nmod) atomicAdd(info + 1, nmod);
    ginfo[0] = 0;
    ginfo[1] = 0;
  }
}

// out(r, c) = in(r, c) * s[c] or / s[c] (column scaling, LDL^T panels).
__global__ void k_scale_cols(const double* in, int ldi, double* out, int ldo, const double* s,
                             int rows, int cols, int inverse) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)rows * cols) return;
  const int r = (int)(e % rows), c = (int)(e / rows);
  const double v = in[r + (size_t)c * ldi];
  out[r + (size_t)c * ldo] = inverse ? v / s[c] : v * s[c];
}

// X_p = L_pp^{-1} B_p or L_pp^{-T} B_p on rows [p0, p0 + w) of B: 64
// right-hand sides per workgroup, one thread per right-hand side, the
// triangle and the right-hand sides in LDS.
__global__ __launch_bounds__(64) void k_trsm_diag(const double* L, int ldl, double* B, int ldb,
                                                  int p0, int w, int n, int unit, int trans) {
  __shared__ double S[NB][NB + 1];   // S[c][r] = L(p0 + r, p0 + c)
  __shared__ double X[64][NB + 1];   // X[col][row]
  const int tid = threadIdx.x;
  const int col0 = blockIdx.x * 64;
  for (int e = tid; e < w * w; e += 64) {
    const int r = e % w, c = e / w;
    S[c][r] = (c <= r) ? L[(p0 + r) + (size_t)(p0 + c) * ldl] : 0.0;
  }
  for (int c = 0; c < 64; ++c) {
    const int gc = col0 + c;
    if (gc < n && tid < w) X[c][tid] = B[(p0 + tid) + (size_t)gc * ldb];
  }
  __syncthreads();
  if (col0 + tid < n) {
    double* x = X[tid];
    if (!trans) {
      for (int j = 0; j < w; ++j) {
        double v = x[j];
        for (int c = 0; c < j; ++c) v -= S[c][j] * x[c];
        x[j] = unit ? v : v / S[j][j];
      }
    } else {
      for (int j = w - 1; j >= 0; --j) {
        double v = x[j];
        for (int r = j + 1; r < w; ++r) v -= S[j][r] * x[r];
        x[j] = unit ? v : v / S[j][j];
      }
    }
  }
  __syncthreads();
  for (int c = 0; c < 64; ++c) {
    const int gc = col0 + c;
    if (gc < n && tid < w) B[(p0 + tid) + (size_t)gc * ldb] = X[c][tid];
  }
}

}  // namespace

int diag_block_size() { return ND; }

hipError_t launch_potrf_first(bool chol, double* A, int lda, int m, double* Inv, int ldi,
                              double* dvec, int* info, int row_base, const double* tolp,
                              hipStream_t s) {
  if (m <= 0) return hipErrorInvalidValue;
  if (chol)
    hipLaunchKernelGGL(k_potrf_first<true>, dim3(1), dim3(FT), 0, s, A, lda, m, Inv, ldi, dvec,
                       info, row_base, tolp);
  else
    hipLaunchKernelGGL(k_potrf_first<false>, dim3(1), dim3(FT), 0, s, A, lda, m, Inv, ldi, dvec,
                       info, row_base, tolp);
  return hipGetLastError();
}

hipError_t launch_potrf_step(bool chol, double* A, int lda, int m, int p0, double* Lp, int ldp,
                             double* Inv, int ldi, double* dvec, int* info, int row_base,
                             const double* tolp, hipStream_t s) {
  if (p0 < 0 || p0 % ND != 0 || p0 + ND >= m) return hipErrorInvalidValue;
  const int nt = (m - p0 - ND + TT - 1) / TT;
  const unsigned nwg = (unsigned)(nt * (nt + 1) / 2);
  if (chol)
    hipLaunchKernelGGL(k_potrf_step<true>, dim3(nwg), dim3(256), 0, s, A, lda, m, p0, Lp, ldp, Inv,
                       ldi, dvec, info, row_base, tolp);
  else
    hipLaunchKernelGGL(k_potrf_step<false>, dim3(nwg), dim3(256), 0, s, A, lda, m, p0, Lp, ldp,
                       Inv, ldi, dvec, info, row_base, tolp);
  return hipGetLastError();
}

hipError_t launch_diag_out(const double* A, double* Adst, const double* Linv, double* Ldst,
                           const double* D, double* Ddst, int m, int* ginfo, int* info,
                           int row_base, hipStream_t s) {
  const long long n = (long long)m * m;
  if (n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_diag_out, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, Adst, Linv,
                     Ldst, D, Ddst, m, ginfo, info, row_base);
  return hipGetLastError();
}

hipError_t launch_tri_finish(double* A, int lda, const double* Lp, int ldp, int m, hipStream_t s) {
  const long long n = (long long)m * m;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tri_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, lda, Lp,
                     ldp, m);
  return hipGetLastError();
}

hipError_t launch_scale_cols(const double* in, int ldi, double* out, int ldo, const double* sc,
                             int rows, int cols, bool inverse, hipStream_t s) {
  const long long n = (long long)rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, ldi, out,
                     ldo, sc, rows, cols, inverse ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_trsm_diag(const double* L, int ldl, double* B, int ldb, int p0, int w, int n,
                            bool unit, bool trans, hipStream_t s) {
  if (w <= 0 || w > NB || n <= 0) return w > NB ? hipErrorInvalidValue : hipSuccess;
  hipLaunchKernelGGL(k_trsm_diag, dim3((n + 63) / 64), dim3(64), 0, s, L, ldl, B, ldb, p0, w, n,
                     unit ? 1 : 0, trans ? 1 : 0);
  return hipGetLastError();
}

}  // namespace tlr
