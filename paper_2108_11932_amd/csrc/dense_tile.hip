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

// One wave factors the w x w (w <= 32) symmetric block S (LDS, lower
// triangle read, ld ND + 1) whose top-left entry sits at (b0, b0) of the
// tile A: Cholesky S = L L^T, or unit LDL^T S = L D L^T with scalar
// pivots.  L goes to A (zeros above its diagonal); L^{-1} (the unit
// inverse for LDL^T) to Inv at (b0, b0) (zeros above); the pivots to
// dvec[b0..] (LDL^T).
//
// Lanes r and r + 32 hold the two halves of row r of S, and of row r of
// X, in registers (rows and columns beyond w are the identity, which leaves
// the real part unchanged).  At step j the lanes holding column j put it
// into LDS, and by symmetry that column is also row j, so each lane reads
// d = S(j, j), its own S(r, j) and the S(c, j) of its half as LDS
// broadcasts and subtracts l_rj S(j, c) from S(r, c), l_rj = S(r, j) / d.
// The same row operation applied to X, which starts as the identity,
// leaves X = L_unit^{-1} after the last step (Gauss-Jordan elimination:
// the product of the elimination matrices), with row j of X read from the
// two lanes that hold it; L^{-1} = D^{-1/2} X for Cholesky.
//
// info receives the 1-based row (row_base + b0 + j + 1) of the first
// failing pivot (the pivot is then taken as 1 so that the factor stays
// finite).  LDL^T: a pivot fails when |d| <= *tolp.  Cholesky: when d <= 0,
// or, with tolp set (modified Cholesky), d becomes max(|d|, *tolp) and is
// counted in info[1] instead.
template <bool CHOL>
__device__ __forceinline__ void factor_block(const double (*S)[ND + 1], int w, double* A, int lda, int b0,
                                    double* Inv, int ldi, double* dvec, int* info, int row_base,
                                    const double* tolp) {
  __shared__ double colb[2][ND];
  __shared__ double xrow[2][ND];
  __shared__ double Ls[ND][ND + 1];   // Ls[r][j] = L(r, j)
  const int lane = threadIdx.x & 63;
  const int r = lane & (ND - 1);
  const int hf = lane >> 5;   // this lane holds columns [16 hf, 16 hf + 16) of row r
  constexpr int HC = ND / 2;
  double row[HC], xr[HC];
#pragma unroll
  for (int cc = 0; cc < HC; ++cc) {
    const int c = HC * hf + cc;
    double v = (r == c) ? 1.0 : 0.0;
    if (r < w && c < w && c <= r) v = S[r][c];
    row[cc] = v;
    xr[cc] = (r == c) ? 1.0 : 0.0;
  }
  const bool modify = CHOL && tolp != nullptr;
  const double tol = CHOL ? (modify ? *tolp : 0.0) : *tolp;
  int bad_row = 0, nmod = 0;
  double my_rs = 1.0, my_d = 1.0;
  // the steps in two halves of 16 (a fully unrolled loop of 32 lets the
  // compiler hoist across steps until the registers run out)
#pragma unroll 1
  for (int hb = 0; hb < 2; ++hb) {
#pragma unroll
    for (int jj = 0; jj < HC; ++jj) {
      const int j = HC * hb + jj;
      double* cb = colb[jj & 1];
      double* xb = xrow[jj & 1];
      if (hf == hb) cb[r] = row[jj];
      if (r == j) {
#pragma unroll
        for (int cc = 0; cc < HC; ++cc) xb[HC * hf + cc] = xr[cc];
      }
      // the caller runs this on one wave, whose LDS operations complete in
      // issue order: the reads below see the writes above without a wait
      __builtin_amdgcn_wave_barrier();
      double d = cb[j];
      const double a = cb[r];   // S(r, j)
      double cv[HC], xv[HC];
#pragma unroll
      for (int cc = 0; cc < HC; ++cc) {
        cv[cc] = cb[HC * hf + cc];
        xv[cc] = xb[HC * hf + cc];
      }
      __builtin_amdgcn_sched_barrier(0);
      const bool bad = CHOL ? !(d > 0.0) : !(fabs(d) > tol);
      if (bad && modify) {
        if (j < w) ++nmod;
        d = fmax(fabs(d), tol);
      } else if (bad) {
        if (j < w && bad_row == 0) bad_row = row_base + b0 + j + 1;
        d = 1.0;
      }
      // 1/sqrt(d) (Cholesky) or 1/d from the hardware estimate and two
      // Newton steps: a handful of FMAs instead of the division and
      // square-root sequences on the step's dependency chain
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
      // every column of the half of S (finished columns and the upper
      // triangle only collect values that are never read again); X only on
      // the rows below j
      const double xm = (r > j) ? mr : 0.0;
#pragma unroll
      for (int cc = 0; cc < HC; ++cc) {
        row[cc] = fma(-mr, cv[cc], row[cc]);
        xr[cc] = fma(-xm, xv[cc], xr[cc]);
      }
      if (r == j) {
        my_rs = rs;
        my_d = d;
      }
      double lv;
      if (CHOL)
        lv = (r == j) ? d * rs : (r > j ? a * rs : 0.0);
      else
        lv = (r == j) ? 1.0 : (r > j ? mr : 0.0);
      if (hf == 0) Ls[r][j] = lv;
    }
  }
  __builtin_amdgcn_wave_barrier();
  if (bad_row && lane == 0) atomicCAS(info, 0, bad_row);
  if (nmod && lane == 0) atomicAdd(info + 1, nmod);
  if (!CHOL && hf == 0 && r < w) gmem(dvec)[b0 + r] = my_d;
  gdouble* Ag = gmem(A);
  gdouble* Ig = gmem(Inv);
#pragma unroll
  for (int cc = 0; cc < HC; ++cc) {
    const int c = HC * hf + cc;
    if (r < w && c < w) {
      Ag[(b0 + r) + (size_t)(b0 + c) * lda] = Ls[r][c];
      Ig[(b0 + r) + (size_t)(b0 + c) * ldi] = (c <= r) ? (CHOL ? my_rs * xr[cc] : xr[cc]) : 0.0;
    }
  }
}

// The first diagonal block of the tile: factor and invert (one wave).
template <bool CHOL>
__global__ __launch_bounds__(64) void k_potrf_first(double* A, int lda, int m, double* Inv, int ldi,
                                                    double* dvec, int* info, int row_base,
                                                    const double* tolp) {
  __shared__ double S[ND][ND + 1];
  const int w = min(ND, m);
  for (int e = threadIdx.x; e < ND * ND; e += 64) {
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
// block updated, then factors and inverts it (factor_block on its first
// wave).
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
  const gdouble* Ag = gmem((const double*)A);
  for (int e = tid; e < ND * ND; e += 256) {
    const int r = e % ND, c = e / ND;
    Lv[r][c] = gmem((const double*)Inv)[(p0 + r) + (size_t)(p0 + c) * ldi];
  }
  for (int e = tid; e < TT * ND; e += 256) {
    const int r = e % TT, q = e / TT;
    Ai[r][q] = (r < nr) ? Ag[(r0 + r) + (size_t)(p0 + q) * lda] : 0.0;
    if (!diag) Aj[r][q] = (r < nc) ? Ag[(c0 + r) + (size_t)(p0 + q) * lda] : 0.0;
  }
  if (!CHOL && tid < ND) Dp[tid] = gmem((const double*)dvec)[p0 + tid];
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
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
  d4 acc[4];
  gdouble* Tg = gmem(A);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int lr = 16 * wv + g + 4 * rr, lc = 16 * ct + li;
      acc[ct][rr] = (lr < nr && lc < nc) ? Tg[(r0 + lr) + (size_t)(c0 + lc) * lda] : 0.0;
    }
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
  if (wv == 0)
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
    hipLaunchKernelGGL(k_potrf_first<true>, dim3(1), dim3(64), 0, s, A, lda, m, Inv, ldi, dvec,
                       info, row_base, tolp);
  else
    hipLaunchKernelGGL(k_potrf_first<false>, dim3(1), dim3(64), 0, s, A, lda, m, Inv, ldi, dvec,
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
