// Device-side tile routines on the FP64 matrix cores, shared by the generic
// batched products and the ARA iteration kernels.
//
// MFMA f64 16x16x4 operand layout (measured on gfx950): lane l supplies
// A(l % 16, l / 16) and B(l / 16, l % 16); accumulator register r of lane l
// holds D(l / 16 + 4 r, l % 16).
#pragma once

#include <hip/hip_runtime.h>

namespace tlr {

typedef double d4 __attribute__((ext_vector_type(4)));

// Global-memory views of the pointers the kernels find in descriptors: the
// compiler cannot tell their address space and would emit flat accesses,
// whose completion counter is the one LDS accesses use, so that every wait
// for an LDS read would also wait for all outstanding memory loads.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) float gfloat;
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) dv2 gdv2;
typedef __attribute__((address_space(1))) int gint;
__device__ inline const gdouble* gmem(const double* p) { return (const gdouble*)p; }
__device__ inline gdouble* gmem(double* p) { return (gdouble*)p; }
__device__ inline const gfloat* gmem(const float* p) { return (const gfloat*)p; }
__device__ inline gint* gmem(int* p) { return (gint*)p; }
__device__ inline const gint* gmem(const int* p) { return (const gint*)p; }

// C(row0 : row0 + 16 FM, col0 : col0 + 16 FN) = alpha A^T B + beta C with A
// stored K x M and B stored K x N (column-major; the contraction runs down
// their columns), over k in [kbeg, kend).  NW waves of the workgroup take
// interleaved 16-row slices of K; within a slice lane (i, g) reads rows
// 4g..4g+3 of column i of A and of B, so both operands are read in 32-byte
// runs down their columns, and MFMA t of the slice consumes row 4g + t: the
// same permutation of k on both operands, so the sum is unchanged.  U slices
// per pass have all their loads in flight before the first MFMA (K is ~1000
// and the grids are small, so latency, not bandwidth, is the limit); loads
// past the end of K read a clamped in-range address and are zeroed.  The NW
// partial tiles are added in LDS (red, NW x FM FN 4 x 64) in a fixed order.
// Every thread of the workgroup must call it.
// With LOCAL set, the raw sum (no alpha, beta or bounds) is written to the
// dense 16 FM x 16 FN tile C (ld 16 FM) instead: a partial of a split-K sum.
template <int FM, int FN, int NW, int U = 4, bool LOCAL = false>
__device__ inline void tn_tile(const double* __restrict__ A, int lda, const double* __restrict__ B,
                               int ldb, double* C, int ldc, int M, int N, int kbeg, int kend,
                               double alpha, double beta, int row0, int col0,
                               double (*red)[FM * FN * 4][64]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  d4 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  const gdouble* acol[FM];
  const gdouble* bcol[FN];
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    const int i = row0 + a * 16 + li;
    acol[a] = gmem(A) + (size_t)(i < M ? i : 0) * lda;
  }
#pragma unroll
  for (int b = 0; b < FN; ++b) {
    const int j = col0 + b * 16 + li;
    bcol[b] = gmem(B) + (size_t)(j < N ? j : 0) * ldb;
  }
  for (int k0 = kbeg + wave * 16; k0 < kend; k0 += 16 * NW * U) {
    double av[U][FM][4], bv[U][FN][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kr = k0 + u * 16 * NW + 4 * g;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int kk = min(kr + t, kend - 1);
#pragma unroll
        for (int a = 0; a < FM; ++a) av[u][a][t] = acol[a][kk];
#pragma unroll
        for (int b = 0; b < FN; ++b) bv[u][b][t] = bcol[b][kk];
      }
    }
    // keep every load of the pass ahead of its first use (the scheduler
    // would otherwise pair each load with its use and serialise the
    // latency); rows past K are zeroed afterwards on the A side.  Columns of
    // A past M and of B past N were read from a clamped in-range address:
    // they only reach outputs that are not stored.
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (k0 + u * 16 * NW + 4 * g + t >= kend)
#pragma unroll
          for (int a = 0; a < FM; ++a) av[u][a][t] = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b)
            acc[a][b] =
                __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][a][t], bv[u][b][t], acc[a][b], 0, 0, 0);
  }
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave][(a * FN + b) * 4 + r][lane] = acc[a][b][r];
  __syncthreads();
  for (int e = threadIdx.x; e < FM * FN * 4 * 64; e += 64 * NW) {
    const int slot = e >> 6, l = e & 63;
    const int ab = slot >> 2, r = slot & 3;
    const int a = ab / FN, b = ab % FN;
    const int lr = a * 16 + (l >> 4) + 4 * r, lc = b * 16 + (l & 15);
    const int gr = row0 + lr, gc = col0 + lc;
    double v = red[0][slot][l];
#pragma unroll
    for (int w = 1; w < NW; ++w) v += red[w][slot][l];
    if (LOCAL) {
      gmem(C)[lr + lc * 16 * FM] = v;
      continue;
    }
    if (gr >= M || gc >= N) continue;
    gdouble* cp = gmem(C) + gr + (size_t)gc * ldc;
    double out = alpha * v;
    if (beta != 0.0) out += beta * *cp;
    *cp = out;
  }
}

// Packed low-precision copies of a row panel (the FP32 and BF16 mirrors of
// the factor's U panels, precision P = 1 and 2): the columns are cut into
// slices of Pack<P>::K columns; a slice holds the panel's row blocks of 16
// rows one after another, each stored as 64 lanes x Pack<P>::V values, lane
// i + 16 g holding row i and columns g V .. g V + V - 1 of the slice.  That is
// the MFMA operand of one wave: one contiguous 16-byte load per lane, 1 KiB
// per wave.  FP32: K = 16, V = 4 (four v_mfma_f32_16x16x4f32 per slice);
// BF16: K = 32, V = 8 (one v_mfma_f32_16x16x32_bf16).  A panel of m rows has
// ceil(m / 16) row blocks.
template <int P>
struct Pack;
template <>
struct Pack<1> {
  static constexpr int K = 16, V = 4;
};
template <>
struct Pack<2> {
  static constexpr int K = 32, V = 8;
};
__host__ __device__ inline size_t pack_index(int row, int col, int nrb, int pk, int pv) {
  return ((size_t)(col / pk) * nrb + (row >> 4)) * (size_t)(64 * pv) +
         (size_t)(((row & 15) + 16 * ((col % pk) / pv)) * pv + col % pv);
}
// BF16 bits of x: rounded to FP32, then to the nearest BF16, ties to even
// (finite values).
__device__ inline unsigned short bf16_bits(double x) {
  unsigned u = __float_as_uint((float)x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(1))) u4v gu4v;
// Row of the 16 x 16 block held by accumulator register r of lane l of the
// FP32-accumulating MFMAs (v_mfma_f32_16x16x4f32, v_mfma_f32_16x16x32_bf16;
// column l % 16), and its inverse: the register and lane group of a row.
__device__ inline int f32acc_row(int l, int r) { return 4 * (l >> 4) + r; }
__device__ inline void f32acc_slot(int row, int* r, int* grp) {
  *r = row & 3;
  *grp = row >> 2;
}

// Streaming product of a strip of 16 FM rows (256 threads, 4 waves):
//   C(r0 : r0 + 16 FM, 0 : N) = beta C + A0 B0 + A1 B1,
// A_s m x K_s, B_s K_s x N (column-major FP64), N <= 16 NF.  P1 selects how
// segment 1 is formed: 0, A1 column-major FP64 (ld lda1) on the FP64 matrix
// cores; 1 or 2, A1 packed FP32 or BF16 (lda1 = its number of row blocks),
// B1 rounded to the same precision, products accumulated in FP32 on the FP32
// or BF16 matrix cores, and added to the FP64 result of segment 0 at the end.
//
// FP64 segments: the waves take interleaved 16-wide slices of the K range, U
// slices per pass with all loads in flight; lane (i, g) reads rows i + 16 f of
// A for the four columns k0 + 4 g + t (128-byte runs per column over the 16
// lanes of a group, FM of them one after another down the column) and rows
// k0 + 4 g + t of column i of B, which serve all FM row blocks; MFMA t
// consumes k0 + 4 g + t on both operands.  Packed segment: the waves take
// interleaved slices, lane (i, g) loads its 16 bytes of each row block and
// the V rows of B that match them.  Either way every wave walks the same
// sequence of slices whatever FM, so the accumulation order of an output does
// not depend on the strip height.  The four partial strips are added in LDS
// (red, and red32 for the FP32 accumulators; 4 x FM NF 4 x 64 each) in a
// fixed order.  When ys is not NULL the final strip is also left in
// ys[row - r0][col] (after a barrier).
template <int NF, int P1, int FM = 1>
__device__ inline void seg_strip(const double* A0, int lda0, const double* B0, int ldb0, int K0,
                                 const void* A1v, int lda1, const double* B1, int ldb1, int K1,
                                 double* C, int ldc, int M, int N, double beta, int r0,
                                 double (*red)[FM * NF * 4][64], float (*red32)[FM * NF * 4][64],
                                 double (*ys)[16 * NF + 1]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  // rows r0 + 16 f + li (f < FM); rows past M read row 0 and are not stored
  int rowc[FM];
#pragma unroll
  for (int f = 0; f < FM; ++f) {
    const int row = r0 + 16 * f + li;
    rowc[f] = row < M ? row : 0;
  }
  d4 acc[FM][NF];
#pragma unroll
  for (int f = 0; f < FM; ++f)
#pragma unroll
    for (int b = 0; b < NF; ++b) acc[f][b] = d4{0.0, 0.0, 0.0, 0.0};
  // 64-row K blocks per round of loads
  constexpr int U = FM == 1 ? 4 : 2;
#pragma unroll
  for (int sg = 0; sg < 2; ++sg) {
    const int K = sg ? K1 : K0;
    if (K <= 0 || (sg == 1 && P1 != 0)) continue;
    const gdouble* __restrict__ A = gmem(sg ? (const double*)A1v : A0);
    const gdouble* __restrict__ B = gmem(sg ? B1 : B0);
    const size_t lda = sg ? lda1 : lda0, ldb = sg ? ldb1 : ldb0;
    const gdouble* bcol[NF];
#pragma unroll
    for (int b = 0; b < NF; ++b) {
      const int c = b * 16 + li;
      bcol[b] = B + (size_t)(c < N ? c : 0) * ldb;
    }
    for (int k0 = wave * 16; k0 < K; k0 += 64 * U) {
      double av[U][4][FM], bv[U][NF][4];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int kr = k0 + 64 * u + 4 * g;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int kk = min(kr + t, K - 1);
#pragma unroll
          for (int f = 0; f < FM; ++f) av[u][t][f] = A[rowc[f] + (size_t)kk * lda];
#pragma unroll
          for (int b = 0; b < NF; ++b) bv[u][b][t] = bcol[b][kk];
        }
      }
      // all loads of the pass are issued before the first use; rows past K
      // are zeroed afterwards on the A side (rows of A past M and columns of
      // B past N come from clamped in-range addresses and only reach outputs
      // that are not stored)
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int f = 0; f < FM; ++f)
            if (k0 + 64 * u + 4 * g + t >= K) av[u][t][f] = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int b = 0; b < NF; ++b)
              acc[f][b] =
                  __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][t][f], bv[u][b][t], acc[f][b], 0, 0, 0);
    }
  }
  f4v acc32[FM][NF];
#pragma unroll
  for (int f = 0; f < FM; ++f)
#pragma unroll
    for (int b = 0; b < NF; ++b) acc32[f][b] = f4v{0.f, 0.f, 0.f, 0.f};
  if constexpr (P1 != 0) {
    constexpr int PK = Pack<P1 == 0 ? 1 : P1>::K, PV = Pack<P1 == 0 ? 1 : P1>::V;
    constexpr int U1 = FM == 1 ? 4 : 2;
    const int nrb = lda1;
    const int nsl = (K1 + PK - 1) / PK;
    // the elements of a packed operand are 4 (FP32) or 2 (BF16) bytes: one
    // 16-byte run per lane and row block
    const char* base = (const char*)A1v;
    constexpr size_t blk_bytes = 64 * 16;   // 64 lanes x 16 bytes
    int rb[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) rb[f] = min((r0 >> 4) + f, nrb - 1);
    const gdouble* bcol[NF];
#pragma unroll
    for (int b = 0; b < NF; ++b) {
      const int c = b * 16 + li;
      bcol[b] = gmem(B1) + (size_t)(c < N ? c : 0) * ldb1;
    }
    for (int s0 = wave; s0 < nsl; s0 += 4 * U1) {
      u4v araw[U1][FM];
      double bv[U1][NF][PV];
#pragma unroll
      for (int u = 0; u < U1; ++u) {
        const int s = min(s0 + 4 * u, nsl - 1);
#pragma unroll
        for (int f = 0; f < FM; ++f)
          araw[u][f] = *(const gu4v*)(base + ((size_t)s * nrb + rb[f]) * blk_bytes + (size_t)lane * 16);
#pragma unroll
        for (int v = 0; v < PV; ++v) {
          const int kk = min(s * PK + g * PV + v, K1 - 1);
#pragma unroll
          for (int b = 0; b < NF; ++b) bv[u][b][v] = bcol[b][kk];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U1; ++u) {
        const int kb = (s0 + 4 * u) * PK + g * PV;   // first column of this lane's run
        if constexpr (P1 == 1) {
          // columns past K1 (the tail of the last slice, or a repeated
          // slice past the end) are zeroed on the A side
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int f = 0; f < FM; ++f) {
              const float a = kb + t < K1 ? __uint_as_float(araw[u][f][t]) : 0.f;
#pragma unroll
              for (int b = 0; b < NF; ++b)
                acc32[f][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, (float)bv[u][b][t],
                                                                   acc32[f][b], 0, 0, 0);
            }
        } else {
          u4v bw[NF];
#pragma unroll
          for (int b = 0; b < NF; ++b)
#pragma unroll
            for (int w = 0; w < 4; ++w)
              bw[b][w] = (unsigned)bf16_bits(bv[u][b][2 * w]) |
                         ((unsigned)bf16_bits(bv[u][b][2 * w + 1]) << 16);
#pragma unroll
          for (int f = 0; f < FM; ++f) {
            u4v a = araw[u][f];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
              const unsigned lo = kb + 2 * w < K1 ? 0x0000ffffu : 0u;
              const unsigned hi = kb + 2 * w + 1 < K1 ? 0xffff0000u : 0u;
              a[w] &= lo | hi;
            }
            const bf8v ab = __builtin_bit_cast(bf8v, a);
#pragma unroll
            for (int b = 0; b < NF; ++b)
              acc32[f][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  ab, __builtin_bit_cast(bf8v, bw[b]), acc32[f][b], 0, 0, 0);
          }
        }
      }
    }
  }
#pragma unroll
  for (int f = 0; f < FM; ++f)
#pragma unroll
    for (int b = 0; b < NF; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        red[wave][(f * NF + b) * 4 + r][lane] = acc[f][b][r];
        if (P1 != 0) red32[wave][(f * NF + b) * 4 + r][lane] = acc32[f][b][r];
      }
  __syncthreads();
  for (int e = threadIdx.x; e < FM * NF * 4 * 64; e += 256) {
    const int slot = e >> 6, l = e & 63;
    const int f = slot / (NF * 4), b = (slot >> 2) % NF, r = slot & 3;
    const int rl = (l >> 4) + 4 * r;   // row inside the 16 x 16 block
    const int rr = 16 * f + rl;
    const int c = b * 16 + (l & 15);
    double v = ((red[0][slot][l] + red[1][slot][l]) + red[2][slot][l]) + red[3][slot][l];
    if (P1 != 0) {
      int r32, grp;
      f32acc_slot(rl, &r32, &grp);
      const int s32 = (f * NF + b) * 4 + r32, l32 = 16 * grp + (l & 15);
      v += (((double)red32[0][s32][l32] + (double)red32[1][s32][l32]) +
            (double)red32[2][s32][l32]) + (double)red32[3][s32][l32];
    }
    if (r0 + rr < M && c < N) {
      gdouble* cp = gmem(C) + (r0 + rr) + (size_t)c * ldc;
      if (beta != 0.0) v += beta * *cp;
      *cp = v;
    } else {
      v = 0.0;
    }
    if (ys) ys[rr][c] = v;
  }
  if (ys) __syncthreads();
}

// C(row0 : row0 + BM, col0 : col0 + BN) = alpha A^T B + beta C with A stored
// K x M and B stored K x N (column-major, the contraction running down the
// columns), streamed through LDS in chunks of KC rows.  The loads are
// coalesced: KC / 2 consecutive threads read one column's KC-row run as
// 16-byte pairs (whole cache lines per instruction), the next chunk is
// loaded into registers while the MFMAs consume the current one from LDS,
// and the four waves split each chunk's 16-row slices; their partial tiles
// are added in LDS at the end.  16-byte loads when K and the leading
// dimensions are even and A, B 16-byte aligned, 8-byte loads otherwise; K >=
// 1.  Columns of A past M and of B past N are read
// from a clamped in-range column and only reach outputs that are not
// stored.  With store_t the tile goes to C transposed (element (r, c) at
// C[c + r ldc]).  256 threads; smem holds tn_lds_smem<BM, BN, KC>() doubles.
template <int BM, int BN, int KC>
constexpr int tn_lds_smem() {
  return ((BM + BN) * (KC + 2) > 3 * (BM / 16) * (BN / 16) * 4 * 64)
             ? (BM + BN) * (KC + 2)
             : 3 * (BM / 16) * (BN / 16) * 4 * 64;
}

template <int BM, int BN, int KC>
__device__ inline void tn_lds_tile(const double* __restrict__ A, int lda,
                                   const double* __restrict__ B, int ldb, double* C, int ldc,
                                   int M, int N, int K, double alpha, double beta, int row0,
                                   int col0, bool store_t, double* smem) {
  constexpr int FM = BM / 16, FN = BN / 16, LDK = KC + 2;
  constexpr int TPC = KC / 2;          // threads per column run (one 16-byte pair each)
  constexpr int CPR = 256 / TPC;       // columns per load round
  constexpr int AL = BM / CPR, BL = BN / CPR;
  static_assert(BM % CPR == 0 && BN % CPR == 0, "tile and chunk do not match the loader");
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int li = lane & 15, g = lane >> 4;
  double* As = smem;                   // As[c * LDK + k]
  double* Bs = smem + BM * LDK;
  const int lc = t / TPC, lk = (t % TPC) * 2;
  double2 ra[AL], rb[BL];
  // 16-byte loads when K and the leading dimensions are even and the
  // operands 16-byte aligned (a pair of rows is then wholly inside or
  // outside K), else two 8-byte loads per pair
  const bool vec = (K & 1) == 0 && (lda & 1) == 0 && (ldb & 1) == 0 &&
                   ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0;
  auto load = [&](int k0) {
    if (vec) {
      const int kk = min(k0 + lk, K - 2);
#pragma unroll
      for (int u = 0; u < AL; ++u) {
        const int c = min(row0 + lc + u * CPR, M - 1);
        const dv2 v = *(const gdv2*)(gmem(A) + (size_t)c * lda + kk);
        ra[u] = double2{v.x, v.y};
      }
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int c = min(col0 + lc + u * CPR, N - 1);
        const dv2 v = *(const gdv2*)(gmem(B) + (size_t)c * ldb + kk);
        rb[u] = double2{v.x, v.y};
      }
    } else {
      const int k0c = min(k0 + lk, K - 1), k1c = min(k0 + lk + 1, K - 1);
#pragma unroll
      for (int u = 0; u < AL; ++u) {
        const gdouble* col = gmem(A) + (size_t)min(row0 + lc + u * CPR, M - 1) * lda;
        ra[u] = double2{col[k0c], col[k1c]};
      }
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const gdouble* col = gmem(B) + (size_t)min(col0 + lc + u * CPR, N - 1) * ldb;
        rb[u] = double2{col[k0c], col[k1c]};
      }
    }
  };
  auto store = [&](int k0) {
    const bool ok0 = k0 + lk < K, ok1 = k0 + lk + 1 < K;
#pragma unroll
    for (int u = 0; u < AL; ++u)
      *(double2*)(As + (lc + u * CPR) * LDK + lk) =
          double2{ok0 ? ra[u].x : 0.0, ok1 ? ra[u].y : 0.0};
#pragma unroll
    for (int u = 0; u < BL; ++u)
      *(double2*)(Bs + (lc + u * CPR) * LDK + lk) =
          double2{ok0 ? rb[u].x : 0.0, ok1 ? rb[u].y : 0.0};
  };
  d4 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  load(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
    __syncthreads();   // the previous chunk's LDS reads are done
    store(k0);
    __syncthreads();
    if (k0 + KC < K) load(k0 + KC);
    // lane (i, g) takes rows kb .. kb + 3 of column i; MFMA tt consumes row
    // kb + tt on both operands
#pragma unroll
    for (int sl = wave; sl < KC / 16; sl += 4) {
      const int kb = sl * 16 + 4 * g;
      double av[FM][4], bv[FN][4];
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        const double2 x = *(const double2*)(As + (a * 16 + li) * LDK + kb);
        const double2 y = *(const double2*)(As + (a * 16 + li) * LDK + kb + 2);
        av[a][0] = x.x;
        av[a][1] = x.y;
        av[a][2] = y.x;
        av[a][3] = y.y;
      }
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const double2 x = *(const double2*)(Bs + (b * 16 + li) * LDK + kb);
        const double2 y = *(const double2*)(Bs + (b * 16 + li) * LDK + kb + 2);
        bv[b][0] = x.x;
        bv[b][1] = x.y;
        bv[b][2] = y.x;
        bv[b][3] = y.y;
      }
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][tt], bv[b][tt], acc[a][b], 0, 0, 0);
    }
  }
  // waves 1..3 park their partial tiles in LDS, wave 0 adds them (fixed order)
  __syncthreads();
  if (wave > 0) {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          smem[((wave - 1) * FM * FN * 4 + (a * FN + b) * 4 + r) * 64 + lane] = acc[a][b][r];
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double v = acc[a][b][r];
#pragma unroll
        for (int w = 0; w < 3; ++w) v += smem[(w * FM * FN * 4 + (a * FN + b) * 4 + r) * 64 + lane];
        const int gr = row0 + a * 16 + g + 4 * r, gc = col0 + b * 16 + li;
        if (gr < M && gc < N) {
          gdouble* cp = store_t ? gmem(C) + gc + (size_t)gr * ldc : gmem(C) + gr + (size_t)gc * ldc;
          double out = alpha * v;
          if (beta != 0.0) out += beta * *cp;
          *cp = out;
        }
      }
}

}  // namespace tlr
