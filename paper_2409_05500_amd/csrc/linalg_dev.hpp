// The 64 x 64 diagonal-block factor + inverse of the blocked Cholesky (LDS in, LDS out), shared
// by the single-problem and the batched factorisation kernels.  Matrices are row-major.
#pragma once
#include <math.h>

#include <utility>

#include "common.hpp"

namespace vl {

constexpr int kNb = 64;  // panel width

// ------------------------------------------------------------------------------------------
// Diagonal block of the blocked Cholesky (kb <= 64; rows/columns >= kb act as identity): its
// factor L11 and the inverse L11^{-1}.  A pivot d is rejected (VL_ERR_SINGULAR) unless
// d > kPivotRel * diag0 (the diagonal entry before any elimination), i.e. unless the leading
// block is better conditioned than ~1e11; a rejected pivot is raised to that floor (to 1 when
// diag0 itself is not a positive finite number), so a non-positive pivot spreads no NaN.  The
// floor is one v_max_f64 on the pivot chain (maxNum: a NaN pivot takes the floor too); the test
// that raises the status runs beside the chain.
// ------------------------------------------------------------------------------------------
constexpr double kPivotRel = 1e-11;
constexpr int kLd = kNb + 1;

// sqrt(d) and 1/(2 sqrt(d)) from v_rsq_f64 by two coupled Goldschmidt steps
// (g -> sqrt(d), h -> 1/(2 sqrt(d)); each step r = 1/2 - g h, g += g r, h += h r, the error
// squaring per step): five dependent operations after the seed, one fewer than two Newton
// steps on 1/sqrt(d).
struct SqrtPair {
  double g, h;
};
__device__ __attribute__((always_inline)) inline SqrtPair sqrt_pair_f64(double d) {
  const double y = __builtin_amdgcn_rsq(d);
  double g = d * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  return {g, h};
}

// the pivot floor of a row whose diagonal before elimination is d0
__device__ __attribute__((always_inline)) inline double pivot_floor(double d0) {
  return (d0 > 0.0 && d0 < INFINITY) ? kPivotRel * d0 : 1.0;
}


// ------------------------------------------------------------------------------------------
// 16 x 16 leaf, one wave, registers only: lane r (r = lane % 16; the four 16-lane rows of the
// wave hold the same data) keeps row r of the leaf in a[] and, in y[], the column r of the
// leaf's inverse as the forward substitution L y = e_r runs column by column.  Column C: the
// pivot comes from lane C; every lane forms l_r = a_r[C] / sqrt(d) and the final entry
// Y[C][r] = y_C / sqrt(d); then for each later column Q the one broadcast l_Q = L[Q][C] serves
// both the elimination, a_r[Q] -= l_r l_Q, and the substitution, y_Q -= l_Q Y[C][r].  Entries
// right of the diagonal are updated too and never read.  Values move between lanes by DPP row
// broadcasts (row_newbcast: every lane of a 16-lane row receives lane n of that row).
// ------------------------------------------------------------------------------------------
constexpr int kLeaf = 16;

// One v_mov_b64_dpp into a fresh register (64-bit DPP takes row_newbcast on gfx950; every source
// lane of a row broadcast exists, so bound_ctrl changes nothing).  The 32-bit-pair form with a
// zeroed "old" operand took four instructions per broadcast.
template <int N>
__device__ __attribute__((always_inline)) inline double row_bcast(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + N, 0xF, 0xF, true);
}

template <int C, int Q>
__device__ __attribute__((always_inline)) inline void leaf_update(double (&a)[kLeaf],
                                                                  double (&y)[kLeaf], double l,
                                                                  double yc) {
  if constexpr (Q > C) {
    const double lq = row_bcast<Q>(l);   // L[Q][C]
    a[Q] = fma(-l, lq, a[Q]);
    y[Q] = fma(-lq, yc, y[Q]);
  }
}

template <int C, int... Qs>
__device__ __attribute__((always_inline)) inline void leaf_column(
    std::integer_sequence<int, Qs...>, double (&a)[kLeaf], double (&y)[kLeaf], double floor_own,
    bool& bad_any) {
  const double d_raw = row_bcast<C>(a[C]);
  const double fl = row_bcast<C>(floor_own);
  bad_any |= !(d_raw > fl) || !isfinite(d_raw);
  const double d = __builtin_fmax(d_raw, fl);
  // on lane C, a_CC equals the pivot unless it was rejected (then the status is raised and the
  // leaf's values only need to stay finite)
  const SqrtPair sp = sqrt_pair_f64(d);
  const double l = (2.0 * a[C]) * sp.h;
  const double yc = y[C] * (2.0 * sp.h);
  y[C] = yc;
  (leaf_update<C, Qs>(a, y, l, yc), ...);
}

template <int... Cs>
__device__ __attribute__((always_inline)) inline void leaf_factor(
    std::integer_sequence<int, Cs...>, double (&a)[kLeaf], double (&y)[kLeaf], double floor_own,
    bool& bad_any) {
  (leaf_column<Cs>(std::make_integer_sequence<int, kLeaf>{}, a, y, floor_own, bad_any), ...);
}

// The leaf at (b, b) of S: on return y[rr] = Y[b + rr][b + r] (r = lane % 16) of its inverse,
// zeros above the diagonal included.  S is read, not written: the callers need only the
// inverse of a diagonal leaf.  Called by one whole wave.
__device__ __attribute__((always_inline)) inline void leaf_factor_regs(const double (*S)[kLd],
                                                                        const double* D0, int b,
                                                                        bool& bad_any,
                                                                        double (&y)[kLeaf]) {
  const int r = threadIdx.x & 15;
  double a[kLeaf];
#pragma unroll
  for (int q = 0; q < kLeaf; ++q) {
    a[q] = S[b + r][b + q];
    y[q] = q == r ? 1.0 : 0.0;
  }
  const double floor_own = pivot_floor(D0[b + r]);
  leaf_factor(std::make_integer_sequence<int, kLeaf>{}, a, y, floor_own, bad_any);
}

__device__ __attribute__((always_inline)) inline void leaf_store_y(double (*Y)[kLd], int b,
                                                                    const double (&y)[kLeaf]) {
  const int lane = threadIdx.x & 63;
  if (lane < kLeaf) {
#pragma unroll
    for (int rr = 0; rr < kLeaf; ++rr) Y[b + rr][b + lane] = y[rr];
  }
}

// The leaf at (b, b): its inverse into the same block of Y.
__device__ __attribute__((always_inline)) inline void leaf_factor_inv(const double (*S)[kLd],
                                                                       double (*Y)[kLd],
                                                                       const double* D0, int b,
                                                                       bool& bad_any) {
  double y[kLeaf];
  leaf_factor_regs(S, D0, b, bad_any, y);
  leaf_store_y(Y, b, y);
}

typedef double f64x4_t __attribute__((ext_vector_type(4)));

// acc += P Q for 16 x 16 blocks in LDS: P[i][k] = P0[i * ldp + k]; Q[k][j] = Q0[k * ldq + j]
// (kTQ: Q[k][j] = Q0[j * ldq + k]).  One wave, v_mfma_f64_16x16x4f64 (A operand lane l ->
// (row l % 16, k l / 16), B operand -> (k l / 16, column l % 16)).
template <bool kTQ>
__device__ inline void mfma_blk16(const double* P0, int ldp, const double* Q0, int ldq,
                                  f64x4_t& acc) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < kLeaf; kk += 4) {
    const double a = P0[li * ldp + kk + lk];
    const double b = kTQ ? Q0[li * ldq + kk + lk] : Q0[(kk + lk) * ldq + li];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
}

// result element (lane l, register r) of a 16 x 16 block product: row l / 16 + 4 r, column l % 16
template <class F>
__device__ inline void blk16_each(const f64x4_t& acc, F f) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < 4; ++r) f((lane >> 4) + 4 * r, lane & 15, acc[r]);
}

// Block (t, u), u < t, of L^{-1} below the diagonal: Y_tu = -Y_tt sum_{u <= v < t} L_tv Y_vu.
// One wave; T is 16 x 16 doubles of LDS scratch of its own.
__device__ __attribute__((always_inline)) inline void inv_block(double (*S)[kLd], double (*Y)[kLd],
                                                                double* T, int t, int u) {
  f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int v = u; v < t; ++v)
    mfma_blk16<false>(&S[t * kLeaf][v * kLeaf], kLd, &Y[v * kLeaf][u * kLeaf], kLd, acc);
  blk16_each(acc, [&](int i, int j, double v) { T[i * kLeaf + j] = v; });
  // the same wave reads its block back (LDS accesses of a wave complete in order)
  f64x4_t acc2 = {0.0, 0.0, 0.0, 0.0};
  mfma_blk16<false>(&Y[t * kLeaf][t * kLeaf], kLd, T, kLeaf, acc2);
  blk16_each(acc2, [&](int i, int j, double v) { Y[t * kLeaf + i][u * kLeaf + j] = -v; });
}

// Factor and invert the 64 x 64 block already in S (LDS; rows / columns >= kb hold the identity)
// with D0 (LDS) the diagonal before any elimination.  On return Y holds L11^{-1} in its diagonal
// 16 x 16 blocks (zeros above their diagonals included) and in the blocks below them; the blocks
// above are neither written nor read.  The blocks of S below the diagonal leaves hold those of
// L11 (the leaves themselves keep the updated input); buf is kFactorBuf doubles of LDS
// scratch.  Raises
// VL_ERR_SINGULAR on a rejected pivot.  Starts and ends with a workgroup barrier.  Blocked by
// 16-column leaves (right-looking), 16 x 16 block products on MFMA; after leaf s:
//   panel (wave per block row):  L_is = A_is L_ss^{-T} for the block rows i > s
//   then wave 0 alone updates the next diagonal block, A_{s+1,s+1} -= L_{s+1,s} L_{s+1,s}^T,
//   and factors leaf s + 1 at once, while waves 1.. apply the rest of the trailing update
//   (A_ij -= L_is L_js^T, s < j <= i, (i, j) != (s+1, s+1)) and row s of L^{-1} below the
//   diagonal, Y_su = -Y_ss sum_{u <= v < s} L_sv Y_vu (it needs only leaves <= s and panels
//   < s).  The last row of L^{-1} follows the last leaf.
constexpr int kFactorBuf = 3 * kLeaf * kLeaf;

//
// block_factor_rest is the part after leaf 0: it starts once Y's block (0, 0) holds the leaf's
// inverse and S holds the input (a workgroup barrier after those writes); bad_any carries the
// pivot test of leaf 0.
__device__ __attribute__((always_inline)) inline void block_factor_rest(double (*S)[kLd],
                                                                         double (*Y)[kLd],
                                                                         double* buf,
                                                                         const double* D0,
                                                                         int32_t* st,
                                                                         bool bad_any) {
  const int tid = threadIdx.x, w = tid >> 6;
  constexpr int kB = kNb / kLeaf;  // 4 block rows
  for (int sb = 0; sb < kB - 1; ++sb) {
    const int b = sb * kLeaf;
    // panel: wave w takes block row sb + 1 + w (reads and writes only its own block)
    if (sb + 1 + w < kB) {
      const int i0 = (sb + 1 + w) * kLeaf;
      f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
      mfma_blk16<true>(&S[i0][b], kLd, &Y[b][b], kLd, acc);
      blk16_each(acc, [&](int i, int j, double v) { S[i0 + i][b + j] = v; });
    }
    __syncthreads();
    if (w == 0) {
      const int d0 = b + kLeaf;
      f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
      mfma_blk16<true>(&S[d0][b], kLd, &S[d0][b], kLd, acc);
      blk16_each(acc, [&](int i, int j, double v) { S[d0 + i][d0 + j] -= v; });
      // the same wave reads the block back (LDS accesses of a wave complete in order)
      leaf_factor_inv(S, Y, D0, d0, bad_any);
    } else {
      // tasks: the trailing blocks (i, j), sb < j <= i < kB, but (sb+1, sb+1), then the blocks
      // (sb, u), u < sb, of L^{-1}; round-robin over waves 1..3
      const int t = kB - 1 - sb, ntrail = t * (t + 1) / 2 - 1;
      for (int e = w - 1; e < ntrail + sb; e += 3) {
        if (e < ntrail) {
          const int f = e + 1;                   // skip block 0 = (sb+1, sb+1)
          int ii = 0;
          while ((ii + 1) * (ii + 2) / 2 <= f) ++ii;
          const int jj = f - ii * (ii + 1) / 2;
          const int i0 = (sb + 1 + ii) * kLeaf, j0 = (sb + 1 + jj) * kLeaf;
          f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
          mfma_blk16<true>(&S[i0][b], kLd, &S[j0][b], kLd, acc);
          blk16_each(acc, [&](int i, int j, double v) { S[i0 + i][j0 + j] -= v; });
        } else {
          inv_block(S, Y, buf + (w - 1) * kLeaf * kLeaf, sb, e - ntrail);
        }
      }
    }
    __syncthreads();
  }
  // the last row of L^{-1}: blocks (kB - 1, u), one wave each
  if (w < kB - 1) inv_block(S, Y, buf + w * kLeaf * kLeaf, kB - 1, w);
  __syncthreads();
  if (bad_any) raise_status(st, VL_ERR_SINGULAR);
}

__device__ __attribute__((always_inline)) inline void block_factor_inv(double (*S)[kLd],
                                                                        double (*Y)[kLd],
                                                                        double* buf,
                                                                        const double* D0,
                                                                        int32_t* st) {
  __syncthreads();
  bool bad_any = false;
  if ((threadIdx.x >> 6) == 0) leaf_factor_inv(S, Y, D0, 0, bad_any);
  __syncthreads();
  block_factor_rest(S, Y, buf, D0, st, bad_any);
}

}  // namespace vl
