// Block-wide FP64 dense linear algebra bodies shared by the single-problem kernels and the
// batched (one workgroup per problem) kernels: the 64 x 64 diagonal-block factor + inverse of
// the blocked Cholesky, a 64 x 64 FP64 GEMM tile, and workgroup-level drivers of the blocked
// factorisation and triangular solves.  Matrices are row-major with explicit leading dimensions.
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
// block is better conditioned than ~1e11; a rejected pivot is replaced by 1 so that no NaN
// spreads.  1/sqrt(d) is v_rsq_f64 refined by two Newton steps.
// ------------------------------------------------------------------------------------------
constexpr double kPivotRel = 1e-11;
constexpr int kLd = kNb + 1;

__device__ inline double rsqrt_f64(double d) {
  double r = __builtin_amdgcn_rsq(d);
  r = r * fma(-0.5 * d, r * r, 1.5);
  r = r * fma(-0.5 * d, r * r, 1.5);
  return r;
}


// ------------------------------------------------------------------------------------------
// 16 x 16 leaf, one wave, registers only: lane r (r = lane % 16; the four 16-lane rows of the
// wave hold the same data) keeps row r of the leaf in a[].  Column C: the pivot comes from lane
// C, every lane scales its entry, l_r = a[C] / sqrt(d), and subtracts l_r l_q from its entries
// q > C.  Entries right of the diagonal are updated too and never read.  The inverse: lane j
// computes column j of the leaf's L^{-1} by forward substitution, reading the rows of L from the
// lanes that hold them.  Values move between lanes by DPP row broadcasts (row_newbcast: every
// lane of a 16-lane row receives lane n of that row).
// ------------------------------------------------------------------------------------------
constexpr int kLeaf = 16;

template <int N>
__device__ __attribute__((always_inline)) inline double row_bcast(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x150 + N, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x150 + N, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

template <int C, int Q>
__device__ __attribute__((always_inline)) inline void leaf_update(double (&a)[kLeaf], double l) {
  if constexpr (Q > C) a[Q] = fma(-l, row_bcast<Q>(l), a[Q]);
}

template <int C, int... Qs>
__device__ __attribute__((always_inline)) inline void leaf_column(
    std::integer_sequence<int, Qs...>, double (&a)[kLeaf], int r, double d0, double& isd_own,
    bool& bad_any) {
  double d = row_bcast<C>(a[C]);
  const bool bad = !(d > kPivotRel * row_bcast<C>(d0)) || !isfinite(d);
  bad_any |= bad;
  if (bad) d = 1.0;
  const double isd = rsqrt_f64(d);
  const double l = (r == C ? d : a[C]) * isd;
  a[C] = l;
  if (r == C) isd_own = isd;
  (leaf_update<C, Qs>(a, l), ...);
}

template <int RR, int Q>
__device__ __attribute__((always_inline)) inline void leaf_inverse_term(
    double& s0, double& s1, const double (&a)[kLeaf], const double (&y)[kLeaf]) {
  if constexpr (Q < RR) {
    const double lq = row_bcast<RR>(a[Q]);        // L[RR][Q]
    if constexpr ((Q & 1) != 0) s1 = fma(lq, y[Q], s1);
    else s0 = fma(lq, y[Q], s0);
  }
}

template <int RR, int... Qs>
__device__ __attribute__((always_inline)) inline void leaf_inverse_row(
    std::integer_sequence<int, Qs...>, double (&y)[kLeaf], const double (&a)[kLeaf], int j,
    double isd_own) {
  double s0 = 0.0, s1 = 0.0;
  (leaf_inverse_term<RR, Qs>(s0, s1, a, y), ...);
  const double id = row_bcast<RR>(isd_own);
  y[RR] = j == RR ? id : (j < RR ? -id * (s0 + s1) : 0.0);
}

template <int... Cs>
__device__ __attribute__((always_inline)) inline void leaf_factor(
    std::integer_sequence<int, Cs...>, double (&a)[kLeaf], int r, double d0, double& isd_own,
    bool& bad_any) {
  (leaf_column<Cs>(std::make_integer_sequence<int, kLeaf>{}, a, r, d0, isd_own, bad_any), ...);
}

template <int... Rs>
__device__ __attribute__((always_inline)) inline void leaf_inverse(
    std::integer_sequence<int, Rs...>, double (&y)[kLeaf], const double (&a)[kLeaf], int j,
    double isd_own) {
  (leaf_inverse_row<Rs>(std::make_integer_sequence<int, kLeaf>{}, y, a, j, isd_own), ...);
}

// The leaf at (b, b): its L into S (lower part; the part right of the diagonal is scratch) and
// its inverse into the same block of Y.  Called by one whole wave.
__device__ __attribute__((always_inline)) inline void leaf_factor_inv(double (*S)[kLd],
                                                                       double (*Y)[kLd],
                                                                       const double* D0, int b,
                                                                       bool& bad_any) {
  const int lane = threadIdx.x & 63, r = lane & 15;
  double a[kLeaf];
#pragma unroll
  for (int q = 0; q < kLeaf; ++q) a[q] = S[b + r][b + q];
  const double d0 = D0[b + r];
  double isd_own = 1.0;
  leaf_factor(std::make_integer_sequence<int, kLeaf>{}, a, r, d0, isd_own, bad_any);
  double y[kLeaf];
  leaf_inverse(std::make_integer_sequence<int, kLeaf>{}, y, a, r, isd_own);
  if (lane < kLeaf) {
#pragma unroll
    for (int q = 0; q < kLeaf; ++q) S[b + r][b + q] = a[q];
#pragma unroll
    for (int rr = 0; rr < kLeaf; ++rr) Y[b + rr][b + r] = y[rr];
  }
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

// Factor and invert the 64 x 64 block already in S (LDS; rows / columns >= kb hold the identity)
// with D0 (LDS) the diagonal before any elimination.  On return the lower triangle of S holds
// L11 and Y holds L11^{-1} (strict upper triangle zero); buf is kFactorBuf doubles of LDS
// scratch.  Raises VL_ERR_SINGULAR on a rejected pivot.  Starts and ends with a workgroup
// barrier.  Blocked by 16-column leaves (right-looking), 16 x 16 block products on MFMA:
//   leaf s (wave 0):            L_ss and L_ss^{-1}
//   panel (wave per block row):  L_is = A_is L_ss^{-T} for the block rows below the leaf
//   trailing (wave per block):   A_ij -= L_is L_js^T  (blocks on and below the diagonal)
// then the blocks of L^{-1} below the diagonal, block row t after block row t - 1, one wave per
// block:  Y_tu = -Y_tt sum_{u <= v < t} L_tv Y_vu.
constexpr int kFactorBuf = 3 * kLeaf * kLeaf;

__device__ __attribute__((always_inline)) inline void block_factor_inv(double (*S)[kLd],
                                                                        double (*Y)[kLd],
                                                                        double* buf,
                                                                        const double* D0,
                                                                        int32_t* st) {
  const int tid = threadIdx.x, w = tid >> 6;
  constexpr int kB = kNb / kLeaf;  // 4 block rows
  for (int e = tid; e < kNb * kNb; e += 256) Y[e >> 6][e & 63] = 0.0;
  __syncthreads();
  bool bad_any = false;
  for (int sb = 0; sb < kB; ++sb) {
    const int b = sb * kLeaf;
    if (w == 0) leaf_factor_inv(S, Y, D0, b, bad_any);
    __syncthreads();
    if (sb == kB - 1) break;
    // panel: wave w takes block row sb + 1 + w (reads and writes only its own block)
    if (sb + 1 + w < kB) {
      const int i0 = (sb + 1 + w) * kLeaf;
      f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
      mfma_blk16<true>(&S[i0][b], kLd, &Y[b][b], kLd, acc);
      blk16_each(acc, [&](int i, int j, double v) { S[i0 + i][b + j] = v; });
    }
    __syncthreads();
    // trailing blocks (i, j), sb < j <= i < kB
    const int t = kB - 1 - sb, nblk = t * (t + 1) / 2;
    for (int e = w; e < nblk; e += 4) {
      int ii = 0;
      while ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
      const int jj = e - ii * (ii + 1) / 2;
      const int i0 = (sb + 1 + ii) * kLeaf, j0 = (sb + 1 + jj) * kLeaf;
      f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
      mfma_blk16<true>(&S[i0][b], kLd, &S[j0][b], kLd, acc);
      blk16_each(acc, [&](int i, int j, double v) { S[i0 + i][j0 + j] -= v; });
    }
    __syncthreads();
  }
  // blocks of L^{-1} below the diagonal; wave u computes block (t, u), u < t
  for (int t = 1; t < kB; ++t) {
    if (w < t) {
      const int u = w;
      f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
      for (int v = u; v < t; ++v)
        mfma_blk16<false>(&S[t * kLeaf][v * kLeaf], kLd, &Y[v * kLeaf][u * kLeaf], kLd, acc);
      double* T = buf + u * kLeaf * kLeaf;
      blk16_each(acc, [&](int i, int j, double v) { T[i * kLeaf + j] = v; });
      // the same wave reads its block back (LDS accesses of a wave complete in order)
      f64x4_t acc2 = {0.0, 0.0, 0.0, 0.0};
      mfma_blk16<false>(&Y[t * kLeaf][t * kLeaf], kLd, T, kLeaf, acc2);
      blk16_each(acc2, [&](int i, int j, double v) { Y[t * kLeaf + i][u * kLeaf + j] = -v; });
    }
    __syncthreads();
  }
  if (bad_any) raise_status(st, VL_ERR_SINGULAR);
}

// The diagonal block at A (kb x kb, leading dimension lda) factored and inverted: L11 into L
// (kb x kb, strict upper part written as zero), L11^{-1} into Linv (64 x 64, dense).
__device__ inline void potf2_inv_block(const double* __restrict__ A, int64_t lda, int kb,
                                const double* __restrict__ diag0, double* __restrict__ L,
                                int64_t ldl, double* __restrict__ Linv, int32_t* st) {
  __shared__ double S[kNb][kLd];
  __shared__ double Y[kNb][kLd];
  __shared__ double buf[kFactorBuf];
  __shared__ double D0[kNb];
  const int t = threadIdx.x;
  for (int e = t; e < kNb * kNb; e += 256) {
    const int r = e >> 6, q = e & 63;
    S[r][q] = (r < kb && q < kb) ? A[(int64_t)r * lda + q] : (r == q ? 1.0 : 0.0);
  }
  if (t < kNb) D0[t] = t < kb ? diag0[t] : 1.0;
  block_factor_inv(S, Y, buf, D0, st);
  for (int e = t; e < kNb * kNb; e += 256) {
    const int r = e >> 6, q = e & 63;
    if (r < kb && q < kb) L[(int64_t)r * ldl + q] = q <= r ? S[r][q] : 0.0;
    Linv[e] = q <= r ? Y[r][q] : 0.0;
  }
  __syncthreads();
}

// ------------------------------------------------------------------------------------------
// C = beta C + alpha op(A) op(B); FP64; 64 x 64 tiles, 256 threads x (4 x 4), K step 16;
// tri skips the K range a triangular op(A) holds zeros in (i0 and K steps are multiples of 16).
// op(A) is M x K: transA ? A[k * lda + i] : A[i * lda + k]; op(B) is K x N likewise.
// lower_only: tiles strictly above the diagonal are skipped (and in diagonal tiles only
// entries with j <= i are written).
// ------------------------------------------------------------------------------------------
__device__ inline void gemm_f64_tile(int64_t M, int64_t N, int64_t K, double alpha,
                              const double* __restrict__ A, int64_t lda, int transA,
                              const double* __restrict__ Bm, int64_t ldb, int transB, double beta,
                              double* __restrict__ C, int64_t ldc, int lower_only, int64_t i0,
                              int64_t j0, int tri = 0) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  if (lower_only && j0 > i0 + 63) return;
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  // this thread's four loads per operand and K step; consecutive threads walk the contiguous
  // dimension of each operand
  int ak[4], ai[4], bk[4], bj[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u;
    ak[u] = transA ? e / 64 : e % 16;
    ai[u] = transA ? e % 64 : e / 16;
    bk[u] = transB ? e % 16 : e / 64;
    bj[u] = transB ? e / 16 : e % 64;
  }
  auto load = [&](int64_t k0, double (&ra)[4], double (&rb)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t gi = i0 + ai[u], gk = k0 + ak[u];
      ra[u] = (gi < M && gk < K) ? (transA ? A[gk * lda + gi] : A[gi * lda + gk]) : 0.0;
      const int64_t gj = j0 + bj[u], gk2 = k0 + bk[u];
      rb[u] = (gj < N && gk2 < K) ? (transB ? Bm[gj * ldb + gk2] : Bm[gk2 * ldb + gj]) : 0.0;
    }
  };
  // tri = 1: op(A) lower triangular (terms k > i vanish); tri = 2: upper (k < i vanish)
  const int64_t kbeg = tri == 2 ? (i0 < K ? i0 : K) : 0;
  const int64_t kend = tri == 1 ? (i0 + 64 < K ? i0 + 64 : K) : K;
  double acc[4][4] = {};
  double ra[4], rb[4];
  load(kbeg, ra, rb);
  for (int64_t k0 = kbeg; k0 < kend; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      As[ak[u]][ai[u]] = ra[u];
      Bs[bk[u]][bj[u]] = rb[u];
    }
    __syncthreads();
    if (k0 + 16 < kend) load(k0 + 16, ra, rb);   // in flight during the products below
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        a[r] = As[kk][ti + 16 * r];
        b[r] = Bs[kk][tj + 16 * r];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = fma(a[r], b[q], acc[r][q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t gi = i0 + ti + 16 * r, gj = j0 + tj + 16 * q;
      if (gi < M && gj < N && (!lower_only || gj <= gi)) {
        double* c = C + gi * ldc + gj;
        *c = (beta == 0.0 ? 0.0 : beta * *c) + alpha * acc[r][q];
      }
    }
}

// ------------------------------------------------------------------------------------------
// The same factorisation and solves run by ONE workgroup of 256 threads (small matrices, one
// workgroup per problem of a batch).  Phases are separated by workgroup barriers; the
// workgroup's own global-memory writes are visible to it after each barrier.
// ------------------------------------------------------------------------------------------
__device__ inline void wg_gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                            int64_t lda, bool transA, const double* B, int64_t ldb, bool transB,
                            double beta, double* C, int64_t ldc, bool lower_only) {
  const int64_t tm = ceil_div(M, 64), tn = ceil_div(N, 64);
  for (int64_t t = 0; t < tm * tn; ++t)
    gemm_f64_tile(M, N, K, alpha, A, lda, transA ? 1 : 0, B, ldb, transB ? 1 : 0, beta, C, ldc,
                  lower_only ? 1 : 0, (t / tn) * 64, (t % tn) * 64);
  __syncthreads();
}

__device__ inline void wg_potrf_lower(double* A, int64_t n, int64_t lda, double* L, int64_t ldl,
                               double* ws, int32_t* st) {
  double* diag0 = ws;
  double* inv = ws + n;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) diag0[i] = A[i * lda + i];
  __syncthreads();
  for (int64_t k0 = 0; k0 < n; k0 += kNb) {
    const int kb = (int)(n - k0 < kNb ? n - k0 : kNb);
    double* invk = inv + (k0 / kNb) * kNb * kNb;
    potf2_inv_block(A + k0 * lda + k0, lda, kb, diag0 + k0, L + k0 * ldl + k0, ldl, invk, st);
    const int64_t rest = n - k0 - kb;
    if (rest <= 0) break;
    wg_gemm_f64(rest, kb, kb, 1.0, A + (k0 + kb) * lda + k0, lda, false, invk, kNb, true, 0.0,
                L + (k0 + kb) * ldl + k0, ldl, false);
    wg_gemm_f64(rest, rest, kb, -1.0, L + (k0 + kb) * ldl + k0, ldl, false,
                L + (k0 + kb) * ldl + k0, ldl, true, 1.0, A + (k0 + kb) * lda + (k0 + kb), lda,
                true);
  }
}

__device__ inline void wg_trsm_lower(const double* L, int64_t n, int64_t ldl, const double* ws,
                              bool trans, double* B, int64_t nrhs, int64_t ldb, double* X,
                              int64_t ldx) {
  const double* inv = ws + n;
  const int64_t nblk = ceil_div(n, kNb);
  if (!trans) {
    for (int64_t b = 0; b < nblk; ++b) {
      const int64_t k0 = b * kNb;
      const int kb = (int)(n - k0 < kNb ? n - k0 : kNb);
      wg_gemm_f64(kb, nrhs, kb, 1.0, inv + b * kNb * kNb, kNb, false, B + k0 * ldb, ldb, false,
                  0.0, X + k0 * ldx, ldx, false);
      const int64_t rest = n - k0 - kb;
      if (rest > 0)
        wg_gemm_f64(rest, nrhs, kb, -1.0, L + (k0 + kb) * ldl + k0, ldl, false, X + k0 * ldx,
                    ldx, false, 1.0, B + (k0 + kb) * ldb, ldb, false);
    }
  } else {
    for (int64_t b = nblk - 1; b >= 0; --b) {
      const int64_t k0 = b * kNb;
      const int kb = (int)(n - k0 < kNb ? n - k0 : kNb);
      wg_gemm_f64(kb, nrhs, kb, 1.0, inv + b * kNb * kNb, kNb, true, B + k0 * ldb, ldb, false,
                  0.0, X + k0 * ldx, ldx, false);
      if (k0 > 0)
        wg_gemm_f64(k0, nrhs, kb, -1.0, L + k0 * ldl, ldl, true, X + k0 * ldx, ldx, false, 1.0, B,
                    ldb, false);
    }
  }
}

}  // namespace vl
