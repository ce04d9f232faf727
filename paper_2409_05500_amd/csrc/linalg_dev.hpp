// Block-wide FP64 dense linear algebra bodies shared by the single-problem kernels and the
// batched (one workgroup per problem) kernels: the 64 x 64 diagonal-block factor + inverse of
// the blocked Cholesky, a 64 x 64 FP64 GEMM tile, and workgroup-level drivers of the blocked
// factorisation and triangular solves.  Matrices are row-major with explicit leading dimensions.
#pragma once
#include <math.h>

#include "common.hpp"

namespace vl {

constexpr int kNb = 64;  // panel width

// ------------------------------------------------------------------------------------------
// Diagonal block of the blocked Cholesky (kb <= 64; rows/columns >= kb act as identity), one
// workgroup of 256 threads, in LDS.  Produces the factor L11 and its inverse, recursively as
// 2 x 2 blocks of 32:
//   [L11 L21; . L22]:  factor+invert A11;  L21 = A21 L11^{-T};  A22 -= L21 L21^T;
//   factor+invert A22;  (L^{-1})21 = -L22^{-1} L21 L11^{-1}.
// A 32-block is factored by right-looking elimination applied to [A | I] (the identity ends as
// the inverse).  Column c, phase 1 (d = A[c][c], column c of A and row c of Y unscaled):
//     A[r][q] -= (A[r][c] / d) A[q][c]   (c < q <= r),   Y[r][q] -= (A[r][c] / d) Y[c][q]  (q <= c)
// phase 2 scales column c of A and row c of Y by 1/sqrt(d) (A[c][c] = sqrt(d)); phase 2 of column
// c touches only column c of A and row c of Y, which phase 1 of column c + 1 does not, so one
// barrier per column suffices.  1/sqrt(d) is v_rsq_f64 refined by two Newton steps.
// A pivot d is rejected (VL_ERR_SINGULAR) unless d > kPivotRel * diag0 (the diagonal entry before
// any elimination), i.e. unless the leading block is better conditioned than ~1e11; a rejected
// pivot is replaced by 1 so that no NaN spreads.
// ------------------------------------------------------------------------------------------
constexpr double kPivotRel = 1e-11;
constexpr int kLd = kNb + 1;

__device__ inline double rsqrt_f64(double d) {
  double r = __builtin_amdgcn_rsq(d);
  r = r * fma(-0.5 * d, r * r, 1.5);
  r = r * fma(-0.5 * d, r * r, 1.5);
  return r;
}

// Factor and invert the 32 x 32 diagonal block at (b, b) of S, writing the inverse into Y at
// (b, b).  Thread t: column q = t & 31, rows w + 8 k (w = t >> 5, k = 0..3).  Ends with a
// workgroup barrier.
__device__ inline void factor_inv32(double (*S)[kLd], double (*Y)[kLd], const double* D0, int b,
                             bool& bad_any) {
  const int t = threadIdx.x, q = t & 31, w = t >> 5;
  for (int c = 0; c < 32; ++c) {
    double d = S[b + c][b + c];
    const bool bad = !(d > kPivotRel * D0[b + c]) || !isfinite(d);
    bad_any |= bad;
    if (bad) d = 1.0;
    const double inv_sd = rsqrt_f64(d);
    const double inv_d = inv_sd * inv_sd;
    // phase 1: all reads first
    const double colq = S[b + q][b + c];
    const double rowq = Y[b + c][b + q];
    double arc[4], cur[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = w + 8 * k;
      arc[k] = S[b + r][b + c];
      cur[k] = q > c ? S[b + r][b + q] : Y[b + r][b + q];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = w + 8 * k;
      if (r > c) {
        const double f = arc[k] * inv_d;
        if (q > c) {
          if (q <= r) S[b + r][b + q] = cur[k] - f * colq;
        } else {
          Y[b + r][b + q] = cur[k] - f * rowq;
        }
      }
    }
    __syncthreads();
    // phase 2
    if (t < 32) {
      if (t == c) S[b + c][b + c] = d * inv_sd;
      else if (t > c) S[b + t][b + c] *= inv_sd;
    } else if (t < 64) {
      const int j = t - 32;
      if (j <= c) Y[b + c][b + j] *= inv_sd;
    }
  }
  __syncthreads();
}

__device__ inline void potf2_inv_block(const double* __restrict__ A, int64_t lda, int kb,
                                const double* __restrict__ diag0, double* __restrict__ L,
                                int64_t ldl, double* __restrict__ Linv, int32_t* st) {
  __shared__ double S[kNb][kLd];
  __shared__ double Y[kNb][kLd];
  __shared__ double T[32][33];
  __shared__ double D0[kNb];
  const int t = threadIdx.x;
  for (int e = t; e < kNb * kNb; e += 256) {
    const int r = e >> 6, q = e & 63;
    S[r][q] = (r < kb && q < kb) ? A[(int64_t)r * lda + q] : (r == q ? 1.0 : 0.0);
    Y[r][q] = r == q ? 1.0 : 0.0;
  }
  if (t < kNb) D0[t] = t < kb ? diag0[t] : 1.0;
  __syncthreads();
  bool bad_any = false;
  factor_inv32(S, Y, D0, 0, bad_any);
  // each thread owns 4 entries (i, j) of a 32 x 32 block: i = t >> 3 (0..31), j = (t & 7) + 8 u
  const int i = t >> 3, j0 = t & 7;
  double v[4];
  // The triangular operands hold exact zeros in their unused halves, so every product below
  // is a fixed 32-term sum (fully unrolled: the LDS reads issue together).
  // L21 = A21 L11^{-T}:  L21[i][j] = sum_k A21[i][k] Y11[j][k]
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = 0.0;
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const double a = S[32 + i][k];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = fma(a, Y[j0 + 8 * u][k], v[u]);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) S[32 + i][j0 + 8 * u] = v[u];
  __syncthreads();
  // A22 -= L21 L21^T (lower part is what the next factorisation reads)
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = 0.0;
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const double a = S[32 + i][k];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = fma(a, S[32 + j0 + 8 * u][k], v[u]);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) S[32 + i][32 + j0 + 8 * u] -= v[u];
  __syncthreads();
  factor_inv32(S, Y, D0, 32, bad_any);
  // T = L21 Y11, then Y21 = -Y22 T
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = 0.0;
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const double a = S[32 + i][k];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = fma(a, Y[k][j0 + 8 * u], v[u]);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) T[i][j0 + 8 * u] = v[u];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = 0.0;
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const double a = Y[32 + i][32 + k];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = fma(a, T[k][j0 + 8 * u], v[u]);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) Y[32 + i][j0 + 8 * u] = -v[u];
  if (bad_any) raise_status(st, VL_ERR_SINGULAR);
  __syncthreads();
  for (int e = t; e < kNb * kNb; e += 256) {
    const int r = e >> 6, q = e & 63;
    if (r < kb && q < kb) L[(int64_t)r * ldl + q] = q <= r ? S[r][q] : 0.0;
    Linv[e] = q <= r ? Y[r][q] : 0.0;
  }
  __syncthreads();
}

// ------------------------------------------------------------------------------------------
// C = beta C + alpha op(A) op(B); FP64; 64 x 64 tiles, 256 threads x (4 x 4), K step 16.
// op(A) is M x K: transA ? A[k * lda + i] : A[i * lda + k]; op(B) is K x N likewise.
// lower_only: tiles strictly above the diagonal are skipped (and in diagonal tiles only
// entries with j <= i are written).
// ------------------------------------------------------------------------------------------
__device__ inline void gemm_f64_tile(int64_t M, int64_t N, int64_t K, double alpha,
                              const double* __restrict__ A, int64_t lda, int transA,
                              const double* __restrict__ Bm, int64_t ldb, int transB, double beta,
                              double* __restrict__ C, int64_t ldc, int lower_only, int64_t i0,
                              int64_t j0) {
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
  double acc[4][4] = {};
  double ra[4], rb[4];
  load(0, ra, rb);
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      As[ak[u]][ai[u]] = ra[u];
      Bs[bk[u]][bj[u]] = rb[u];
    }
    __syncthreads();
    if (k0 + 16 < K) load(k0 + 16, ra, rb);      // in flight during the products below
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
