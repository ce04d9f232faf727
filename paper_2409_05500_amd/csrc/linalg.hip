// FP64 dense linear algebra for the VAR normal equations and the B0 estimator:
// blocked right-looking Cholesky, blocked triangular solves with many right-hand sides, and
// a tiled FP64 GEMM.  Matrices are row-major with explicit leading dimensions.
#include "linalg.hpp"

#include <math.h>

namespace vl {

constexpr int kNb = 64;  // panel width

// ------------------------------------------------------------------------------------------
// Unblocked Cholesky of the kb x kb diagonal block at A (kb <= 64), in LDS.
// ------------------------------------------------------------------------------------------
// A pivot d is rejected (VL_ERR_SINGULAR) unless d > kPivotRel * diag0 (the diagonal entry before
// any elimination), i.e. unless the leading block is better conditioned than ~1e11.
constexpr double kPivotRel = 1e-11;

__global__ __launch_bounds__(256) void potf2_kernel(double* __restrict__ A, int64_t lda, int kb,
                                                    const double* __restrict__ diag0, int32_t* st) {
  __shared__ double L[kNb][kNb + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < kb * kb; e += 256) L[e / kb][e % kb] = A[(e / kb) * lda + (e % kb)];
  __syncthreads();
  for (int c = 0; c < kb; ++c) {
    if (tid == 0) {
      double d = L[c][c];
      if (!(d > kPivotRel * diag0[c]) || !isfinite(d)) {
        raise_status(st, VL_ERR_SINGULAR);
        d = 1.0;
      }
      L[c][c] = sqrt(d);
    }
    __syncthreads();
    const double inv = 1.0 / L[c][c];
    for (int r = c + 1 + tid; r < kb; r += 256) L[r][c] *= inv;
    __syncthreads();
    const int rem = kb - c - 1;
    for (int e = tid; e < rem * rem; e += 256) {
      const int r = c + 1 + e / rem, q = c + 1 + e % rem;
      if (q <= r) L[r][q] -= L[r][c] * L[q][c];
    }
    __syncthreads();
  }
  for (int e = tid; e < kb * kb; e += 256) {
    const int r = e / kb, q = e % kb;
    A[r * lda + q] = q <= r ? L[r][q] : 0.0;
  }
}

// ------------------------------------------------------------------------------------------
// Triangular solve against a kb x kb lower-triangular block L (kb <= 64) for many vectors:
// vector j has element r at B[r * rs + j * cs].  trans == 0: L x = b;  trans == 1: L^T x = b.
// One thread per vector, the vector in registers, L in LDS.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void trsv_block_kernel(const double* __restrict__ Lg,
                                                        int64_t ldl, int kb,
                                                        double* __restrict__ B, int64_t rs,
                                                        int64_t cs, int64_t nvec, int trans) {
  __shared__ double L[kNb][kNb + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < kb * kb; e += 64) L[e / kb][e % kb] = Lg[(e / kb) * ldl + (e % kb)];
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * 64 + tid;
  if (j >= nvec) return;
  double x[kNb];
#pragma unroll
  for (int r = 0; r < kNb; ++r) x[r] = r < kb ? B[r * rs + j * cs] : 0.0;
  if (!trans) {
#pragma unroll
    for (int r = 0; r < kNb; ++r) {
      if (r < kb) {
        double s = x[r];
#pragma unroll
        for (int q = 0; q < r; ++q) s -= L[r][q] * x[q];
        x[r] = s / L[r][r];
      }
    }
  } else {
#pragma unroll
    for (int r = kNb - 1; r >= 0; --r) {
      if (r < kb) {
        double s = x[r];
#pragma unroll
        for (int q = r + 1; q < kNb; ++q)
          if (q < kb) s -= L[q][r] * x[q];
        x[r] = s / L[r][r];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kNb; ++r)
    if (r < kb) B[r * rs + j * cs] = x[r];
}

// ------------------------------------------------------------------------------------------
// C = beta C + alpha op(A) op(B); FP64; 64 x 64 tiles, 256 threads x (4 x 4), K step 16.
// op(A) is M x K: transA ? A[k * lda + i] : A[i * lda + k]; op(B) is K x N likewise.
// lower_only: tiles strictly above the diagonal are skipped (and in diagonal tiles only
// entries with j <= i are written).
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gemm_f64_kernel(int64_t M, int64_t N, int64_t K,
                                                       double alpha, const double* __restrict__ A,
                                                       int64_t lda, int transA,
                                                       const double* __restrict__ Bm,
                                                       int64_t ldb, int transB, double beta,
                                                       double* __restrict__ C, int64_t ldc,
                                                       int lower_only) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  if (lower_only && j0 > i0 + 63) return;
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  double acc[4][4] = {};
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int kk = e / 64, ii = e % 64;
      const int64_t gi = i0 + ii, gk = k0 + kk;
      double va = 0.0;
      if (gi < M && gk < K) va = transA ? A[gk * lda + gi] : A[gi * lda + gk];
      As[kk][ii] = va;
      const int64_t gj = j0 + ii;
      double vb = 0.0;
      if (gj < N && gk < K) vb = transB ? Bm[gj * ldb + gk] : Bm[gk * ldb + gj];
      Bs[kk][ii] = vb;
    }
    __syncthreads();
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

int gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
             bool transA, const double* B, int64_t ldb, bool transB, double beta, double* C,
             int64_t ldc, bool lower_only, hipStream_t stream) {
  if (M <= 0 || N <= 0) return VL_OK;
  dim3 grid((unsigned)ceil_div(N, 64), (unsigned)ceil_div(M, 64));
  gemm_f64_kernel<<<grid, 256, 0, stream>>>(M, N, K, alpha, A, lda, transA ? 1 : 0, B, ldb,
                                            transB ? 1 : 0, beta, C, ldc, lower_only ? 1 : 0);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

__global__ void diag_copy_kernel(const double* __restrict__ A, int64_t n, int64_t lda,
                                 double* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = A[i * lda + i];
}

int potrf_lower(double* A, int64_t n, int64_t lda, double* diag0, int32_t* st,
                hipStream_t stream) {
  diag_copy_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, stream>>>(A, n, lda, diag0);
  VL_LAUNCH_CHECK();
  for (int64_t k0 = 0; k0 < n; k0 += kNb) {
    const int kb = (int)(n - k0 < kNb ? n - k0 : kNb);
    double* A11 = A + k0 * lda + k0;
    potf2_kernel<<<1, 256, 0, stream>>>(A11, lda, kb, diag0 + k0, st);
    VL_LAUNCH_CHECK();
    const int64_t rest = n - k0 - kb;
    if (rest <= 0) break;
    double* A21 = A + (k0 + kb) * lda + k0;
    // rows of A21 are the right-hand sides of L11 x = a (x^T = row of L21)
    trsv_block_kernel<<<(unsigned)ceil_div(rest, 64), 64, 0, stream>>>(A11, lda, kb, A21, 1, lda,
                                                                        rest, 0);
    VL_LAUNCH_CHECK();
    double* A22 = A + (k0 + kb) * lda + (k0 + kb);
    int rc = gemm_f64(rest, rest, kb, -1.0, A21, lda, false, A21, lda, true, 1.0, A22, lda, true,
                      stream);
    if (rc) return rc;
  }
  return VL_OK;
}

int trsm_lower(const double* L, int64_t n, int64_t ldl, bool trans, double* B, int64_t nrhs,
               int64_t ldb, hipStream_t stream) {
  const unsigned vb = (unsigned)ceil_div(nrhs, 64);
  if (!trans) {
    for (int64_t k0 = 0; k0 < n; k0 += kNb) {
      const int kb = (int)(n - k0 < kNb ? n - k0 : kNb);
      trsv_block_kernel<<<vb, 64, 0, stream>>>(L + k0 * ldl + k0, ldl, kb, B + k0 * ldb, ldb, 1,
                                               nrhs, 0);
      VL_LAUNCH_CHECK();
      const int64_t rest = n - k0 - kb;
      if (rest > 0) {
        int rc = gemm_f64(rest, nrhs, kb, -1.0, L + (k0 + kb) * ldl + k0, ldl, false,
                          B + k0 * ldb, ldb, false, 1.0, B + (k0 + kb) * ldb, ldb, false, stream);
        if (rc) return rc;
      }
    }
  } else {
    const int64_t last = ((n - 1) / kNb) * kNb;
    for (int64_t k0 = last; k0 >= 0; k0 -= kNb) {
      const int kb = (int)(n - k0 < kNb ? n - k0 : kNb);
      trsv_block_kernel<<<vb, 64, 0, stream>>>(L + k0 * ldl + k0, ldl, kb, B + k0 * ldb, ldb, 1,
                                               nrhs, 1);
      VL_LAUNCH_CHECK();
      if (k0 > 0) {
        // B[0:k0] -= L[k0:k0+kb, 0:k0]^T X[k0:k0+kb]
        int rc = gemm_f64(k0, nrhs, kb, -1.0, L + k0 * ldl, ldl, true, B + k0 * ldb, ldb, false,
                          1.0, B, ldb, false, stream);
        if (rc) return rc;
      }
    }
  }
  return VL_OK;
}

}  // namespace vl
