// FP64 dense linear algebra for the VAR normal equations and the B0 estimator:
// blocked right-looking Cholesky whose 64 x 64 diagonal blocks are factored and inverted by one
// wave each, triangular solves with many right-hand sides as GEMMs against those inverted
// blocks, and a tiled FP64 GEMM.  Matrices are row-major with explicit leading dimensions.
#include "linalg.hpp"
#include "linalg_dev.hpp"

#include <math.h>

namespace vl {

__global__ __launch_bounds__(256) void potf2_inv_kernel(const double* __restrict__ A, int64_t lda,
                                                        int kb, const double* __restrict__ diag0,
                                                        double* __restrict__ L, int64_t ldl,
                                                        double* __restrict__ Linv, int32_t* st) {
  potf2_inv_block(A, lda, kb, diag0, L, ldl, Linv, st);
}

__global__ __launch_bounds__(256) void gemm_f64_kernel(int64_t M, int64_t N, int64_t K,
                                                       double alpha, const double* __restrict__ A,
                                                       int64_t lda, int transA,
                                                       const double* __restrict__ Bm,
                                                       int64_t ldb, int transB, double beta,
                                                       double* __restrict__ C, int64_t ldc,
                                                       int lower_only) {
  gemm_f64_tile(M, N, K, alpha, A, lda, transA, Bm, ldb, transB, beta, C, ldc, lower_only,
                (int64_t)blockIdx.y * 64, (int64_t)blockIdx.x * 64);
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

size_t chol_ws_doubles(int64_t n) { return (size_t)n + (size_t)ceil_div(n, kNb) * kNb * kNb; }

int potrf_lower(double* A, int64_t n, int64_t lda, double* L, int64_t ldl, double* ws,
                int32_t* st, hipStream_t stream) {
  double* diag0 = ws;
  double* inv = ws + n;
  diag_copy_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, stream>>>(A, n, lda, diag0);
  VL_LAUNCH_CHECK();
  for (int64_t k0 = 0; k0 < n; k0 += kNb) {
    const int kb = (int)(n - k0 < kNb ? n - k0 : kNb);
    double* invk = inv + (k0 / kNb) * kNb * kNb;
    potf2_inv_kernel<<<1, 256, 0, stream>>>(A + k0 * lda + k0, lda, kb, diag0 + k0,
                                            L + k0 * ldl + k0, ldl, invk, st);
    VL_LAUNCH_CHECK();
    const int64_t rest = n - k0 - kb;
    if (rest <= 0) break;
    // L21 = A21 L11^{-T}
    int rc = gemm_f64(rest, kb, kb, 1.0, A + (k0 + kb) * lda + k0, lda, false, invk, kNb, true,
                      0.0, L + (k0 + kb) * ldl + k0, ldl, false, stream);
    if (rc) return rc;
    // A22 -= L21 L21^T (lower triangle)
    rc = gemm_f64(rest, rest, kb, -1.0, L + (k0 + kb) * ldl + k0, ldl, false,
                  L + (k0 + kb) * ldl + k0, ldl, true, 1.0, A + (k0 + kb) * lda + (k0 + kb), lda,
                  true, stream);
    if (rc) return rc;
  }
  return VL_OK;
}

int trsm_lower(const double* L, int64_t n, int64_t ldl, const double* ws, bool trans, double* B,
               int64_t nrhs, int64_t ldb, double* X, int64_t ldx, hipStream_t stream) {
  const double* inv = ws + n;
  const int64_t nblk = ceil_div(n, kNb);
  if (!trans) {
    for (int64_t b = 0; b < nblk; ++b) {
      const int64_t k0 = b * kNb;
      const int kb = (int)(n - k0 < kNb ? n - k0 : kNb);
      // X_k = L_kk^{-1} B_k
      int rc = gemm_f64(kb, nrhs, kb, 1.0, inv + b * kNb * kNb, kNb, false, B + k0 * ldb, ldb,
                        false, 0.0, X + k0 * ldx, ldx, false, stream);
      if (rc) return rc;
      const int64_t rest = n - k0 - kb;
      if (rest > 0) {
        // B_rest -= L_rest,k X_k
        rc = gemm_f64(rest, nrhs, kb, -1.0, L + (k0 + kb) * ldl + k0, ldl, false, X + k0 * ldx,
                      ldx, false, 1.0, B + (k0 + kb) * ldb, ldb, false, stream);
        if (rc) return rc;
      }
    }
  } else {
    for (int64_t b = nblk - 1; b >= 0; --b) {
      const int64_t k0 = b * kNb;
      const int kb = (int)(n - k0 < kNb ? n - k0 : kNb);
      // X_k = L_kk^{-T} B_k
      int rc = gemm_f64(kb, nrhs, kb, 1.0, inv + b * kNb * kNb, kNb, true, B + k0 * ldb, ldb,
                        false, 0.0, X + k0 * ldx, ldx, false, stream);
      if (rc) return rc;
      if (k0 > 0) {
        // B_0:k -= L_k,0:k^T X_k
        rc = gemm_f64(k0, nrhs, kb, -1.0, L + k0 * ldl, ldl, true, X + k0 * ldx, ldx, false, 1.0,
                      B, ldb, false, stream);
        if (rc) return rc;
      }
    }
  }
  return VL_OK;
}

}  // namespace vl
