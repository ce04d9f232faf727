// FP64 dense linear algebra (declarations).
#pragma once
#include "common.hpp"

namespace vl {

// C = beta C + alpha op(A) op(B)   (row-major; lower_only writes only j <= i)
int gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
             bool transA, const double* B, int64_t ldb, bool transB, double beta, double* C,
             int64_t ldc, bool lower_only, hipStream_t stream);

// In-place lower Cholesky A = L L^T (upper triangle of each diagonal block set to 0).  Raises
// VL_ERR_SINGULAR when a pivot is not above 1e-11 times its original diagonal entry or is not
// finite (and continues with pivot 1 so no NaN spreads).  diag0: n doubles of scratch.
int potrf_lower(double* A, int64_t n, int64_t lda, double* diag0, int32_t* st,
                hipStream_t stream);

// In place: B <- L^{-1} B (trans = false) or L^{-T} B (trans = true); B is n x nrhs.
int trsm_lower(const double* L, int64_t n, int64_t ldl, bool trans, double* B, int64_t nrhs,
               int64_t ldb, hipStream_t stream);

}  // namespace vl
