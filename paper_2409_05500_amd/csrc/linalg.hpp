// FP64 dense linear algebra (declarations).
#pragma once
#include "common.hpp"

namespace vl {

// C = beta C + alpha op(A) op(B)   (row-major; lower_only writes only j <= i)
int gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
             bool transA, const double* B, int64_t ldb, bool transB, double beta, double* C,
             int64_t ldc, bool lower_only, hipStream_t stream);

// Scratch doubles the factorisation keeps for the solves: the original diagonal (n) and the
// inverted 64 x 64 diagonal blocks of the factor.
size_t chol_ws_doubles(int64_t n);

// Lower Cholesky A = L L^T into L (lower triangle and the diagonal blocks' upper part written;
// the rest of L is not touched).  A is destroyed (trailing updates).  Raises VL_ERR_SINGULAR
// when a pivot is not above 1e-11 times its original diagonal entry or is not finite (and
// continues with pivot 1 so no NaN spreads).  ws: chol_ws_doubles(n) doubles, kept for
// trsm_lower().
int potrf_lower(double* A, int64_t n, int64_t lda, double* L, int64_t ldl, double* ws,
                int32_t* st, hipStream_t stream);

// X = L^{-1} B (trans = false) or X = L^{-T} B (trans = true), B n x nrhs destroyed, X
// separate from B.  ws: the scratch potrf_lower() filled for this L.
int trsm_lower(const double* L, int64_t n, int64_t ldl, const double* ws, bool trans, double* B,
               int64_t nrhs, int64_t ldb, double* X, int64_t ldx, hipStream_t stream);

}  // namespace vl
