// FP64 dense linear algebra (declarations).
#pragma once
#include "common.hpp"

namespace vl {

// C = beta C + alpha op(A) op(B)   (row-major; lower_only writes only j <= i).  tri = 1 / 2
// declares op(A) lower / upper triangular (its zero half is skipped, not read).
int gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
             bool transA, const double* B, int64_t ldb, bool transB, double beta, double* C,
             int64_t ldc, bool lower_only, hipStream_t stream, int tri = 0);

// Scratch doubles of chol_solve_lower(): the original diagonal (n), and per 64-row block the
// inverse of the diagonal factor block and of the updated diagonal block (2 x 64 x 64 each).
size_t chol_ws_doubles(int64_t n);

// Cholesky A = L L^T of the SPD matrix A (n x n; lower triangle read; A destroyed by the
// trailing updates) fused with the forward substitution: on return R (n x nrhs, in place;
// nrhs may be 0) holds L^{-1} R and, when Linv is not null, Linv (n x n) holds L^{-1} (strict
// upper triangle zero).  L itself is not formed.  Raises VL_ERR_SINGULAR (status word) when a
// pivot is not above 1e-11 times its original diagonal entry or is not finite (and continues
// with pivot 1 so no NaN spreads).  ws: chol_ws_doubles(n) doubles.
int chol_solve_lower(double* A, int64_t n, int64_t lda, double* R, int64_t nrhs, int64_t ldr,
                     double* Linv, int64_t ldli, double* ws, int32_t* st, hipStream_t stream);

}  // namespace vl
