// FP64 dense linear algebra for the VAR normal equations and the B0 estimator: a blocked
// right-looking Cholesky fused with the forward substitution (one launch per 64-wide panel),
// and a tiled FP64 GEMM.  Matrices are row-major with explicit leading dimensions.
#include "linalg.hpp"
#include "chol_dev.hpp"

#include <math.h>

namespace vl {

__global__ __launch_bounds__(256) void gemm_f64_kernel(int64_t M, int64_t N, int64_t K,
                                                       double alpha, const double* __restrict__ A,
                                                       int64_t lda, int transA,
                                                       const double* __restrict__ Bm,
                                                       int64_t ldb, int transB, double beta,
                                                       double* __restrict__ C, int64_t ldc,
                                                       int lower_only, int tri) {
  gemm_f64_block(M, N, K, alpha, A, lda, transA, Bm, ldb, transB, beta, C, ldc, lower_only, tri,
                 (int64_t)blockIdx.y * 32, (int64_t)blockIdx.x * 32);
}

int gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
             bool transA, const double* B, int64_t ldb, bool transB, double beta, double* C,
             int64_t ldc, bool lower_only, hipStream_t stream, int tri) {
  if (M <= 0 || N <= 0) return VL_OK;
  dim3 grid((unsigned)ceil_div(N, (int64_t)32), (unsigned)ceil_div(M, (int64_t)32));
  gemm_f64_kernel<<<grid, 256, 0, stream>>>(M, N, K, alpha, A, lda, transA ? 1 : 0, B, ldb,
                                            transB ? 1 : 0, beta, C, ldc, lower_only ? 1 : 0,
                                            tri);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

__global__ __launch_bounds__(256) void chol_prologue_kernel(CholArgs a) {
  if (blockIdx.x > 0) {
    chol_linv_init(a, (int64_t)(blockIdx.x - 1) * 256 + threadIdx.x);
    return;
  }
  chol_prologue_block(a);
}

__global__ __launch_bounds__(256) void chol_step_kernel(CholArgs a, int64_t k) {
  chol_step_item(a, k, blockIdx.x);
}

size_t chol_ws_doubles(int64_t n) { return (size_t)chol_ws_doubles_dev(n); }

int chol_solve_lower(double* A, int64_t n, int64_t lda, double* R, int64_t nrhs, int64_t ldr,
                     double* Linv, int64_t ldli, double* ws, int32_t* st, hipStream_t stream) {
  if (n <= 0) return VL_OK;
  const int64_t nb = ceil_div(n, (int64_t)kNb);
  CholArgs a;
  a.A = A;
  a.n = n;
  a.lda = lda;
  a.R = nrhs > 0 ? R : nullptr;
  a.nrhs = nrhs;
  a.ldr = ldr;
  a.Li = Linv;
  a.ldli = ldli;
  a.diag0 = ws;
  a.Yb = ws + n;
  a.st = st;
  const int64_t cr = a.R ? ceil_div(nrhs, (int64_t)kNb) : 0;
  const unsigned init = Linv ? (unsigned)ceil_div(n * n, (int64_t)256) : 0u;
  chol_prologue_kernel<<<1 + init, 256, 0, stream>>>(a);
  VL_LAUNCH_CHECK();
  for (int64_t k = 0; k < nb; ++k) {
    const int64_t items = step_items(nb, k, cr, Linv != nullptr).total();
    if (items == 0) continue;
    chol_step_kernel<<<(unsigned)items, 256, 0, stream>>>(a, k);
    VL_LAUNCH_CHECK();
  }
  return VL_OK;
}

}  // namespace vl
