// B0 and lag matrices from the causal order (Sec. 4: estimation of the instantaneous matrix
// B0; Sec. 2.1: VarLiNGAM lag matrices).
//
// Regressing each variable on its predecessors in the order K by least squares is the LDL^T
// factorisation of the order-permuted covariance:  Sigma_KK = L D L^T with L unit lower-
// triangular, and the regression coefficients are B0_KK = I - L^{-1} (row k holds the
// coefficients of variable K_k on K_0 .. K_{k-1}).  With the Cholesky factor Lc = L D^{1/2},
// L^{-1} = diag(Lc) Lc^{-1}, and diag(Lc) = 1 / diag(Lc^{-1}): only Lc^{-1} is formed (by the
// fused factorisation).  Then B_tau = (I - B0) M_tau.
#include "estimate_b.hpp"
#include "chol_dev.hpp"
#include "linalg.hpp"
#include "profile.hpp"

namespace vl {

// P[a][b] = Cov[K_a][K_b].  The permutation check rides along: an index out of range, or two
// positions a != b holding the same index (m values in [0, m) without a repeat are a
// permutation), raises VL_ERR_INVALID_ARG before the factorisation can raise anything.
__global__ void permute_cov_kernel(const double* __restrict__ Cov, const int32_t* __restrict__ K,
                                   int64_t m, double* __restrict__ P, int32_t* st) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  const int64_t a = e / m, b = e % m;
  const int32_t ka = K[a], kb = K[b];
  if (ka < 0 || ka >= m || kb < 0 || kb >= m || (a != b && ka == kb)) {
    raise_status(st, VL_ERR_INVALID_ARG);
    P[e] = a == b ? 1.0 : 0.0;
    return;
  }
  P[e] = Cov[(int64_t)ka * m + kb];
}

// B0[K_a][K_b] = -Linv[a][b] / Linv[a][a] for b < a (Lc[a][a] = 1 / Linv[a][a]); 0 otherwise
// (zero diagonal).
__global__ void assemble_b0_kernel(const double* __restrict__ Linv, const int32_t* __restrict__ K,
                                   int64_t m, double* __restrict__ B0) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  const int64_t a = e / m, b = e % m;
  int32_t ka = K[a], kb = K[b];
  if (ka < 0 || ka >= m || kb < 0 || kb >= m) return;
  B0[(int64_t)ka * m + kb] = b < a ? -Linv[a * m + b] / Linv[a * m + a] : 0.0;
}

// B_tau = M_tau - B0 M_tau for every lag in one launch (blockIdx.z = tau - 1): the FP64 MFMA
// GEMM block with its beta term read from M_tau, so no copy of M_tau into B_tau first.
__global__ __launch_bounds__(256) void blag_kernel(const double* __restrict__ B0,
                                                   const double* __restrict__ M, int64_t m,
                                                   double* __restrict__ Blag) {
  const int64_t off = (int64_t)blockIdx.z * m * m;
  gemm_f64_block(m, m, m, -1.0, B0, m, 0, M + off, m, 0, 1.0, Blag + off, m, 0, 0,
                 (int64_t)blockIdx.y * 32, (int64_t)blockIdx.x * 32, M + off);
}

size_t b_ws_bytes(int64_t m, void* base, BWs* out) {
  Carver c(base);
  BWs w;
  w.P = c.take<double>(m * m);
  w.Linv = c.take<double>(m * m);
  w.chol = c.take<double>(chol_ws_doubles(m));
  if (out) *out = w;
  return c.used;
}

int run_estimate_b(const BWs& w, const double* Cov, const double* M, const int32_t* K, int64_t m,
                   int p, double* B0, double* Blag, int32_t* st, hipStream_t stream) {
  ProfileScope ps("estimate_b", stream);
  const unsigned g = (unsigned)ceil_div(m * m, 256);
  permute_cov_kernel<<<g, 256, 0, stream>>>(Cov, K, m, w.P, st);
  VL_LAUNCH_CHECK();
  int rc = chol_solve_lower(w.P, m, m, nullptr, 0, 0, w.Linv, m, w.chol, st, stream);
  if (rc) return rc;
  assemble_b0_kernel<<<g, 256, 0, stream>>>(w.Linv, K, m, B0);
  VL_LAUNCH_CHECK();
  if (p > 0) {
    dim3 grid((unsigned)ceil_div(m, (int64_t)32), (unsigned)ceil_div(m, (int64_t)32), (unsigned)p);
    blag_kernel<<<grid, 256, 0, stream>>>(B0, M, m, Blag);
    VL_LAUNCH_CHECK();
  }
  return VL_OK;
}

}  // namespace vl
