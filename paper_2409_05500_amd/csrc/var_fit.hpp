// VAR(p) least-squares fit (declarations).
#pragma once
#include "common.hpp"

namespace vl {

struct VarPlan {
  int64_t n = 0, m = 0, n_eff = 0, dz = 0;
  int p = 0;
  bool sliced = false;        // int8-slice products (VL_PREC_SLICED): slice buffers in the ws
};

struct VarWs {
  int64_t* colmap = nullptr;  // m (p+1) sample offsets of the lag-embedded columns
  double* mu = nullptr;       // m (p+1) column means (Y first, then Z)
  double* G = nullptr;        // dz x dz Gram (destroyed by the factorisation)
  double* Coef = nullptr;     // dz x m solution
  double* Rres = nullptr;     // dz x m refinement right-hand side
  float* CoefF = nullptr;     // dz x m float copy for the residual GEMM
  double* L = nullptr;        // dz x dz inverse of the Cholesky factor of G
  double* Tmp = nullptr;      // dz x m intermediate of the two triangular solves
  double* chol = nullptr;     // factorisation scratch kept for the solves
  double* E64 = nullptr;      // n_eff x m FP64 residual of the refinement step
  double* F = nullptr;        // m x m (p+1) lag products F_h (see var_normal_equations)
  double* mu0 = nullptr;      // m (p+1): the lag-0 means repeated for every lag block
  double* scratch = nullptr;  // split-K partials
  // VL_PREC_SLICED only: slice planes of the lag-embedded columns (the lag products), then of
  // the design rows and the coefficient columns (the residual), sharing one region
  int8_t* slices = nullptr;
  int8_t* slicesC = nullptr;  // coefficient columns (m rows of dz)
  int32_t* ex = nullptr;      // m (p+1): exponent per lag-embedded column
  int32_t* ez = nullptr;      // m (p+1): exponent per lag-embedded column about its own mean
  int32_t* ec = nullptr;      // m: exponent per coefficient column
};

// Lag-order selection workspace: the VAR workspace of the p_max plan, then m x m buffers.
struct LagWs {
  VarWs var;
  double* Syy = nullptr;    // T Sigma_p, updated in place from p = 0
  double* A = nullptr;      // copy factored for the log-determinant
  double* Li = nullptr;     // its L^{-1}
  double* chol = nullptr;   // factorisation scratch (m)
};

VarPlan plan_var(int64_t n, int64_t m, int p, bool sliced = false);
size_t var_ws_bytes(const VarPlan& v, void* base, VarWs* out);
int run_var(const VarPlan& v, const VarWs& w, const float* X, int64_t ldx, int prec, double* M,
            double* intercept, float* E, int64_t lde, int32_t* st, hipStream_t stream);

// C = centred cross-products (not divided by the sample count) of the m (p + 1) lag-embedded
// columns x(t), x(t-1), .., x(t-p) over t = p .. n-1, FP64 from the FP32 data, both triangles;
// column tau m + i is x_i(t - tau).  colmap, mu: m (p + 1) each; scratch:
// lag_cov_scratch_doubles() doubles.
size_t lag_cov_scratch_doubles(int64_t n, int64_t m, int p);
int lag_covariance(int64_t n, int64_t m, int p, const float* X, int64_t ldx, int64_t* colmap,
                   double* mu, double* C, double* scratch, int32_t* st, hipStream_t stream);

// v = plan_var(n, m, p_max).  logdet / aic / bic: p_max doubles each; best: {p_AIC, p_BIC}.
size_t lag_ws_bytes(const VarPlan& v, void* base, LagWs* out);
int run_lag_select(const VarPlan& v, const LagWs& w, const float* X, int64_t ldx, double* logdet,
                   double* aic, double* bic, int32_t* best, int32_t* st, hipStream_t stream);

}  // namespace vl
