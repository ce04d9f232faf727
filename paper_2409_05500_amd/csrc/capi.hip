// extern "C" entry points: argument validation, workspace carving, status handling.
#include <map>
#include <mutex>

#include "backward.hpp"
#include "certify.hpp"
#include "ensemble.hpp"
#include "estimate_b.hpp"
#include "iterative.hpp"
#include "order.hpp"
#include "pairwise.hpp"
#include "prune.hpp"
#include "var_fit.hpp"

using namespace vl;

namespace {

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline bool valid_prec(int prec) {
  return prec == VL_PREC_FP32 || prec == VL_PREC_MIXED || prec == VL_PREC_BF16 ||
         prec == VL_PREC_FP32_REFINED || prec == VL_PREC_SLICED;
}

// The precompute's entry points also take the compensated-sum flag.
inline bool valid_pairwise_prec(int prec) { return valid_prec(prec & ~VL_PAIRWISE_COMPENSATED); }
inline bool compensated(int prec) { return (prec & VL_PAIRWISE_COMPENSATED) != 0; }
inline bool sliced(int prec) { return (prec & ~VL_PAIRWISE_COMPENSATED) == VL_PREC_SLICED;
}

inline bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

int begin(int32_t* dev_status, hipStream_t stream) {
  reset_status_kernel<<<1, 64, 0, stream>>>(dev_status);
  return hipGetLastError() == hipSuccess ? VL_OK : VL_ERR_HIP;
}

// Library-owned scratch of pairwise_stats_noalloc: one copy per GPU, held until the process
// ends.  Host code never passes `scratch` itself (on the host it only names the symbol): the
// device address comes from hipGetSymbolAddress, taken once per device with that device
// current, and is kept in g_scratch.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch;

int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return VL_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return VL_ERR_HIP;
    it = g_scratch.emplace(dev, p).first;
  }
  *out = it->second;
  return VL_OK;
}

}  // namespace

extern "C" {

const char* varlingam_status_string(int status) {
  switch (status) {
    case VL_OK: return "ok";
    case VL_ERR_INVALID_ARG: return "invalid argument";
    case VL_ERR_SHAPE: return "unsupported shape";
    case VL_ERR_DEGENERATE: return "degenerate data (zero variance or |rho| = 1)";
    case VL_ERR_SINGULAR: return "matrix not positive definite";
    case VL_ERR_NONFINITE: return "non-finite input";
    case VL_ERR_WORKSPACE: return "workspace too small";
    case VL_ERR_HIP: return "HIP launch failure";
    default: return "unknown status";
  }
}

// ----------------------------------------------------------------------------------------
size_t varlingam_fit_var_workspace_bytes(int64_t n, int64_t m, int p, int prec) {
  if (m < 1 || p < 1 || n - p <= m * p + 1) return 0;
  return var_ws_bytes(plan_var(n, m, p, prec == VL_PREC_SLICED), nullptr, nullptr);
}

int varlingam_fit_var(const float* X, int64_t n, int64_t m, int64_t ldx, int p, int prec,
                      double* M, double* intercept, float* E, int64_t lde, void* ws,
                      size_t ws_bytes, int32_t* dev_status, void* stream) {
  if (!X || !M || !intercept || !E || !dev_status || !valid_prec(prec)) return VL_ERR_INVALID_ARG;
  if (m < 1 || p < 1 || n - p <= m * p + 1 || m * p > 4096) return VL_ERR_SHAPE;
  if (ldx < m || lde < m) return VL_ERR_INVALID_ARG;
  const VarPlan v = plan_var(n, m, p, prec == VL_PREC_SLICED);
  const size_t need = var_ws_bytes(v, nullptr, nullptr);
  if (!ws || ws_bytes < need || !aligned256(ws)) return VL_ERR_WORKSPACE;
  VarWs w;
  var_ws_bytes(v, ws, &w);
  hipStream_t s = as_stream(stream);
  int rc = begin(dev_status, s);
  if (rc) return rc;
  return run_var(v, w, X, ldx, prec, M, intercept, E, lde, dev_status, s);
}

// ----------------------------------------------------------------------------------------
size_t varlingam_select_lag_workspace_bytes(int64_t n, int64_t m, int p_max) {
  if (m < 1 || p_max < 1 || n - p_max <= m * p_max + 1 || m * p_max > 4096) return 0;
  return lag_ws_bytes(plan_var(n, m, p_max), nullptr, nullptr);
}

int varlingam_select_lag(const float* X, int64_t n, int64_t m, int64_t ldx, int p_max,
                         double* logdet, double* aic, double* bic, int32_t* best, void* ws,
                         size_t ws_bytes, int32_t* dev_status, void* stream) {
  if (!X || !logdet || !aic || !bic || !best || !dev_status) return VL_ERR_INVALID_ARG;
  if (m < 1 || p_max < 1 || n - p_max <= m * p_max + 1 || m * p_max > 4096) return VL_ERR_SHAPE;
  if (ldx < m) return VL_ERR_INVALID_ARG;
  const VarPlan v = plan_var(n, m, p_max);
  const size_t need = lag_ws_bytes(v, nullptr, nullptr);
  if (!ws || ws_bytes < need || !aligned256(ws)) return VL_ERR_WORKSPACE;
  LagWs w;
  lag_ws_bytes(v, ws, &w);
  hipStream_t s = as_stream(stream);
  int rc = begin(dev_status, s);
  if (rc) return rc;
  return run_lag_select(v, w, X, ldx, logdet, aic, bic, best, dev_status, s);
}

// ----------------------------------------------------------------------------------------
size_t pairwise_stats_workspace_bytes(int64_t n_eff, int64_t m, int prec) {
  if (m < 2 || n_eff < 2 || m > 65536 || !valid_pairwise_prec(prec)) return 0;
  return pairwise_ws_bytes(plan_pairwise(n_eff, m, compensated(prec), sliced(prec)), nullptr,
                           nullptr);
}

int pairwise_stats(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec, double* Hx,
                   double* Hr, double* S, double* Cov, void* ws, size_t ws_bytes,
                   int32_t* dev_status, void* stream) {
  if (!E || !Hx || !Hr || !S || !dev_status || !valid_pairwise_prec(prec))
    return VL_ERR_INVALID_ARG;
  if (m < 2 || n_eff < 2 || m > 65536) return VL_ERR_SHAPE;
  if (lde < m) return VL_ERR_INVALID_ARG;
  const PairwisePlan p = plan_pairwise(n_eff, m, compensated(prec), sliced(prec));
  const size_t need = pairwise_ws_bytes(p, nullptr, nullptr);
  if (!ws || ws_bytes < need || !aligned256(ws)) return VL_ERR_WORKSPACE;
  PairwiseWs w;
  pairwise_ws_bytes(p, ws, &w);
  hipStream_t s = as_stream(stream);
  int rc = begin(dev_status, s);
  if (rc) return rc;
  return run_pairwise(p, w, E, lde, prec, Hx, Hr, S, Cov, nullptr, dev_status, s);
}

size_t pairwise_stats_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

int pairwise_stats_noalloc(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec,
                           double* Hx, double* Hr, double* S, double* Cov, int32_t* dev_status,
                           void* stream) {
  if (!E || !Hx || !Hr || !S || !dev_status || !valid_pairwise_prec(prec))
    return VL_ERR_INVALID_ARG;
  if (m < 2 || n_eff < 2 || m > 65536) return VL_ERR_SHAPE;
  if (lde < m) return VL_ERR_INVALID_ARG;
  const PairwisePlan p = plan_pairwise(n_eff, m, compensated(prec), sliced(prec));
  if (pairwise_ws_bytes(p, nullptr, nullptr) > kNoAllocScratchBytes) return VL_ERR_WORKSPACE;
  void* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  PairwiseWs w;
  pairwise_ws_bytes(p, ws, &w);
  hipStream_t s = as_stream(stream);
  rc = begin(dev_status, s);
  if (rc) return rc;
  return run_pairwise(p, w, E, lde, prec, Hx, Hr, S, Cov, nullptr, dev_status, s);
}

// ----------------------------------------------------------------------------------------
size_t varlingam_order_iterative_workspace_bytes(int64_t n_eff, int64_t m, int prec) {
  (void)prec;
  if (m < 1 || m > 4096 || n_eff < 2) return 0;
  return iter_ws_bytes(n_eff, m, nullptr, nullptr);
}

int varlingam_order_iterative(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec,
                              int32_t* order, double* margin, void* ws, size_t ws_bytes,
                              int32_t* dev_status, void* stream) {
  if (!E || !order || !margin || !dev_status || !valid_prec(prec)) return VL_ERR_INVALID_ARG;
  if (m < 1 || m > 4096 || n_eff < 2) return VL_ERR_SHAPE;
  if (lde < m) return VL_ERR_INVALID_ARG;
  const size_t need = iter_ws_bytes(n_eff, m, nullptr, nullptr);
  if (!ws || ws_bytes < need || !aligned256(ws)) return VL_ERR_WORKSPACE;
  IterWs w;
  iter_ws_bytes(n_eff, m, ws, &w);
  hipStream_t s = as_stream(stream);
  int rc = begin(dev_status, s);
  if (rc) return rc;
  return run_order_iterative(E, n_eff, m, lde, prec, m, order, margin, w, dev_status, s);
}

size_t varlingam_order_hybrid_workspace_bytes(int64_t n_eff, int64_t m, int prec) {
  return varlingam_order_iterative_workspace_bytes(n_eff, m, prec);
}

int varlingam_order_hybrid(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec,
                           int64_t k_exact, int32_t* order, double* margin, void* ws,
                           size_t ws_bytes, int32_t* dev_status, void* stream) {
  if (!E || !order || !margin || !dev_status || !valid_prec(prec) || k_exact < 0)
    return VL_ERR_INVALID_ARG;
  if (m < 1 || m > 4096 || n_eff < 2) return VL_ERR_SHAPE;
  if (lde < m) return VL_ERR_INVALID_ARG;
  const size_t need = iter_ws_bytes(n_eff, m, nullptr, nullptr);
  if (!ws || ws_bytes < need || !aligned256(ws)) return VL_ERR_WORKSPACE;
  IterWs w;
  iter_ws_bytes(n_eff, m, ws, &w);
  hipStream_t s = as_stream(stream);
  int rc = begin(dev_status, s);
  if (rc) return rc;
  return run_order_iterative(E, n_eff, m, lde, prec, k_exact, order, margin, w, dev_status, s);
}

// ----------------------------------------------------------------------------------------
size_t pairwise_stats_backward_workspace_bytes(int64_t n_eff, int64_t m, int prec) {
  (void)prec;
  if (m < 2 || n_eff < 2 || m > 65536) return 0;
  return bwd_ws_bytes(plan_backward(n_eff, m), nullptr, nullptr);
}

size_t pairwise_stats_saved_doubles(int64_t m) {
  if (m < 2 || m > 65536) return 0;
  return (size_t)(3 * m * m + 3 * m);
}

int pairwise_stats_save(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec,
                        double* Hx, double* Hr, double* S, double* Cov, double* saved, void* ws,
                        size_t ws_bytes, int32_t* dev_status, void* stream) {
  if (!E || !Hx || !Hr || !S || !saved || !dev_status || !valid_prec(prec))
    return VL_ERR_INVALID_ARG;
  if (m < 2 || n_eff < 2 || m > 65536) return VL_ERR_SHAPE;
  if (lde < m) return VL_ERR_INVALID_ARG;
  const PairwisePlan p = plan_pairwise(n_eff, m);
  const size_t need = pairwise_ws_bytes(p, nullptr, nullptr);
  if (!ws || ws_bytes < need || !aligned256(ws)) return VL_ERR_WORKSPACE;
  PairwiseWs w;
  pairwise_ws_bytes(p, ws, &w);
  hipStream_t s = as_stream(stream);
  int rc = begin(dev_status, s);
  if (rc) return rc;
  double* cov = saved + 2 * m * m + 2 * m;
  rc = run_pairwise(p, w, E, lde, prec, Hx, Hr, S, cov, saved, dev_status, s);
  if (rc) return rc;
  const size_t d = sizeof(double);
  if (hipMemcpyAsync(saved + 2 * m * m, w.momx, 2 * m * d, hipMemcpyDeviceToDevice, s) ||
      hipMemcpyAsync(saved + 3 * m * m + 2 * m, w.mu, m * d, hipMemcpyDeviceToDevice, s) ||
      (Cov && hipMemcpyAsync(Cov, cov, m * m * d, hipMemcpyDeviceToDevice, s)))
    return VL_ERR_HIP;
  return VL_OK;
}

int pairwise_stats_backward(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec,
                            const double* saved, const double* G, float* dE, int64_t ldde,
                            void* ws, size_t ws_bytes, int32_t* dev_status, void* stream) {
  if (!E || !G || !dE || !dev_status || !valid_prec(prec)) return VL_ERR_INVALID_ARG;
  if (m < 2 || n_eff < 2 || m > 65536) return VL_ERR_SHAPE;
  if (lde < m || ldde < m) return VL_ERR_INVALID_ARG;
  const BwdPlan b = plan_backward(n_eff, m);
  if (!ws || ws_bytes < bwd_ws_bytes(b, nullptr, nullptr) || !aligned256(ws))
    return VL_ERR_WORKSPACE;
  BwdWs w;
  bwd_ws_bytes(b, ws, &w);
  hipStream_t s = as_stream(stream);
  int rc = begin(dev_status, s);
  if (rc) return rc;
  return run_backward(b, w, E, lde, prec, saved, G, dE, ldde, dev_status, s);
}

// ----------------------------------------------------------------------------------------
size_t approx_order_workspace_bytes(int64_t m) {
  if (m < 1 || m > kMaxOrderM) return 0;
  Carver c(nullptr);
  c.take<double>(m);
  return c.used;
}

int approx_order(const double* S, int64_t m, int32_t* order, double* margin, void* ws,
                 size_t ws_bytes, int32_t* dev_status, void* stream) {
  if (!S || !order || !margin || !dev_status) return VL_ERR_INVALID_ARG;
  if (m < 1 || m > kMaxOrderM) return VL_ERR_SHAPE;
  if (!ws || ws_bytes < approx_order_workspace_bytes(m) || !aligned256(ws)) return VL_ERR_WORKSPACE;
  hipStream_t s = as_stream(stream);
  int rc = begin(dev_status, s);
  if (rc) return rc;
  return run_order(S, m, order, margin, static_cast<double*>(ws), dev_status, s);
}

// ----------------------------------------------------------------------------------------
size_t approx_order_certified_workspace_bytes(int64_t n_eff, int64_t m) {
  if (m < 1 || m > 4096 || n_eff < 2) return 0;
  return cert_ws_bytes(n_eff, m, nullptr, nullptr);
}

int approx_order_certified(const float* E, int64_t n_eff, int64_t m, int64_t lde, double* S,
                           double eps_S, int32_t* order, double* margin, int32_t* refined,
                           int64_t* n_refined, void* ws, size_t ws_bytes, int32_t* dev_status,
                           void* stream) {
  if (!E || !S || !order || !margin || !dev_status || !(eps_S >= 0.0)) return VL_ERR_INVALID_ARG;
  if (m < 1 || m > 4096 || n_eff < 2) return VL_ERR_SHAPE;
  if (lde < m) return VL_ERR_INVALID_ARG;
  if (!ws || ws_bytes < cert_ws_bytes(n_eff, m, nullptr, nullptr) || !aligned256(ws))
    return VL_ERR_WORKSPACE;
  CertWs w;
  cert_ws_bytes(n_eff, m, ws, &w);
  hipStream_t s = as_stream(stream);
  int rc = begin(dev_status, s);
  if (rc) return rc;
  int64_t rounds = 0;
  return run_order_certified(E, n_eff, m, lde, S, eps_S, order, margin, refined, n_refined,
                             &rounds, w, dev_status, s);
}

// ----------------------------------------------------------------------------------------
size_t estimate_B_workspace_bytes(int64_t m, int p) {
  if (m < 1 || m > kMaxOrderM || p < 0) return 0;
  return b_ws_bytes(m, nullptr, nullptr);
}

int estimate_B(const double* Cov, const double* M, const int32_t* order, int64_t m, int p,
               double* B0, double* Blag, void* ws, size_t ws_bytes, int32_t* dev_status,
               void* stream) {
  if (!Cov || !order || !B0 || !dev_status) return VL_ERR_INVALID_ARG;
  if (m < 1 || m > kMaxOrderM || p < 0) return VL_ERR_SHAPE;
  if (p > 0 && (!M || !Blag)) return VL_ERR_INVALID_ARG;
  if (!ws || ws_bytes < b_ws_bytes(m, nullptr, nullptr) || !aligned256(ws)) return VL_ERR_WORKSPACE;
  BWs w;
  b_ws_bytes(m, ws, &w);
  hipStream_t s = as_stream(stream);
  int rc = begin(dev_status, s);
  if (rc) return rc;
  return run_estimate_b(w, Cov, M, order, m, p, B0, Blag, dev_status, s);
}

// ----------------------------------------------------------------------------------------
static bool prune_shape_ok(int64_t n, int64_t m, int p, int64_t max_steps) {
  return m >= 1 && p >= 1 && max_steps >= 0 && m * (p + 1) <= 4096 &&
         n - p > m * (p + 1) + 1;
}

size_t varlingam_prune_workspace_bytes(int64_t n, int64_t m, int p, int64_t max_steps) {
  if (!prune_shape_ok(n, m, p, max_steps)) return 0;
  return prune_ws_bytes(n, m, p, max_steps, nullptr, nullptr);
}

int varlingam_prune(const float* X, int64_t n, int64_t m, int64_t ldx, int p,
                    const int32_t* order, const double* B0, const double* Blag, int64_t max_steps,
                    double* B0_out, double* Blag_out, int32_t* info, void* ws, size_t ws_bytes,
                    int32_t* dev_status, void* stream) {
  if (!X || !order || !B0 || !Blag || !B0_out || !Blag_out || !dev_status)
    return VL_ERR_INVALID_ARG;
  if (!prune_shape_ok(n, m, p, max_steps)) return VL_ERR_SHAPE;
  if (ldx < m) return VL_ERR_INVALID_ARG;
  const size_t need = prune_ws_bytes(n, m, p, max_steps, nullptr, nullptr);
  if (!ws || ws_bytes < need || !aligned256(ws)) return VL_ERR_WORKSPACE;
  PruneWs w;
  prune_ws_bytes(n, m, p, max_steps, ws, &w);
  hipStream_t s = as_stream(stream);
  int rc = begin(dev_status, s);
  if (rc) return rc;
  return run_prune(n, m, p, w, X, ldx, order, B0, Blag, max_steps, B0_out, Blag_out, info,
                   dev_status, s);
}

// ----------------------------------------------------------------------------------------
static bool sim_shape_ok(int64_t m, int p, int64_t n_e, int64_t R, int64_t T) {
  return m >= 1 && p >= 1 && m * p <= 4096 && m * (p + 1) <= kSimMaxRing && n_e >= 1 &&
         R >= 1 && R <= 0x7fffffff && T >= 1;
}

size_t varlingam_var_simulate_workspace_bytes(int64_t m, int p) {
  if (!sim_shape_ok(m, p, 1, 1, 1)) return 0;
  return sim_ws_bytes(m, p);
}

int varlingam_var_simulate(const double* M, const double* intercept, int64_t m, int p,
                           const float* X0, int64_t ldx0, const float* E, int64_t n_e,
                           int64_t lde, const int32_t* idx, int64_t R, int64_t T, float* Xout,
                           int64_t ldxo, int64_t series_stride, void* ws, size_t ws_bytes,
                           int32_t* dev_status, void* stream) {
  if (!M || !intercept || !X0 || !E || !idx || !Xout || !dev_status) return VL_ERR_INVALID_ARG;
  if (!sim_shape_ok(m, p, n_e, R, T)) return VL_ERR_SHAPE;
  if (ldx0 < m || lde < m || ldxo < m || series_stride < (p + T) * ldxo)
    return VL_ERR_INVALID_ARG;
  if (!ws || ws_bytes < sim_ws_bytes(m, p) || !aligned256(ws)) return VL_ERR_WORKSPACE;
  hipStream_t s = as_stream(stream);
  int rc = begin(dev_status, s);
  if (rc) return rc;
  return run_var_simulate(M, intercept, m, p, X0, ldx0, E, n_e, lde, idx, R, T, Xout, ldxo,
                          series_stride, ws, dev_status, s);
}

size_t varlingam_edge_frequency_workspace_bytes(int64_t K, int64_t m) {
  if (K < 1 || m < 1 || m > 65536) return 0;
  return freq_ws_bytes(K, m);
}

int varlingam_edge_frequency(const int32_t* orders, const double* B0s, const double* Blags,
                             int64_t K, int64_t m, int p, double threshold,
                             const int32_t* problem_status, double* P0, double* Plag,
                             double* P_order, int32_t* count, void* ws, size_t ws_bytes,
                             int32_t* dev_status, void* stream) {
  if (!orders || !B0s || !P0 || !P_order || !count || !dev_status) return VL_ERR_INVALID_ARG;
  if (K < 1 || m < 1 || m > 65536 || p < 0) return VL_ERR_SHAPE;
  if (p > 0 && (!Blags || !Plag)) return VL_ERR_INVALID_ARG;
  if (!(threshold >= 0.0)) return VL_ERR_INVALID_ARG;
  if (!ws || ws_bytes < freq_ws_bytes(K, m) || !aligned256(ws)) return VL_ERR_WORKSPACE;
  hipStream_t s = as_stream(stream);
  int rc = begin(dev_status, s);
  if (rc) return rc;
  return run_edge_frequency(orders, B0s, Blags, K, m, p, threshold, problem_status, P0, Plag,
                            P_order, count, ws, dev_status, s);
}

}  // extern "C"
