/*
 * varlingam.h -- C ABI of the MI355X (gfx950) heuristic VarLiNGAM library.
 *
 * The library computes the hot path of the heuristic VarLiNGAM of Jiao, Guo and Luk,
 * "Scalable Time-Series Causal Discovery with Approximate Causal Ordering":
 *   VAR fit (Sec. 2.1)  ->  one-time precompute of every pairwise entropy statistic
 *   (Sec. 3 steps 1-3, Eqs. 1-2; Sec. 4.2 steps 1-2)  ->  lookup-only ordering
 *   (Alg. 1 with Eq. 3)  ->  B0 and lag matrices B_tau (Sec. 4, Sec. 2.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array arguments are DEVICE pointers owned by the caller.  Matrices are row-major
 *   with an explicit leading dimension (in elements).  Nothing is allocated inside the
 *   library: scratch memory comes from the caller's workspace `ws` of `ws_bytes` bytes,
 *   sized by the matching *_workspace_bytes() query and aligned to 256 bytes.
 * - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL = default stream).
 *   No entry point synchronises the stream.
 * - Errors a host check can see (null pointers, shapes, leading dimensions, workspace too
 *   small, unsupported sizes) are returned synchronously and nothing is enqueued.
 * - Errors that depend on the data (a constant column, |rho| = 1, a singular design, a
 *   non-finite input) are written by the kernels to the int32 `*dev_status` on the stream
 *   (VL_OK = 0 is written first by every call).  The caller reads it after synchronising.
 *   When dev_status holds an error the numerical outputs of that call are unspecified.
 * - Calls are reentrant given distinct workspaces and status words.
 */
#ifndef VARLINGAM_H
#define VARLINGAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VL_OK = 0,
  VL_ERR_INVALID_ARG = -1, /* null pointer, bad enum, leading dimension too small        */
  VL_ERR_SHAPE = -2,       /* sizes outside what the method or the library supports      */
  VL_ERR_DEGENERATE = -3,  /* zero-variance column or a pair with 1 - rho^2 < 1e-12      */
  VL_ERR_SINGULAR = -4,    /* VAR design (or residual covariance) not positive definite  */
  VL_ERR_NONFINITE = -5,   /* NaN or Inf in the input                                    */
  VL_ERR_WORKSPACE = -6,   /* workspace smaller than the *_workspace_bytes() query       */
  VL_ERR_HIP = -7          /* a HIP launch failed                                        */
} vl_status;

/* Arithmetic of the GEMM-shaped stages (the input series and E are always FP32; the pairwise
 * moments are always evaluated per sample in FP32, summed per wave in FP32 and across waves in
 * FP64; the score combination, the ordering and the B estimation always run in FP64).
 *   VL_PREC_FP32:  VAR Gram matrices, VAR residual GEMM and residual covariance by FP32 MFMA
 *                  with FP32 sums; FP64 Cholesky of the FP32 Gram.
 *   VL_PREC_MIXED: the same three products by FP64 MFMA on the widened FP32 data (exact
 *                  products, FP64 sums); FP64 Cholesky.
 *   VL_PREC_BF16:  VAR Gram matrices by BF16 MFMA (FP32 partial sums added in FP64), FP64
 *                  Cholesky of that Gram, then three FP64 refinement steps (the residual and
 *                  its correlation with the lags formed in FP64); residual GEMM and covariance
 *                  as MIXED.  Meant for well-conditioned lag designs: when the last
 *                  refinement step still changes the coefficients by more than 1e-6 of their
 *                  largest magnitude, the fit raises VL_ERR_SINGULAR.
 *   VL_PREC_FP32_REFINED: the FP32 Gram matrices of VL_PREC_FP32, FP64 Cholesky, one FP64
 *                  refinement step as in VL_PREC_BF16 (same convergence check), residual GEMM
 *                  and covariance as MIXED.  The cheapest form on the FP32 Gram that meets
 *                  the FP64 solution's accuracy.
 *   VL_PREC_SLICED: the three products of MIXED by int8 MFMA on slices of the data (each
 *                  vector scaled by a power of two and written as six signed 7-bit digits; the
 *                  digit pairs' products summed exactly in int32 and combined in FP64: the
 *                  Ozaki scheme), FP64 Cholesky.  Each product term is within 2^-39 of
 *                  2^(e_a + e_b), the two vectors' power-of-two scales: FP64-grade for the
 *                  Grams, far below the FP32 rounding of E.  Workspace: six int8 planes of the
 *                  lag-embedded columns (fit) or of E's columns (covariance).
 * The batched fit takes FP32 and MIXED only.
 *   VL_PAIRWISE_COMPENSATED: a flag OR-ed into the precision of pairwise_stats,
 *                  pairwise_stats_noalloc and pairwise_stats_workspace_bytes (no other call
 *                  takes it).  The pairwise moments are summed per lane with Kahan
 *                  compensation (Sec. 3 step 3, Eq. 2: the two sample means of each ordered
 *                  pair), reduced across the wave and stored per chunk in FP64, so their
 *                  rounding no longer grows with the samples a lane sums; the per-sample
 *                  evaluation stays FP32.  Costs six VALU operations more per pair, sample and
 *                  direction, and twice the chunk partials' workspace. */
typedef enum {
  VL_PREC_FP32 = 0,
  VL_PREC_MIXED = 1,
  VL_PREC_BF16 = 2,
  VL_PREC_FP32_REFINED = 3,
  VL_PREC_SLICED = 4,
  VL_PAIRWISE_COMPENSATED = 16
} vl_precision;

/* Human-readable name of a status code (static string, never NULL). */
const char* varlingam_status_string(int status);

/* ------------------------------------------------------------------------------------- */
/* VAR(p) least-squares fit (Sec. 2.1: VarLiNGAM first fits a VAR model and runs the      */
/* ordering on its residuals).                                                            */
/*                                                                                        */
/*   x(t) = sum_{tau=1..p} M_tau x(t - tau) + c + e(t),   t = p .. n-1                     */
/*                                                                                        */
/* X         n x m series, row t = sample t, leading dimension ldx >= m (float32).        */
/* M         out, p x m x m (float64): M[(tau-1)*m*m + i*m + k] = coefficient of           */
/*           x_k(t - tau) in the equation of x_i(t).                                       */
/* intercept out, m (float64).                                                             */
/* E         out, (n - p) x m residuals (float32), leading dimension lde >= m.             */
/* Host errors: m < 1, p < 1, n - p <= m p + 1, m p > 4096 -> VL_ERR_SHAPE.                */
/* Device errors: VL_ERR_NONFINITE, VL_ERR_SINGULAR (Gram of the centred lags not PD).     */
/* ------------------------------------------------------------------------------------- */
size_t varlingam_fit_var_workspace_bytes(int64_t n, int64_t m, int p, int prec);
int varlingam_fit_var(const float* X, int64_t n, int64_t m, int64_t ldx, int p, int prec,
                      double* M, double* intercept, float* E, int64_t lde, void* ws,
                      size_t ws_bytes, int32_t* dev_status, void* stream);

/* ------------------------------------------------------------------------------------- */
/* VAR lag-order selection, the step before the fit (Sec. 2.1 fits a VAR model with a     */
/* given p; the paper does not choose it).  Every p = 1 .. p_max is fitted by least        */
/* squares with intercept on the same sample t = p_max .. n-1 (T = n - p_max rows) and     */
/* scored with the maximum-likelihood residual covariance Sigma_p = E_p^T E_p / T:         */
/*   AIC(p) = ln det Sigma_p + 2 p m^2 / T,   BIC(p) = ln det Sigma_p + ln(T) p m^2 / T     */
/* (Lutkepohl 2005; the m intercepts, common to every p, are not counted).  FP64 Gram      */
/* (exact products of the FP32 data) and FP64 factorisations throughout.                   */
/* X       in, n x m float32 (leading dimension ldx >= m).                                  */
/* logdet, aic, bic  out, p_max float64 each (entry p - 1 for lag order p).                 */
/* best    out, 2 int32: the p minimising AIC and BIC (lowest p on ties).                   */
/* Host errors: m < 1, p_max < 1, n - p_max <= m p_max + 1 or m p_max > 4096 ->            */
/* VL_ERR_SHAPE.  Status: VL_ERR_NONFINITE, VL_ERR_SINGULAR (a singular design or residual */
/* covariance).                                                                            */
/* ------------------------------------------------------------------------------------- */
size_t varlingam_select_lag_workspace_bytes(int64_t n, int64_t m, int p_max);
int varlingam_select_lag(const float* X, int64_t n, int64_t m, int64_t ldx, int p_max,
                         double* logdet, double* aic, double* bic, int32_t* best, void* ws,
                         size_t ws_bytes, int32_t* dev_status, void* stream);

/* ------------------------------------------------------------------------------------- */
/* Precompute of every pairwise statistic, once (Sec. 4.2 steps 1-2; Alg. 1 first two     */
/* lines), from the unaltered residual matrix.                                            */
/*                                                                                        */
/* Each column e_i is standardised with population moments (Sec. 3 step 1) into x_i;       */
/* for every ordered pair i != j the residual r_{i<-j} = x_i - cov/var x_j of Eq. 1 is      */
/* re-standardised to u_{i<-j} and its entropy is approximated (Eq. 2) by                  */
/*   H(u) = (1 + ln 2pi)/2 - 79.047 (E[log cosh u] - 0.37457)^2 - 7.4129 (E[u e^{-u^2/2}])^2 */
/* Outputs (all float64, row-major m x m, leading dimension m):                            */
/*   Hx[i]      = H(x_i)                                           (size m)                */
/*   Hr[i*m+j]  = H(u_{i<-j}), diagonal 0                                                  */
/*   S[i*m+j]   = (Hx[j] + Hr[i,j]) - (Hx[i] + Hr[j,i]) = T_{j<-i} - T_{i<-j}; S = -S^T      */
/*                exactly; S[i,j] > 0 favours i before j                                   */
/*   Cov[i*m+j] = population covariance of e_i, e_j (feeds estimate_B)  -- may be NULL      */
/* E is n_eff x m float32 with leading dimension lde >= m.                                  */
/* Host errors: m < 2, n_eff < 2, m > 65536 -> VL_ERR_SHAPE.                                */
/* Device errors: VL_ERR_NONFINITE, VL_ERR_DEGENERATE.                                      */
/* ------------------------------------------------------------------------------------- */
size_t pairwise_stats_workspace_bytes(int64_t n_eff, int64_t m, int prec);
int pairwise_stats(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec, double* Hx,
                   double* Hr, double* S, double* Cov, void* ws, size_t ws_bytes,
                   int32_t* dev_status, void* stream);

/* ------------------------------------------------------------------------------------- */
/* pairwise_stats without a workspace argument, for callers that cannot allocate device    */
/* memory (code under HIP graph capture, tight serving loops, harnesses that forbid        */
/* hipMalloc).  Arguments, outputs and errors as pairwise_stats.                          */
/* Its scratch is a library-owned static device array of pairwise_stats_noalloc_max_bytes() */
/* bytes (64 MiB) per GPU, held from the first call on that GPU until the process ends:    */
/* n_eff and m whose pairwise_stats_workspace_bytes() exceed it return VL_ERR_WORKSPACE     */
/* (m = 400 with n_eff = 10^4 needs about 39 MB).  Nothing is allocated, freed or cleared   */
/* by the call: every scratch word the kernels read is written earlier in the same call.   */
/* All calls on one GPU share that array, so calls that overlap on one GPU (other streams,  */
/* other threads) race: serialise them.                                                    */
/* ------------------------------------------------------------------------------------- */
size_t pairwise_stats_noalloc_max_bytes(void);
int pairwise_stats_noalloc(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec,
                           double* Hx, double* Hr, double* S, double* Cov, int32_t* dev_status,
                           void* stream);

/* ------------------------------------------------------------------------------------- */
/* Gradient of the pairwise score (the precompute of Sec. 4.2 steps 1-2 with Eq. 1-2 made  */
/* differentiable): dE = d<G, S(E)>/dE for an m x m cotangent G.                           */
/*                                                                                        */
/* pairwise_stats_save() is pairwise_stats() that also writes `saved`, the statistics the  */
/* backward needs (pairwise_stats_saved_doubles(m) = 3 m^2 + 3 m doubles, device memory):  */
/* the moments (A, B) of every ordered pair, of every variable, the covariance and the     */
/* column means.  Its workspace is pairwise_stats_workspace_bytes().                        */
/*                                                                                        */
/* E     in, n_eff x m float32, leading dimension lde >= m (the same input as the forward). */
/* saved in, nullable: the block pairwise_stats_save() wrote for this E; with NULL the      */
/*       forward statistics are recomputed inside the call.  Nothing of size m^2 n is kept. */
/* G     in, m x m float64 row-major cotangent of S (only G - G^T matters: S is            */
/*       antisymmetric; the diagonal is ignored).                                          */
/* dE    out, n_eff x m float32, leading dimension ldde >= m.                              */
/* prec  arithmetic of the recomputed covariance (VL_PREC_FP32 or VL_PREC_MIXED); the      */
/*       per-sample terms are FP32, per-pair coefficients and column reductions FP64.      */
/* Deterministic: no floating-point atomics; repeated calls give identical bits.           */
/* Host errors: m < 2, n_eff < 2, m > 65536 -> VL_ERR_SHAPE.                                */
/* Device errors: as pairwise_stats (VL_ERR_NONFINITE, VL_ERR_DEGENERATE).                  */
/* ------------------------------------------------------------------------------------- */
size_t pairwise_stats_saved_doubles(int64_t m);
int pairwise_stats_save(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec,
                        double* Hx, double* Hr, double* S, double* Cov, double* saved, void* ws,
                        size_t ws_bytes, int32_t* dev_status, void* stream);
size_t pairwise_stats_backward_workspace_bytes(int64_t n_eff, int64_t m, int prec);
int pairwise_stats_backward(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec,
                            const double* saved, const double* G, float* dE, int64_t ldde,
                            void* ws, size_t ws_bytes, int32_t* dev_status, void* stream);

/* ------------------------------------------------------------------------------------- */
/* Lookup-only causal ordering (Alg. 1 main loop with Eq. 3): m steps over the static S.  */
/* At step k, with U the variables not yet ordered,                                       */
/*   M_i = sum_{j in U, j != i} min(0, S[i,j])^2,   c_k = argmin_{i in U} M_i              */
/* (exact ties -> lowest index), then U <- U \ {c_k}.                                      */
/* S        in, m x m float64 (leading dimension m), antisymmetric.                        */
/* order    out, m int32: order[k] = c_k.                                                  */
/* margin   out, m float64: second-smallest minus smallest M at step k; +inf at the last.  */
/* Host errors: m < 1 or m > 16384 -> VL_ERR_SHAPE.                                         */
/* ------------------------------------------------------------------------------------- */
size_t approx_order_workspace_bytes(int64_t m);
int approx_order(const double* S, int64_t m, int32_t* order, double* margin, void* ws,
                 size_t ws_bytes, int32_t* dev_status, void* stream);

/* ------------------------------------------------------------------------------------- */
/* Certified ordering: Alg. 1 as approx_order, where every step that the scores' error     */
/* bound cannot decide is re-decided on scores recomputed in FP64 (Eq. 1-3 in FP64 from E).  */
/* With |S_ij - S*_ij| <= eps_S for the scores passed in (S* the exact ones), M_i of Eq. 3   */
/* is within EM_i = sum_{j in U, S_ij < eps} eps (2 |min(0, S_ij)| + eps) of its exact      */
/* value; a step is settled when M_c + EM_c - (M_i - EM_i) <= 1e-9 for every other i (the  */
/* pick is then within 1e-9 of the exact minimum).  Otherwise the pick and every i that     */
/* breaks it have their rows and columns of S recomputed in FP64 (population-moment        */
/* standardisation, rho = mean(x_i x_j), both residuals, the Eq. 2 moments and H, FP64      */
/* throughout; those entries then count as exact), and the ordering runs again, until no    */
/* step is in doubt (at most m rounds; each refines at least one new row).                  */
/* E        in, n_eff x m float32 (leading dimension lde >= m): the data S was computed from. */
/* S        in/out, m x m float64 (from pairwise_stats): the refined rows are written back.  */
/* eps_S    in, the error bound of S's entries (>= 0; the FP32-moment scores of            */
/*          pairwise_stats stay within 6.1e-7 of the FP64 oracle on every workload tested).  */
/* order, margin  out as approx_order (margins of the final round).                           */
/* refined  out, nullable, m int32: 1 for a row recomputed in FP64.                           */
/* n_refined out, nullable, HOST pointer: number of rows recomputed.                          */
/* Unlike the other calls this one synchronises `stream` (once per round) to size the FP64  */
/* recomputation.  Host errors: m < 1, m > 4096, n_eff < 2 -> VL_ERR_SHAPE; eps_S < 0 or a  */
/* null pointer -> VL_ERR_INVALID_ARG.  Status: VL_ERR_DEGENERATE (a constant column or a    */
/* pair with 1 - rho^2 < 1e-12 among the recomputed ones).                                   */
/* ------------------------------------------------------------------------------------- */
size_t approx_order_certified_workspace_bytes(int64_t n_eff, int64_t m);
int approx_order_certified(const float* E, int64_t n_eff, int64_t m, int64_t lde, double* S,
                           double eps_S, int32_t* order, double* margin, int32_t* refined,
                           int64_t* n_refined, void* ws, size_t ws_bytes, int32_t* dev_status,
                           void* stream);

/* ------------------------------------------------------------------------------------- */
/* The original iterative DirectLiNGAM ordering (Sec. 3 steps 1-5), the search the       */
/* heuristic replaces: at step k, with U the variables not yet ordered and x_i their       */
/* current data, the pairwise scores S are recomputed on the current data exactly as       */
/* pairwise_stats does, c_k = argmin_{i in U} sum_{j in U, j != i} min(0, S[i,j])^2 (exact */
/* ties -> lowest index), and every other variable of U is replaced by its residual on     */
/* x_{c_k}, taken between the standardised columns (population moments):                 */
/*   x_j <- std(x_j) - rho_{j,c_k} std(x_{c_k}).                                           */
/* O(m^3 n) work: one pairwise pass over the remaining variables per step.                 */
/* E        in, n_eff x m float32 (leading dimension lde >= m), not modified.              */
/* prec     VL_PREC_FP32, VL_PREC_MIXED or VL_PREC_BF16 as for pairwise_stats.             */
/* order    out, m int32: order[k] = c_k (original variable index).                        */
/* margin   out, m float64: second-smallest minus smallest aggregate at step k; +inf at    */
/*          the last step.                                                                  */
/* Host errors: m < 1, m > 4096 or n_eff < 2 -> VL_ERR_SHAPE.  Status: as pairwise_stats   */
/* (a variable that becomes constant or collinear after the residual updates is           */
/* VL_ERR_DEGENERATE).                                                                     */
/* ------------------------------------------------------------------------------------- */
size_t varlingam_order_iterative_workspace_bytes(int64_t n_eff, int64_t m, int prec);
int varlingam_order_iterative(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec,
                              int32_t* order, double* margin, void* ws, size_t ws_bytes,
                              int32_t* dev_status, void* stream);

/* ------------------------------------------------------------------------------------- */
/* Hybrid ordering: the first k_exact picks of the original search above (with its residual */
/* updates), then the heuristic (Sec. 4.2, Alg. 1) on the refined data of the remaining     */
/* variables: one pairwise precompute and the lookup-only selection.  k_exact = 0 orders E */
/* exactly as pairwise_stats + approx_order do; k_exact >= m - 1 is the original search.   */
/* Arguments, workspace and errors as varlingam_order_iterative; order / margin entries     */
/* from k_exact on are the heuristic's.  k_exact < 0 -> VL_ERR_INVALID_ARG.                 */
/* ------------------------------------------------------------------------------------- */
size_t varlingam_order_hybrid_workspace_bytes(int64_t n_eff, int64_t m, int prec);
int varlingam_order_hybrid(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec,
                           int64_t k_exact, int32_t* order, double* margin, void* ws,
                           size_t ws_bytes, int32_t* dev_status, void* stream);

/* ------------------------------------------------------------------------------------- */
/* B0 and lag matrices from the order (Sec. 4: estimation of the instantaneous matrix B0; */
/* Sec. 2.1: VarLiNGAM lag matrices).                                                     */
/*   B0[K_k, K_<k] = least-squares coefficients of e_{K_k} on its predecessors, obtained   */
/*                   from the LDL^T factor of the order-permuted covariance:               */
/*                   Sigma_KK = L D L^T,  B0_KK = I - L^{-1};  every other entry 0;         */
/*   B_tau = (I - B0) M_tau.                                                               */
/* Cov   in, m x m float64 population covariance of the residuals (from pairwise_stats).  */
/* M     in, p x m x m float64 (from varlingam_fit_var); may be NULL when p == 0.          */
/* order in, m int32 permutation (from approx_order).                                      */
/* B0    out, m x m float64.   Blag out, p x m x m float64 (may be NULL when p == 0).       */
/* Host errors: m < 1, m > 16384, p < 0 -> VL_ERR_SHAPE.                                    */
/* Device errors: VL_ERR_SINGULAR (Cov not positive definite), VL_ERR_INVALID_ARG (order   */
/* is not a permutation).                                                                  */
/* ------------------------------------------------------------------------------------- */
size_t estimate_B_workspace_bytes(int64_t m, int p);
int estimate_B(const double* Cov, const double* M, const int32_t* order, int64_t m, int p,
               double* B0, double* Blag, void* ws, size_t ws_bytes, int32_t* dev_status,
               void* stream);

/* ------------------------------------------------------------------------------------- */
/* Pruning of B0 / B_tau, the step after the fit that the paper names (Sec. 7, future work) */
/* without specifying it.  Adaptive lasso (Zou 2006, weight exponent 1): variable i, at     */
/* position k of the order, is regressed with intercept on its k predecessors at lag 0 and  */
/* on all m variables at lags 1..p over t = p .. n-1 (d = k + m p columns); column j is      */
/* scaled by |b_j|, b = the unpruned coefficients (B0[i,:], B_tau[i,:], which are exactly    */
/* that regression's least-squares solution), and the lasso path is followed by LARS with   */
/* the lasso modification (Efron, Hastie, Johnstone and Tibshirani 2004).  Of its knots     */
/* (knot 0 = all zero) the one minimising BIC = T ln(RSS/T) + df ln T, df = nonzero          */
/* coefficients, is kept (the first on ties); a column with b_j = 0 stays 0.  The path ends  */
/* at the least-squares fit, once the active correlation falls below 1e-12 of its start,     */
/* or after max_steps steps (0: 8 d).  FP64 throughout, from an FP64 covariance of the FP32  */
/* series.                                                                                  */
/* X          in, n x m float32 (leading dimension ldx >= m), the series of the fit.         */
/* order      in, m int32, a permutation (causal order, most exogenous first).                */
/* B0, Blag   in, m x m and p x m x m float64, the unpruned estimates (estimate_B's layout). */
/* B0_out, Blag_out  out, same layouts: the pruned matrices (exact zeros where pruned).      */
/* info       out, nullable, 3 m int32: per variable (path steps, chosen knot, nonzeros).    */
/* Workspace: the m (p+1) square covariance plus, per variable, the inverse of its active    */
/* Gram (up to min(d, max_steps + 1) squared doubles) and 14 d doubles of path state.        */
/* Host errors: m < 1, p < 1, max_steps < 0, m (p+1) > 4096 or n - p <= m (p+1) + 1 ->       */
/* VL_ERR_SHAPE.  Status: VL_ERR_NONFINITE (the series), VL_ERR_INVALID_ARG (order not a     */
/* permutation).  B0 and Blag must be finite.                                                */
/* ------------------------------------------------------------------------------------- */
size_t varlingam_prune_workspace_bytes(int64_t n, int64_t m, int p, int64_t max_steps);
int varlingam_prune(const float* X, int64_t n, int64_t m, int64_t ldx, int p,
                    const int32_t* order, const double* B0, const double* Blag, int64_t max_steps,
                    double* B0_out, double* Blag_out, int32_t* info, void* ws, size_t ws_bytes,
                    int32_t* dev_status, void* stream);

/* ------------------------------------------------------------------------------------- */
/* Ensembles of the fit (rolling windows, residual bootstrap) run on the batched fit below; */
/* these two calls generate bootstrap series and aggregate the ensemble's results.          */
/*                                                                                        */
/* varlingam_var_simulate: residual bootstrap of the VAR of Sec. 2.1 (the model-based time- */
/* series bootstrap).  Resample b is rows 0 .. p+T-1 of Xout + b * series_stride (leading    */
/* dimension ldxo): rows 0..p-1 copy X0, then                                              */
/*   x*(t) = intercept + sum_{tau=1..p} M_tau x*(t - tau) + E[idx[b*T + t - p]]             */
/* in FP64 from the FP32 rows already written, stored as FP32.  M (p x m x m) and intercept  */
/* are varlingam_fit_var's outputs; E is an n_e x m float32 pool of residual rows (leading   */
/* dimension lde); idx (R x T int32) are the draws, made by the caller.                      */
/* Host errors: m < 1, p < 1, m p > 4096, m (p+1) > 8192, n_e < 1, R < 1, T < 1 ->            */
/* VL_ERR_SHAPE; ldx0, lde or ldxo < m, or series_stride < (p+T) ldxo -> VL_ERR_INVALID_ARG.  */
/* Status: VL_ERR_INVALID_ARG for a draw outside [0, n_e) (the nearest row is used).         */
/*                                                                                        */
/* varlingam_edge_frequency: over the K problems whose problem_status is VL_OK (all when    */
/* problem_status is NULL; *count = their number):                                          */
/*   P0[i*m+j]      = fraction with |B0_k[i][j]| > threshold                                 */
/*   Plag[..]       = the same for every B_tau (p x m x m; NULL when p = 0)                  */
/*   P_order[i*m+j] = fraction in which j precedes i in order_k                              */
/* orders K x m int32 (permutations), B0s K x m x m, Blags K x p x m x m float64, contiguous  */
/* stacks.  Exact: integer counts divided once.  threshold >= 0.                             */
/* Host errors: K < 1, m < 1, m > 65536, p < 0 -> VL_ERR_SHAPE; null pointers or a negative  */
/* threshold -> VL_ERR_INVALID_ARG.                                                          */
/* ------------------------------------------------------------------------------------- */
size_t varlingam_var_simulate_workspace_bytes(int64_t m, int p);
int varlingam_var_simulate(const double* M, const double* intercept, int64_t m, int p,
                           const float* X0, int64_t ldx0, const float* E, int64_t n_e,
                           int64_t lde, const int32_t* idx, int64_t R, int64_t T, float* Xout,
                           int64_t ldxo, int64_t series_stride, void* ws, size_t ws_bytes,
                           int32_t* dev_status, void* stream);
size_t varlingam_edge_frequency_workspace_bytes(int64_t K, int64_t m);
int varlingam_edge_frequency(const int32_t* orders, const double* B0s, const double* Blags,
                             int64_t K, int64_t m, int p, double threshold,
                             const int32_t* problem_status, double* P0, double* Plag,
                             double* P_order, int32_t* count, void* ws, size_t ws_bytes,
                             int32_t* dev_status, void* stream);

/* ------------------------------------------------------------------------------------- */
/* Batched fit: many independent VarLiNGAM problems of uneven size (for instance rolling     */
/* windows or many datasets) through the whole path -- VAR fit (Sec. 2.1), pairwise         */
/* precompute (Sec. 4.2, Eq. 1-2), ordering (Alg. 1, Eq. 3), B0 / B_tau -- with one kernel  */
/* launch per stage for all problems.                                                      */
/*                                                                                        */
/* vl_instance describes one problem; all pointers are device pointers owned by the caller. */
/*   X, n, m, ldx, p   the series (n x m float32, leading dimension ldx >= m) and VAR lag.   */
/*   M, intercept, E, lde, S, order, margin, B0, Blag   outputs as in varlingam_fit_var,     */
/*                     pairwise_stats, approx_order and estimate_B (S and margin may be     */
/*                     NULL: they are then kept in the workspace only).                    */
/* Per-problem limits: 2 <= m <= 256, p >= 1, m p <= 256, n - p > m p + 1.                 */
/* Usage: varlingam_batch_create() plans the batch on the host (the descriptors are copied; */
/* the device buffers they name must stay valid); varlingam_batch_bind() uploads the plan's */
/* tables into a workspace of varlingam_batch_workspace_bytes() (256-byte aligned) and      */
/* waits for the copy; varlingam_fit_batched() then only launches kernels on `stream`, so a */
/* caller may capture it in a HIP graph and replay it after refilling the X buffers.        */
/* dev_status has one word per problem (VL_OK or that problem's first data-dependent error); */
/* an error in one problem does not stop the others.                                        */
/* varlingam_batch_autotune() picks the sample-chunk length of the pairwise stage per      */
/* bucket of problems (m <= 32, 64, 128, 256 times n - p <= 1024, 2048, 4096, more), timing */
/* whole fits on the bound data: first the fastest length common to all buckets, then one  */
/* pass of coordinate descent over the buckets by decreasing m^2 (n - p) work (a change is  */
/* kept if the fit gets at least 1% faster); then it rebinds.  Choices are cached per       */
/* device, precision and bucket in the process and in a text file: $VL_TUNE_CACHE (empty:  */
/* no file), else $XDG_CACHE_HOME/varlingam/batch_tune.txt, else                            */
/* $HOME/.cache/varlingam/batch_tune.txt, named anew at each call (the process's copy is   */
/* read again when a call names another file); buckets found there are not timed again.    */
/* Calls on one batch must not overlap.  varlingam_batch_chunk_len() returns the length of  */
/* the bucket with the most problems, varlingam_batch_chunk_len_of() that of one problem    */
/* (0 for a bad index).                                                                     */
/* Host errors: VL_ERR_SHAPE for a problem outside the limits, VL_ERR_INVALID_ARG for null  */
/* pointers, a bad precision or a workspace that is not the bound one.                      */
/* ------------------------------------------------------------------------------------- */
typedef struct {
  const float* X;
  int64_t n, m, ldx;
  int32_t p, reserved;
  double* M;
  double* intercept;
  float* E;
  int64_t lde;
  double* S;
  int32_t* order;
  double* margin;
  double* B0;
  double* Blag;
} vl_instance;

typedef struct vl_batch vl_batch;

int varlingam_batch_create(const vl_instance* inst, int count, int prec, vl_batch** out);
size_t varlingam_batch_workspace_bytes(const vl_batch* batch);
int varlingam_batch_bind(vl_batch* batch, void* ws, size_t ws_bytes, void* stream);
int varlingam_fit_batched(const vl_batch* batch, void* ws, int32_t* dev_status, void* stream);
int varlingam_batch_autotune(vl_batch* batch, void* ws, size_t ws_bytes, int32_t* dev_status,
                             void* stream);
int varlingam_batch_chunk_len(const vl_batch* batch);
int varlingam_batch_chunk_len_of(const vl_batch* batch, int problem);
void varlingam_batch_destroy(vl_batch* batch);

/* ------------------------------------------------------------------------------------- */
/* Stage timing (diagnostics).  varlingam_profile_enable(stages) starts recording a HIP    */
/* event pair, on the caller's stream, around every launch of the named stages ("*" = all; */
/* a comma-separated list; NULL or "" = off) and clears earlier totals.  Stage names:       */
/*   var_gram, var_solve, var_residual, var_refine, pairwise_cov, pairwise_prep,            */
/*   pairwise_moments, pairwise_combine, backward_prep, backward_owner, backward_tail,       */
/*   order, estimate_b, batch_var, batch_pairwise, batch_moments, batch_order_b, iterative, */
/*   certify,                                                                              */
/*   lag_scores, prune, simulate.                                                           */
/* varlingam_profile_read() waits for the recorded events of one stage and returns the      */
/* accumulated milliseconds and the number of recorded launches.  Thread-safe.              */
/* ------------------------------------------------------------------------------------- */
void varlingam_profile_enable(const char* stages);
int varlingam_profile_read(const char* stage, double* total_ms, int64_t* count);

/* ------------------------------------------------------------------------------------- */
/* Issue-rate probes (diagnostics; the measured denominators of the rooflines): rates[0] =   */
/* FP32 exp2 per second (the transcendental unit), rates[1] = FP32 FMA flop per second,      */
/* rates[2] = FP64 MFMA (16x16x4) flop per second, each from a kernel of independent         */
/* dependency chains filling every CU (8 waves per SIMD), timed with HIP events on `stream`.  */
/* rates is a HOST pointer (3 doubles); ws a device buffer of                                 */
/* varlingam_probe_workspace_bytes() bytes.  Synchronises `stream`.                           */
/* ------------------------------------------------------------------------------------- */
size_t varlingam_probe_workspace_bytes(void);
int varlingam_probe_rates(double* rates, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* VARLINGAM_H */
