// VAR(p) least-squares fit with intercept (Sec. 2.1: VarLiNGAM fits a VAR model first and runs
// the ordering on its residuals).
//
//   Y = x(t), Z = [x(t-1), ..., x(t-p)] for t = p .. n-1 (n_eff = n - p rows), centred by their
//   column means so the intercept drops out of the normal equations:
//     G = Zc^T Zc (mp x mp),  R = Zc^T Yc (mp x m),  G Coef = R,
//     E = Yc - Zc Coef,  c = mean(Y) - Coef^T mean(Z).
//   The lagged views are row offsets of X (a column map), never copies.
//   MIXED: Gram matrices by FP64 MFMA on the widened FP32 data (exact products, FP64 sums), FP64
//          Cholesky solve, residual GEMM by FP64 MFMA, E rounded to FP32 once.
//   FP32:  Gram and residual GEMM by FP32 MFMA with FP32 sums; FP64 Cholesky; no refinement.
//   FP32_REFINED: the FP32 Gram of plain FP32, then one refinement step as BF16 below, and
//          the residual GEMM by FP64 MFMA: the cheapest form built on the FP32 Gram that
//          reaches the FP64 solution's accuracy.
//   BF16:  Gram matrices by BF16 MFMA (FP32 sums flushed to FP64), FP64 Cholesky of that Gram,
//          then kBf16RefineSteps refinement steps Coef += G^{-1} Zc^T E64 with the residual
//          E64 = Yc - Zc Coef and its correlation with Zc formed in FP64 (exact products of the
//          FP32 data); each step shrinks the error by about cond(G) times the BF16 Gram's
//          relative error.  A last correction above 1e-6 of max|Coef| (no convergence: the
//          design is too ill-conditioned for a BF16 Gram) raises VL_ERR_SINGULAR.
#include "gram.hpp"
#include "linalg.hpp"
#include "var_fit.hpp"
#include "sliced.hpp"
#include "var_dev.hpp"
#include "profile.hpp"

namespace vl {

// Refinement steps after the BF16 Gram solve (contraction ~cond(G) 2^-8 per step).
constexpr int kBf16RefineSteps = 3;


// colmap[tau*m + i] = (p - tau) * ldx + i  for tau = 0..p  (tau = 0 is Y, tau >= 1 is Z)
__global__ void lag_colmap_kernel(int64_t m, int p, int64_t ldx, int64_t* __restrict__ colmap) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m * (p + 1)) return;
  const int64_t tau = c / m, i = c % m;
  colmap[c] = (p - tau) * ldx + i;
}

__global__ void to_f32_kernel(const double* __restrict__ a, int64_t n, float* __restrict__ b) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = (float)a[e];
}

__global__ void add_f64_kernel(double* __restrict__ a, const double* __restrict__ d, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) a[e] += d[e];
}

// Convergence of the refinement: the last correction d must be below tol * max|c| (and
// finite), else the design is too ill-conditioned for the low-precision Gram and
// VL_ERR_SINGULAR is raised.  BF16 (three steps): the last correction must have shrunk to
// kRefineTolBf16.  FP32_REFINED (one step): the correction is the FP32 solve's error, and
// below kRefineTolFp32 the step contracts it by cond(G) u_FP32 < 1e-3 at least.  Per-workgroup
// partials into the split scratch, then one workgroup.
constexpr double kRefineTolBf16 = 1e-6;
constexpr double kRefineTolFp32 = 1e-3;

constexpr int kCheckBlocks = 256;

// Per workgroup: max |d|, max |c| and a non-finite flag over a grid-stride slice.
__global__ __launch_bounds__(256) void refine_partial_kernel(const double* __restrict__ d,
                                                             const double* __restrict__ c,
                                                             int64_t n, double* __restrict__ part) {
  __shared__ double sd[256], sc[256], sb[256];
  double md = 0.0, mc = 0.0, bad = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const double dv = d[e], cv = c[e];
    if (!isfinite(dv) || !isfinite(cv)) bad = 1.0;
    md = fmax(md, fabs(dv));
    mc = fmax(mc, fabs(cv));
  }
  sd[threadIdx.x] = md;
  sc[threadIdx.x] = mc;
  sb[threadIdx.x] = bad;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + h]);
      sc[threadIdx.x] = fmax(sc[threadIdx.x], sc[threadIdx.x + h]);
      sb[threadIdx.x] = fmax(sb[threadIdx.x], sb[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = sd[0];
    part[3 * blockIdx.x + 1] = sc[0];
    part[3 * blockIdx.x + 2] = sb[0];
  }
}

// One workgroup over the partials: the correction must be finite and below tol of the
// solution.
__global__ __launch_bounds__(256) void refine_check_kernel(const double* __restrict__ part,
                                                           int nb, double tol, int32_t* st) {
  __shared__ double sd[256], sc[256], sb[256];
  double md = 0.0, mc = 0.0, bad = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    md = fmax(md, part[3 * b]);
    mc = fmax(mc, part[3 * b + 1]);
    bad = fmax(bad, part[3 * b + 2]);
  }
  sd[threadIdx.x] = md;
  sc[threadIdx.x] = mc;
  sb[threadIdx.x] = bad;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + h]);
      sc[threadIdx.x] = fmax(sc[threadIdx.x], sc[threadIdx.x + h]);
      sb[threadIdx.x] = fmax(sb[threadIdx.x], sb[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && (sb[0] != 0.0 || !(sd[0] <= tol * sc[0])))
    raise_status(st, VL_ERR_SINGULAR);
}

__global__ __launch_bounds__(256) void var_residual_kernel(
    const float* __restrict__ X, int64_t ldx, const int64_t* __restrict__ colmap,
    const double* __restrict__ mu, int64_t m, int p, int64_t n_eff,
    const float* __restrict__ CoefF, float* __restrict__ E, int64_t lde) {
  var_residual_tile_f32(X, ldx, colmap, mu, m, p, n_eff, CoefF, E, lde,
                        (int64_t)blockIdx.y * 64, (int64_t)blockIdx.x * 64);
}

template <class TOut, int RT, int RK>
__global__ __launch_bounds__(256) void var_residual_f64w_kernel(
    const float* __restrict__ X, int64_t ldx, const int64_t* __restrict__ colmap,
    const double* __restrict__ mu, int64_t m, int p, int64_t n_eff,
    const double* __restrict__ Coef, TOut* __restrict__ E, int64_t lde) {
  var_residual_tile_f64w<TOut, RT, RK>(X, ldx, colmap, mu, m, p, n_eff, Coef, E, lde,
                                       (int64_t)blockIdx.y * RT, (int64_t)blockIdx.x * kRJ);
}

// The residual's tile shape.  The loop is bound by load latency, so occupancy decides: below
// ~8 workgroups per CU at 64 samples a tile, 32-sample tiles with 32 lags a stage (four waves
// per SIMD) beat the wider tiles (m = 400, n = 10000, p = 2: 194 us against 224 us at 64 x 16
// and 288 us at 128 x 16, the same bits); above it 64 x 16 is ~2% ahead.
template <class TOut>
static void launch_residual_f64w(const float* X, int64_t ldx, const int64_t* colmap,
                                 const double* mu, int64_t m, int p, int64_t n_eff,
                                 const double* Coef, TOut* E, int64_t lde, hipStream_t stream) {
  const int64_t tj = ceil_div(m, (int64_t)kRJ);
  if (ceil_div(n_eff, (int64_t)64) * tj >= 8 * 256) {
    dim3 grid((unsigned)tj, (unsigned)ceil_div(n_eff, (int64_t)64));
    var_residual_f64w_kernel<TOut, 64, 16><<<grid, 256, 0, stream>>>(X, ldx, colmap, mu, m, p,
                                                                     n_eff, Coef, E, lde);
  } else {
    dim3 grid((unsigned)tj, (unsigned)ceil_div(n_eff, (int64_t)32));
    var_residual_f64w_kernel<TOut, 32, 32><<<grid, 256, 0, stream>>>(X, ldx, colmap, mu, m, p,
                                                                     n_eff, Coef, E, lde);
  }
}

// After the solve, in one launch: blocks [0, nlag) write the lag matrices,
// M[(tau-1) m m + i m + k] = Coef[(tau-1) m + k][i]; the blocks after them the intercepts,
// c[i] = muY[i] - sum_k' Coef[k'][i] muZ[k'], one wave per variable.
__global__ __launch_bounds__(256) void var_post_kernel(const double* __restrict__ Coef,
                                                       const double* __restrict__ mu, int64_t m,
                                                       int p, int64_t nlag,
                                                       double* __restrict__ M,
                                                       double* __restrict__ intercept) {
  if ((int64_t)blockIdx.x < nlag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)p * m * m) return;
    const int64_t tau1 = e / (m * m), rem = e % (m * m), i = rem / m, k = rem % m;
    M[e] = Coef[(tau1 * m + k) * m + i];
    return;
  }
  const int64_t dz = m * p;
  const int64_t i = ((int64_t)blockIdx.x - nlag) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= m) return;
  double s = 0.0;
  for (int64_t k = lane; k < dz; k += 64) s += Coef[k * m + i] * mu[m + k];
  s = wave_sum_d(s);
  if (lane == 0) intercept[i] = mu[i] - s;
}

VarPlan plan_var(int64_t n, int64_t m, int p, bool sliced) {
  VarPlan v;
  v.sliced = sliced;
  v.n = n;
  v.m = m;
  v.p = p;
  v.n_eff = n - p;
  v.dz = m * p;
  return v;
}

size_t var_ws_bytes(const VarPlan& v, void* base, VarWs* out) {
  Carver c(base);
  VarWs w;
  const int64_t nc = v.m * (v.p + 1);
  w.colmap = c.take<int64_t>(nc);
  w.mu = c.take<double>(nc);
  w.G = c.take<double>(v.dz * v.dz);
  w.Coef = c.take<double>(v.dz * v.m);
  w.Rres = c.take<double>(v.dz * v.m);
  w.CoefF = c.take<float>(v.dz * v.m);
  w.L = c.take<double>(v.dz * v.dz);
  w.Tmp = c.take<double>(v.dz * v.m);
  w.chol = c.take<double>(chol_ws_doubles(v.dz));
  w.E64 = c.take<double>(v.n_eff * v.m);
  w.F = c.take<double>(v.m * nc);
  w.mu0 = c.take<double>(nc);
  size_t s1 = (size_t)colmean_splits(v.n_eff) * nc * (v.sliced ? 3 : 1);
  size_t s2 = (size_t)gram_splits(v.m, nc, v.n_eff) * v.m * nc;      // lag products
  size_t s3 = (size_t)gram_splits(v.dz, v.m, v.n_eff) * v.dz * v.m;   // R, refinement Gram
  size_t s4 = (size_t)gram_splits(v.dz, v.dz, v.n_eff) * v.dz * v.dz; // direct G
  size_t s = s1 > s2 ? s1 : s2;
  s = s > s3 ? s : s3;
  s = s > s4 ? s : s4;
  s = s > (size_t)(3 * kCheckBlocks) ? s : (size_t)(3 * kCheckBlocks);  // refinement check
  if (v.sliced) s = std::max(s, (size_t)slice_gram_splits(v.m, nc, v.n_eff, false) * v.m * nc);
  w.scratch = c.take<double>(s);
  if (v.sliced) {
    w.slices = c.take<int8_t>(std::max(slice_bytes(nc, v.n_eff), slice_bytes(v.n_eff, v.dz)));
    w.slicesC = c.take<int8_t>(slice_bytes(v.m, v.dz));
    w.ex = c.take<int32_t>(nc);
    w.ez = c.take<int32_t>(nc);
    w.ec = c.take<int32_t>(v.m);
  }
  if (out) *out = w;
  return c.used;
}

static int var_residual(const VarPlan& v, const VarWs& w, const float* X, int64_t ldx, float* E,
                        int64_t lde, bool fp64, hipStream_t stream) {
  if (v.sliced) {
    // E = Yc - Zc Coef from the slices of the design rows and of the coefficient columns
    const int64_t kpad = slice_ldk(v.dz);
    const int32_t* f = w.ez + v.m;      // design column k: lag-embedded column m + k
    int rc = slice_design(X, ldx, w.colmap, w.mu, f, v.m, v.dz, v.n_eff, w.slices, stream);
    if (rc) return rc;
    rc = slice_matrix_columns(w.Coef, f, v.dz, v.m, w.slicesC, w.ec, stream);
    if (rc) return rc;
    SliceOp A, B;
    A.D = w.slices;
    A.rows = v.n_eff;
    A.plane = v.n_eff * kpad;
    B.D = w.slicesC;
    B.rows = v.m;
    B.plane = v.m * kpad;
    B.e = w.ec;
    return slice_residual<float>(A, v.n_eff, B, v.m, v.dz, X, ldx, w.colmap, w.mu, E, lde,
                                 stream);
  }
  if (fp64) {
    launch_residual_f64w<float>(X, ldx, w.colmap, w.mu, v.m, v.p, v.n_eff, w.Coef, E, lde,
                                stream);
    VL_LAUNCH_CHECK();
    return VL_OK;
  }
  const int64_t nz = v.dz * v.m;
  to_f32_kernel<<<(unsigned)ceil_div(nz, 256), 256, 0, stream>>>(w.Coef, nz, w.CoefF);
  VL_LAUNCH_CHECK();
  dim3 grid((unsigned)ceil_div(v.m, 64), (unsigned)ceil_div(v.n_eff, 64));
  var_residual_kernel<<<grid, 256, 0, stream>>>(X, ldx, w.colmap, w.mu, v.m, v.p, v.n_eff,
                                                w.CoefF, E, lde);
  VL_LAUNCH_CHECK();
  return VL_OK;
}


// G (dz x dz, both triangles) and R (dz x m) of the VAR normal equations from the lag products
// F (see var_normal_equations).  Column (tau, i) of the regression is x_i(t - tau), t = p .. n-1,
// with window mean mu[tau m + i]; xt = x - mu_0 and d_tau = mu_tau - mu_0.  For tau1 >= tau2,
// h = tau1 - tau2, the window sum sum_t xt_j(t - tau2) xt_i(t - tau1) is F_h[j][i] with the
// tau2 rows that the window gains at its start added and the tau2 rows it loses at its end taken
// away, and G = that sum - n_eff d_tau1[i] d_tau2[j].  R's block tau is F_tau^T (d_0 = 0).
__global__ void var_assemble_kernel(const float* __restrict__ X, int64_t ldx,
                                    const double* __restrict__ F, const double* __restrict__ mu,
                                    int64_t m, int p, int64_t n, double* __restrict__ G,
                                    double* __restrict__ R) {
  const int64_t dz = m * p, nc = m * (p + 1);
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < dz * dz) {
    const int64_t r = e / dz, c = e % dz;
    if (c > r) return;
    const int64_t t1 = r / m + 1, i = r % m, t2 = c / m + 1, j = c % m, h = t1 - t2;
    const double ci = mu[i], cj = mu[j];
    double wv = F[j * nc + h * m + i];
    for (int64_t s = p - t2; s < p; ++s)
      wv += ((double)X[s * ldx + j] - cj) * ((double)X[(s - h) * ldx + i] - ci);
    for (int64_t s = n - t2; s < n; ++s)
      wv -= ((double)X[s * ldx + j] - cj) * ((double)X[(s - h) * ldx + i] - ci);
    const double di = mu[t1 * m + i] - ci, dj = mu[t2 * m + j] - cj;
    const double g = wv - (double)(n - p) * di * dj;
    G[r * dz + c] = g;
    G[c * dz + r] = g;
    return;
  }
  e -= dz * dz;
  if (e >= dz * m) return;
  const int64_t r = e / m, j = e % m;
  R[r * m + j] = F[j * nc + m + r];
}

// Column map, means, G = Zc^T Zc and R = Zc^T Yc (R into Tmp, where the forward substitution
// of the factorisation works on it).
// * FP64 products (kFp64): the p^2 + p blocks of G and R are shifted windows of p + 1 lag
//   products F_h[i][j] = sum_{s = p}^{n-1} xt_i(s) xt_j(s - h), h = 0 .. p, so one Gram of the
//   lag-0 columns against all m (p + 1) columns (every one centred by the lag-0 means) and a
//   rank-2p boundary correction per entry give them: m^2 (p + 1) n products instead of
//   (p^2 / 2 + p) m^2 n.  The products are exact, so the assembled G equals the direct one to
//   FP64 rounding.
// * FP32 and BF16 products: the direct Grams.  A Gram of rounded data is the exact Gram of
//   slightly different data, hence positive semidefinite; G assembled from rounded lag
//   products and exact corrections is not the Gram of anything and loses definiteness at
//   BF16's 2^-9 (an emulation at m = 70, p = 4, cond(G) = 1e4: smallest eigenvalue 136 exact,
//   136 direct, -307 assembled).
static int var_normal_equations(const VarPlan& v, const VarWs& w, const float* X, int64_t ldx,
                                GramMode gmode, int32_t* st, hipStream_t stream) {
  const int64_t m = v.m, dz = v.dz, n_eff = v.n_eff;
  const int64_t nc = m * (v.p + 1);
  int rc;
  {
    ProfileScope ps("var_gram", stream);
    lag_colmap_kernel<<<(unsigned)ceil_div(nc, 256), 256, 0, stream>>>(m, v.p, ldx, w.colmap);
    VL_LAUNCH_CHECK();
    // MIXED also needs the lag-0 means once per lag block (mu0), written by the same pass
    // (sliced: with each lag-embedded column's range exponent about its lag-0 mean)
    const bool fp64 = gmode == GramMode::kFp64 && !v.sliced;
    rc = colmeans(X, ldx, w.colmap, nc, n_eff, w.mu, w.scratch, st, stream,
                  fp64 ? w.mu0 : nullptr, m, v.p + 1, v.sliced ? w.ex : nullptr, m,
                  v.sliced ? w.ez : nullptr);
    if (rc) return rc;
    if (v.sliced) {
      // the same lag products F from int8 slices of the series centred by the lag-0 means
      // (w.mu[0 .. m))
      rc = slice_columns(X, ldx, m, v.p + 1, v.p, n_eff, w.mu, w.ex, w.slices, stream);
      if (rc) return rc;
      SliceOp D;
      D.D = w.slices;
      D.rows = nc;
      D.plane = nc * slice_ldk(n_eff);
      D.e = w.ex;
      rc = slice_gram(D, m, D, nc, n_eff, 1.0, w.F, nc, w.scratch, stream);
      if (rc) return rc;
      var_assemble_kernel<<<(unsigned)ceil_div(dz * dz + dz * m, 256), 256, 0, stream>>>(
          X, ldx, w.F, w.mu, m, v.p, v.n, w.G, w.Tmp);
      VL_LAUNCH_CHECK();
      return VL_OK;
    }
    if (fp64) {
      rc = gram_tn(X, ldx, w.colmap, w.mu, m, X, ldx, w.colmap, w.mu0, nc, n_eff, gmode, 1.0,
                   w.F, nc, w.scratch, stream);
      if (rc) return rc;
      var_assemble_kernel<<<(unsigned)ceil_div(dz * dz + dz * m, 256), 256, 0, stream>>>(
          X, ldx, w.F, w.mu, m, v.p, v.n, w.G, w.Tmp);
      VL_LAUNCH_CHECK();
      return VL_OK;
    }
    const int64_t* mapZ = w.colmap + m;
    const double* muZ = w.mu + m;
    rc = gram_tn(X, ldx, mapZ, muZ, dz, X, ldx, mapZ, muZ, dz, n_eff, gmode, 1.0, w.G, dz,
                 w.scratch, stream, true);
    if (rc) return rc;
    rc = gram_tn(X, ldx, mapZ, muZ, dz, X, ldx, w.colmap, w.mu, m, n_eff, gmode, 1.0, w.Tmp, m,
                 w.scratch, stream);
    if (rc) return rc;
  }
  return VL_OK;
}

size_t lag_cov_scratch_doubles(int64_t n, int64_t m, int p) {
  const int64_t nc = m * (p + 1), n_eff = n - p;
  const size_t s1 = (size_t)colmean_splits(n_eff) * nc;
  const size_t s2 = (size_t)gram_splits(nc, nc, n_eff) * nc * nc;
  return s1 > s2 ? s1 : s2;
}

int lag_covariance(int64_t n, int64_t m, int p, const float* X, int64_t ldx, int64_t* colmap,
                   double* mu, double* C, double* scratch, int32_t* st, hipStream_t stream) {
  const int64_t nc = m * (p + 1), n_eff = n - p;
  lag_colmap_kernel<<<(unsigned)ceil_div(nc, 256), 256, 0, stream>>>(m, p, ldx, colmap);
  VL_LAUNCH_CHECK();
  int rc = colmeans(X, ldx, colmap, nc, n_eff, mu, scratch, st, stream);
  if (rc) return rc;
  return gram_tn(X, ldx, colmap, mu, nc, X, ldx, colmap, mu, nc, n_eff, GramMode::kFp64, 1.0, C,
                 nc, scratch, stream, true);
}

int run_var(const VarPlan& v, const VarWs& w, const float* X, int64_t ldx, int prec, double* M,
            double* intercept, float* E, int64_t lde, int32_t* st, hipStream_t stream) {
  const int64_t m = v.m, dz = v.dz, n_eff = v.n_eff;
  const bool plain = prec == VL_PREC_FP32;
  const bool refine = prec == VL_PREC_BF16 || prec == VL_PREC_FP32_REFINED;
  const GramMode gmode = (plain || prec == VL_PREC_FP32_REFINED) ? GramMode::kFp32
                         : prec == VL_PREC_BF16                 ? GramMode::kBf16
                                                                : GramMode::kFp64;
  const int steps = prec == VL_PREC_BF16 ? kBf16RefineSteps : 1;
  const int64_t* mapZ = w.colmap + m;
  const double* muZ = w.mu + m;
  int rc = var_normal_equations(v, w, X, ldx, gmode, st, stream);
  if (rc) return rc;
  {
    // G = L L^T with Tmp <- L^{-1} R and L <- L^{-1} in the same pass; Coef = L^{-T} Tmp
    ProfileScope ps("var_solve", stream);
    rc = chol_solve_lower(w.G, dz, dz, w.Tmp, m, m, w.L, dz, w.chol, st, stream);
    if (rc) return rc;
    rc = gemm_f64(dz, m, dz, 1.0, w.L, dz, true, w.Tmp, m, false, 0.0, w.Coef, m, false, stream,
                  2);
    if (rc) return rc;
  }
  if (refine) {
    ProfileScope ps("var_refine", stream);
    for (int it = 0; it < steps; ++it) {
      launch_residual_f64w<double>(X, ldx, w.colmap, w.mu, m, v.p, n_eff, w.Coef, w.E64, m,
                                   stream);
      VL_LAUNCH_CHECK();
      rc = gram_tn_f64b(X, ldx, mapZ, muZ, dz, w.E64, m, m, n_eff, w.Rres, m, w.scratch, stream);
      if (rc) return rc;
      // correction L^{-T} L^{-1} Rres (two triangular products with the explicit inverse)
      rc = gemm_f64(dz, m, dz, 1.0, w.L, dz, false, w.Rres, m, false, 0.0, w.Tmp, m, false,
                    stream, 1);
      if (rc) return rc;
      rc = gemm_f64(dz, m, dz, 1.0, w.L, dz, true, w.Tmp, m, false, 0.0, w.Rres, m, false,
                    stream, 2);
      if (rc) return rc;
      add_f64_kernel<<<(unsigned)ceil_div(dz * m, 256), 256, 0, stream>>>(w.Coef, w.Rres, dz * m);
      VL_LAUNCH_CHECK();
    }
    const int64_t nbl = ceil_div(dz * m, 256);
    const int nb = (int)(nbl < kCheckBlocks ? nbl : kCheckBlocks);
    refine_partial_kernel<<<nb, 256, 0, stream>>>(w.Rres, w.Coef, dz * m, w.scratch);
    VL_LAUNCH_CHECK();
    refine_check_kernel<<<1, 256, 0, stream>>>(
        w.scratch, nb, prec == VL_PREC_BF16 ? kRefineTolBf16 : kRefineTolFp32, st);
    VL_LAUNCH_CHECK();
  }
  {
    ProfileScope ps("var_residual", stream);
    rc = var_residual(v, w, X, ldx, E, lde, !plain, stream);
    if (rc) return rc;
  }
  {
    const int64_t nlag = ceil_div(dz * m, (int64_t)256);
    var_post_kernel<<<(unsigned)(nlag + ceil_div(m, (int64_t)4)), 256, 0, stream>>>(
        w.Coef, w.mu, m, v.p, nlag, M, intercept);
    VL_LAUNCH_CHECK();
  }
  return VL_OK;
}

// ------------------------------------------------------------------------------------------
// Lag-order selection, the step before the fit (the paper fixes p): every p = 1 .. p_max on the
// common sample t = p_max .. n-1 (T rows), scored with the ML residual covariance Sigma_p:
//   AIC(p) = ln det Sigma_p + 2 p m^2 / T,   BIC(p) = ln det Sigma_p + ln(T) p m^2 / T.
// On a common sample the lag-p normal equations are the leading (p m) block of the lag-p_max
// ones, and the Cholesky factor of a leading block is the leading block of the factor, so one
// Gram and one factorisation serve every p: with W = L^{-1} R (rows in lag blocks W_1, W_2, ..)
//   T Sigma_p = Yc^T Yc - R_p^T G_p^{-1} R_p = Yc^T Yc - sum_{tau <= p} W_tau^T W_tau,
// and ln det Sigma_p = -2 sum_i ln (L_p^{-1})_ii - m ln T from the factor of T Sigma_p.
// ------------------------------------------------------------------------------------------
__global__ void lag_copy_kernel(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = a[e];
}

__global__ __launch_bounds__(256) void lag_scores_kernel(const double* __restrict__ Li, int64_t m,
                                                         int p, double T,
                                                         double* __restrict__ logdet,
                                                         double* __restrict__ aic,
                                                         double* __restrict__ bic) {
  __shared__ double part[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) s += log(Li[i * m + i]);
  s = wave_sum_d(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double ld = -2.0 * ((part[0] + part[1]) + (part[2] + part[3])) - (double)m * log(T);
    const double k = (double)p * (double)m * (double)m;
    logdet[p - 1] = ld;
    aic[p - 1] = ld + 2.0 * k / T;
    bic[p - 1] = ld + log(T) * k / T;
  }
}

// best[0] = argmin AIC + 1, best[1] = argmin BIC + 1 (lowest p on ties)
__global__ void lag_best_kernel(const double* __restrict__ aic, const double* __restrict__ bic,
                                int p_max, int32_t* __restrict__ best) {
  if (threadIdx.x != 0) return;
  int ba = 0, bb = 0;
  for (int q = 1; q < p_max; ++q) {
    if (aic[q] < aic[ba]) ba = q;
    if (bic[q] < bic[bb]) bb = q;
  }
  best[0] = ba + 1;
  best[1] = bb + 1;
}

size_t lag_ws_bytes(const VarPlan& v, void* base, LagWs* out) {
  Carver c(base);
  LagWs w;
  const size_t vb = var_ws_bytes(v, nullptr, nullptr);
  char* vbase = c.take<char>(vb);
  if (base) var_ws_bytes(v, vbase, &w.var);
  const int64_t m = v.m;
  w.Syy = c.take<double>(m * m);
  w.A = c.take<double>(m * m);
  w.Li = c.take<double>(m * m);
  w.chol = c.take<double>(chol_ws_doubles(m));
  if (out) *out = w;
  return c.used;
}

__global__ void lag_syy_kernel(const double* __restrict__ F, int64_t m, int64_t ldf,
                               double* __restrict__ Syy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  const int64_t i = e / m, j = e % m;
  Syy[e] = i >= j ? F[i * ldf + j] : F[j * ldf + i];
}

int run_lag_select(const VarPlan& v, const LagWs& w, const float* X, int64_t ldx, double* logdet,
                   double* aic, double* bic, int32_t* best, int32_t* st, hipStream_t stream) {
  const int64_t m = v.m, dz = v.dz, n_eff = v.n_eff;
  const VarWs& vw = w.var;
  int rc = var_normal_equations(v, vw, X, ldx, GramMode::kFp64, st, stream);
  if (rc) return rc;
  {
    ProfileScope ps("var_solve", stream);
    rc = chol_solve_lower(vw.G, dz, dz, vw.Tmp, m, m, nullptr, dz, vw.chol, st, stream);
    if (rc) return rc;
  }
  ProfileScope ps("lag_scores", stream);
  // T Sigma_0 = Yc^T Yc: the lag product F_0 of the normal equations (lag-0 columns centred by
  // their own means), its lower triangle mirrored
  lag_syy_kernel<<<(unsigned)ceil_div(m * m, 256), 256, 0, stream>>>(vw.F, m, m * (v.p + 1),
                                                                     w.Syy);
  VL_LAUNCH_CHECK();
  const double T = (double)n_eff;
  for (int p = 1; p <= v.p; ++p) {
    const double* Wp = vw.Tmp + (int64_t)(p - 1) * m * m;
    rc = gemm_f64(m, m, m, -1.0, Wp, m, true, Wp, m, false, 1.0, w.Syy, m, false, stream);
    if (rc) return rc;
    lag_copy_kernel<<<(unsigned)ceil_div(m * m, 256), 256, 0, stream>>>(w.Syy, w.A, m * m);
    VL_LAUNCH_CHECK();
    rc = chol_solve_lower(w.A, m, m, nullptr, 0, 0, w.Li, m, w.chol, st, stream);
    if (rc) return rc;
    lag_scores_kernel<<<1, 256, 0, stream>>>(w.Li, m, p, T, logdet, aic, bic);
    VL_LAUNCH_CHECK();
  }
  lag_best_kernel<<<1, 64, 0, stream>>>(aic, bic, v.p, best);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

}  // namespace vl
