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
//   Low-precision Gram (BF16 mode): solve, then one refinement step Coef += G^{-1} Zc^T E64
//          with the residual E64 and its correlation with Zc formed in FP64.
#include "gram.hpp"
#include "linalg.hpp"
#include "var_fit.hpp"
#include "profile.hpp"

namespace vl {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// colmap[tau*m + i] = (p - tau) * ldx + i  for tau = 0..p  (tau = 0 is Y, tau >= 1 is Z)
__global__ void lag_colmap_kernel(int64_t m, int p, int64_t ldx, int64_t* __restrict__ colmap) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m * (p + 1)) return;
  const int64_t tau = c / m, i = c % m;
  colmap[c] = (p - tau) * ldx + i;
}

__global__ void fill_f64_kernel(double* __restrict__ a, int64_t n, double v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) a[e] = v;
}

__global__ void to_f32_kernel(const double* __restrict__ a, int64_t n, float* __restrict__ b) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = (float)a[e];
}

__global__ void add_f64_kernel(double* __restrict__ a, const double* __restrict__ d, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) a[e] += d[e];
}

// E[t][j] = (Y(t,j) - muY[j]) - sum_k (Z(t,k) - muZ[k]) CoefF[k][j]
// Block tile 64 (t) x 64 (j), 4 waves of 32 x 32, v_mfma_f32_32x32x2f32, k step 32 via LDS.
__global__ __launch_bounds__(256) void var_residual_kernel(
    const float* __restrict__ X, int64_t ldx, const int64_t* __restrict__ colmap,
    const double* __restrict__ mu, int64_t m, int p, int64_t n_eff,
    const float* __restrict__ CoefF, float* __restrict__ E, int64_t lde) {
  __shared__ float Zs[32][64 + 1];
  __shared__ float Cs[32][64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int64_t t0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  const int64_t dz = m * p;
  const int64_t* mapZ = colmap + m;
  const double* muZ = mu + m;
  f32x16 acc = {};
  for (int64_t k0 = 0; k0 < dz; k0 += 32) {
    {
      const int kk = tid & 31, tt = tid >> 5;
      const int64_t k = k0 + kk;
      const bool vk = k < dz;
      const int64_t off = vk ? mapZ[k] : 0;
      const float mz = vk ? (float)muZ[k] : 0.f;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t t = t0 + tt + 8 * r;
        Zs[kk][tt + 8 * r] = (vk && t < n_eff) ? X[off + t * ldx] - mz : 0.f;
      }
      const int jj = tid & 63, kr = tid >> 6;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t kq = k0 + kr + 4 * r, j = j0 + jj;
        Cs[kr + 4 * r][jj] = (kq < dz && j < m) ? CoefF[kq * m + j] : 0.f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 32; kk += 2) {
      const float a = Zs[kk + (lane >> 5)][wi * 32 + (lane & 31)];
      const float b = Cs[kk + (lane >> 5)][wj * 32 + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t t = t0 + wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int64_t j = j0 + wj * 32 + (lane & 31);
    if (t < n_eff && j < m) {
      const float y = X[colmap[j] + t * ldx] - (float)mu[j];
      E[t * lde + j] = y - acc[r];
    }
  }
}

// FP64 variant of the residual GEMM: v_mfma_f64_16x16x4f64 on the widened FP32 lags and the
// FP64 coefficients (exact products, FP64 sums); E is rounded to TOut once at the end (FP32
// for the output, FP64 for the refinement step's own residual).
// Block tile 64 (t) x 64 (j), wave tile 32 x 32 = 2 x 2 blocks of 16 x 16, k step 16.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <class TOut>
__global__ __launch_bounds__(256) void var_residual_f64_kernel(
    const float* __restrict__ X, int64_t ldx, const int64_t* __restrict__ colmap,
    const double* __restrict__ mu, int64_t m, int p, int64_t n_eff,
    const double* __restrict__ Coef, TOut* __restrict__ E, int64_t lde) {
  __shared__ double Zs[16][64 + 1];
  __shared__ double Cs[16][64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int64_t t0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  const int64_t dz = m * p;
  const int64_t* mapZ = colmap + m;
  const double* muZ = mu + m;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int lk = tid & 15, lt = tid >> 4;     // Z loader: 16 lags x 16 sample rows
  const int cj = tid & 63, ck = tid >> 6;     // Coef loader: 64 columns x 4 lag rows
  double rz[4], rcf[4];
  auto load = [&](int64_t k0) {
    const int64_t k = k0 + lk;
    const bool vk = k < dz;
    const int64_t off = vk ? mapZ[k] : 0;
    const double mz = vk ? muZ[k] : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t t = t0 + lt + 16 * r;
      rz[r] = (vk && t < n_eff) ? (double)X[off + t * ldx] - mz : 0.0;
      const int64_t kq = k0 + ck + 4 * r, j = j0 + cj;
      rcf[r] = (kq < dz && j < m) ? Coef[kq * m + j] : 0.0;
    }
  };
  load(0);
  for (int64_t k0 = 0; k0 < dz; k0 += 16) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Zs[lk][lt + 16 * r] = rz[r];
      Cs[ck + 4 * r][cj] = rcf[r];
    }
    __syncthreads();
    if (k0 + 16 < dz) load(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        av[q] = Zs[kk + (lane >> 4)][wi * 32 + q * 16 + (lane & 15)];
        bv[q] = Cs[kk + (lane >> 4)][wj * 32 + q * 16 + (lane & 15)];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t t = t0 + wi * 32 + a * 16 + (lane >> 4) + 4 * r;   // f64 D layout
        const int64_t j = j0 + wj * 32 + b * 16 + (lane & 15);
        if (t < n_eff && j < m) {
          const double y = (double)X[colmap[j] + t * ldx] - mu[j];
          E[t * lde + j] = (TOut)(y - acc[a][b][r]);
        }
      }
}

// M[(tau-1) m m + i m + k] = Coef[(tau-1) m + k][i]
__global__ void var_lag_matrices_kernel(const double* __restrict__ Coef, int64_t m, int p,
                                        double* __restrict__ M) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)p * m * m) return;
  const int64_t tau1 = e / (m * m), rem = e % (m * m), i = rem / m, k = rem % m;
  M[e] = Coef[(tau1 * m + k) * m + i];
}

// c[i] = muY[i] - sum_k' Coef[k'][i] muZ[k'], one wave per variable
__global__ __launch_bounds__(256) void var_intercept_kernel(const double* __restrict__ Coef,
                                                            const double* __restrict__ mu,
                                                            int64_t m, int64_t dz,
                                                            double* __restrict__ intercept) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= m) return;
  double s = 0.0;
  for (int64_t k = lane; k < dz; k += 64) s += Coef[k * m + i] * mu[m + k];
  s = wave_sum_d(s);
  if (lane == 0) intercept[i] = mu[i] - s;
}

VarPlan plan_var(int64_t n, int64_t m, int p) {
  VarPlan v;
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
  w.zeros = c.take<double>(v.m);
  w.G = c.take<double>(v.dz * v.dz);
  w.Coef = c.take<double>(v.dz * v.m);
  w.Rres = c.take<double>(v.dz * v.m);
  w.CoefF = c.take<float>(v.dz * v.m);
  w.L = c.take<double>(v.dz * v.dz);
  w.Tmp = c.take<double>(v.dz * v.m);
  w.chol = c.take<double>(chol_ws_doubles(v.dz));
  w.E64 = c.take<double>(v.n_eff * v.m);
  size_t s1 = (size_t)colmean_splits(v.n_eff) * nc;
  size_t s2 = (size_t)gram_splits(v.dz, v.dz, v.n_eff) * v.dz * v.dz;
  size_t s3 = (size_t)gram_splits(v.dz, v.m, v.n_eff) * v.dz * v.m;
  size_t s = s1 > s2 ? s1 : s2;
  s = s > s3 ? s : s3;
  w.scratch = c.take<double>(s);
  if (out) *out = w;
  return c.used;
}

static int var_residual(const VarPlan& v, const VarWs& w, const float* X, int64_t ldx, float* E,
                        int64_t lde, bool fp64, hipStream_t stream) {
  if (fp64) {
    dim3 grid((unsigned)ceil_div(v.m, 64), (unsigned)ceil_div(v.n_eff, 64));
    var_residual_f64_kernel<float><<<grid, 256, 0, stream>>>(X, ldx, w.colmap, w.mu, v.m, v.p,
                                                             v.n_eff, w.Coef, E, lde);
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

int run_var(const VarPlan& v, const VarWs& w, const float* X, int64_t ldx, int prec, double* M,
            double* intercept, float* E, int64_t lde, int32_t* st, hipStream_t stream) {
  const int64_t m = v.m, dz = v.dz, n_eff = v.n_eff;
  const int64_t nc = m * (v.p + 1);
  const bool plain = prec == VL_PREC_FP32;
  const bool refine = prec == VL_PREC_BF16;
  const GramMode gmode = plain ? GramMode::kFp32 : refine ? GramMode::kFp32Flush64 : GramMode::kFp64;
  const int64_t* mapZ = w.colmap + m;
  const double* muZ = w.mu + m;
  int rc;
  {
    ProfileScope ps("var_gram", stream);
    lag_colmap_kernel<<<(unsigned)ceil_div(nc, 256), 256, 0, stream>>>(m, v.p, ldx, w.colmap);
    VL_LAUNCH_CHECK();
    fill_f64_kernel<<<(unsigned)ceil_div(m, 256), 256, 0, stream>>>(w.zeros, m, 0.0);
    VL_LAUNCH_CHECK();
    rc = colmeans(X, ldx, w.colmap, nc, n_eff, w.mu, w.scratch, st, stream);
    if (rc) return rc;
    // G = Zc^T Zc, R = Zc^T Yc (R goes straight into Coef, solved in place)
    rc = gram_tn(X, ldx, mapZ, muZ, dz, X, ldx, mapZ, muZ, dz, n_eff, gmode, 1.0, w.G, dz,
                 w.scratch, stream);
    if (rc) return rc;
    rc = gram_tn(X, ldx, mapZ, muZ, dz, X, ldx, w.colmap, w.mu, m, n_eff, gmode, 1.0, w.Coef, m,
                 w.scratch, stream);
    if (rc) return rc;
  }
  {
    ProfileScope ps("var_solve", stream);
    rc = potrf_lower(w.G, dz, dz, w.L, dz, w.chol, st, stream);
    if (rc) return rc;
    rc = trsm_lower(w.L, dz, dz, w.chol, false, w.Coef, m, m, w.Tmp, m, stream);
    if (rc) return rc;
    rc = trsm_lower(w.L, dz, dz, w.chol, true, w.Tmp, m, m, w.Coef, m, stream);
    if (rc) return rc;
  }
  {
    ProfileScope ps("var_residual", stream);
    rc = var_residual(v, w, X, ldx, E, lde, !plain, stream);
    if (rc) return rc;
  }
  if (refine) {
    ProfileScope ps("var_refine", stream);
    // one refinement step: Coef += G^{-1} Zc^T E64 with the residual E64 = Yc - Zc Coef and
    // its correlation with Zc both formed in FP64 (exact products of the FP32 data), then E
    {
      dim3 grid((unsigned)ceil_div(m, 64), (unsigned)ceil_div(n_eff, 64));
      var_residual_f64_kernel<double><<<grid, 256, 0, stream>>>(X, ldx, w.colmap, w.mu, m, v.p,
                                                                n_eff, w.Coef, w.E64, m);
      VL_LAUNCH_CHECK();
    }
    rc = gram_tn_f64b(X, ldx, mapZ, muZ, dz, w.E64, m, m, n_eff, w.Rres, m, w.scratch, stream);
    if (rc) return rc;
    rc = trsm_lower(w.L, dz, dz, w.chol, false, w.Rres, m, m, w.Tmp, m, stream);
    if (rc) return rc;
    rc = trsm_lower(w.L, dz, dz, w.chol, true, w.Tmp, m, m, w.Rres, m, stream);
    if (rc) return rc;
    add_f64_kernel<<<(unsigned)ceil_div(dz * m, 256), 256, 0, stream>>>(w.Coef, w.Rres, dz * m);
    VL_LAUNCH_CHECK();
    rc = var_residual(v, w, X, ldx, E, lde, true, stream);
    if (rc) return rc;
  }
  var_lag_matrices_kernel<<<(unsigned)ceil_div(dz * m, 256), 256, 0, stream>>>(w.Coef, m, v.p, M);
  VL_LAUNCH_CHECK();
  var_intercept_kernel<<<(unsigned)ceil_div(m, 4), 256, 0, stream>>>(w.Coef, w.mu, m, dz,
                                                                    intercept);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

}  // namespace vl
