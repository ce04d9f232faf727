// Residual GEMM tiles of the VAR fit, shared by the single-problem and batched kernels.
// Y = x(t) and Z = [x(t-1), ..., x(t-p)] are read through the column map of the lagged views
// (colmap[tau m + i] = offset of x_i(t - tau) at t = 0), centred by mu (same layout).
#pragma once
#include "common.hpp"

namespace vl {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// E[t][j] = (Y(t,j) - muY[j]) - sum_k (Z(t,k) - muZ[k]) CoefF[k][j]
// Block tile 64 (t) x 64 (j), 4 waves of 32 x 32, v_mfma_f32_32x32x2f32, k step 32 via LDS.
__device__ inline void var_residual_tile_f32(
    const float* __restrict__ X, int64_t ldx, const int64_t* __restrict__ colmap,
    const double* __restrict__ mu, int64_t m, int p, int64_t n_eff,
    const float* __restrict__ CoefF, float* __restrict__ E, int64_t lde, int64_t t0,
    int64_t j0) {
  __shared__ float Zs[32][64 + 1];
  __shared__ float Cs[32][64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int64_t dz = m * p;
  const int64_t* mapZ = colmap + m;
  const double* muZ = mu + m;
  f32x16 acc = {};
  // the output column's offset and mean, read before the products
  const int64_t jo = j0 + wj * 32 + (lane & 31);
  const int64_t offy = colmap[jo < m ? jo : 0];
  const float muy = (float)mu[jo < m ? jo : 0];
  for (int64_t k0 = 0; k0 < dz; k0 += 32) {
    {
      const int kk = tid & 31, tt = tid >> 5;
      const int64_t k = k0 + kk;
      const bool vk = k < dz;
      // clamped in-bounds addresses, padding masked after the loads (no branch per load)
      const int64_t off = mapZ[vk ? k : dz - 1];
      const float mz = vk ? (float)muZ[k] : 0.f;
      float xv[8], cv[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t t = t0 + tt + 8 * r;
        xv[r] = X[off + (t < n_eff ? t : n_eff - 1) * ldx];
      }
      const int jj = tid & 63, kr = tid >> 6;
      const int64_t jc = j0 + jj < m ? j0 + jj : m - 1;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t kq = k0 + kr + 4 * r;
        cv[r] = CoefF[(kq < dz ? kq : dz - 1) * m + jc];
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t t = t0 + tt + 8 * r;
        Zs[kk][tt + 8 * r] = mask_f32(xv[r] - mz, vk && t < n_eff);
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t kq = k0 + kr + 4 * r;
        Cs[kr + 4 * r][jj] = mask_f32(cv[r], kq < dz && j0 + jj < m);
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
  // Y at this lane's outputs: every load issued before the first store (clamped addresses;
  // a load under each store's bounds test would wait for each in turn)
  float yin[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t t = t0 + wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    yin[r] = X[offy + (t < n_eff ? t : n_eff - 1) * ldx];
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t t = t0 + wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (t < n_eff && jo < m) E[t * lde + jo] = (yin[r] - muy) - acc[r];
  }
}

// FP64 variant of the residual GEMM: v_mfma_f64_16x16x4f64 on the widened FP32 lags and the
// FP64 coefficients (exact products, FP64 sums); E is rounded to TOut once at the end (FP32
// for the output, FP64 for the refinement step's own residual).
// Block tile 64 (t) x 64 (j), wave tile 32 x 32 = 2 x 2 blocks of 16 x 16, k step 16.

template <class TOut>
__device__ inline void var_residual_tile_f64(
    const float* __restrict__ X, int64_t ldx, const int64_t* __restrict__ colmap,
    const double* __restrict__ mu, int64_t m, int p, int64_t n_eff,
    const double* __restrict__ Coef, TOut* __restrict__ E, int64_t lde, int64_t t0, int64_t j0) {
  __shared__ double Zs[16][64 + 1];
  __shared__ double Cs[16][64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const bool live_a[2] = {t0 + wi * 32 < n_eff, t0 + wi * 32 + 16 < n_eff};
  const bool live_b[2] = {j0 + wj * 32 < m, j0 + wj * 32 + 16 < m};
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
    const int64_t off = mapZ[vk ? k : dz - 1];
    const double mz = vk ? muZ[k] : 0.0;
    const int64_t j = j0 + cj, jc = j < m ? j : m - 1;
    float xv[4];
    double cv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t t = t0 + lt + 16 * r, kq = k0 + ck + 4 * r;
      xv[r] = X[off + (t < n_eff ? t : n_eff - 1) * ldx];
      cv[r] = Coef[(kq < dz ? kq : dz - 1) * m + jc];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t t = t0 + lt + 16 * r, kq = k0 + ck + 4 * r;
      rz[r] = mask_f64((double)xv[r] - mz, vk && t < n_eff);
      rcf[r] = mask_f64(cv[r], kq < dz && j < m);
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
          if (live_a[a] && live_b[b])   // 16 x 16 blocks wholly in the padding are skipped
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

// ------------------------------------------------------------------------------------------
// FP64 residual tile: RT samples x 64 variables per workgroup; wave (wi, wj) of the 2 x 2 waves
// owns RT/2 x 32 = RT/32 x 2 blocks of v_mfma_f64_16x16x4f64.  Stages of RK lags through LDS
// (the centred lag values widened to FP64 once, at load); the next stage's global loads are in
// flight during the products.  Every output element sums its products in lag order four at a
// time whatever RT and RK, so all shapes give the same bits, and the same as
// var_residual_tile_f64.
// ------------------------------------------------------------------------------------------
constexpr int kRJ = 64;        // variables per tile

template <class TOut, int RT, int RK>
__device__ inline void var_residual_tile_f64w(
    const float* __restrict__ X, int64_t ldx, const int64_t* __restrict__ colmap,
    const double* __restrict__ mu, int64_t m, int p, int64_t n_eff,
    const double* __restrict__ Coef, TOut* __restrict__ E, int64_t lde, int64_t t0, int64_t j0) {
  constexpr int XB = RT / 32;                  // 16-row blocks per wave
  __shared__ double Zs[RK][RT + 1];
  __shared__ double Cs[RK][kRJ + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1, li = lane & 15, lk = lane >> 4;
  const int64_t dz = m * p;
  const int64_t* mapZ = colmap + m;
  const double* muZ = mu + m;
  f64x4 acc[XB][2];
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
  constexpr int kZRows = 256 / RK;             // Z loader: RK lags x kZRows sample rows a pass
  constexpr int kZPass = RT / kZRows;
  const int zk = tid % RK, zt = tid / RK;
  const int cj = tid & 63, ck = tid >> 6;      // Coef loader: 64 variables x 4 lags per pass
  double rz[kZPass], rc[RK / 4];
  // Every load reads a clamped in-bounds address and the padding is selected afterwards, so
  // the loads of a stage issue back to back (no branch, no wait per load).
  const int64_t jc = j0 + cj < m ? j0 + cj : m - 1;
  const bool vj = j0 + cj < m;
  auto load = [&](int64_t k0) {
    const int64_t k = k0 + zk;
    const bool vk = k < dz;
    const int64_t off = mapZ[vk ? k : dz - 1];
    const double mz = vk ? muZ[k] : 0.0;
    float xv[kZPass];
#pragma unroll
    for (int u = 0; u < kZPass; ++u) {
      const int64_t t = t0 + zt + kZRows * u;
      xv[u] = X[off + (t < n_eff ? t : n_eff - 1) * ldx];
    }
#pragma unroll
    for (int u = 0; u < RK / 4; ++u) {
      const int64_t kq = k0 + ck + 4 * u;
      const double cv = Coef[(kq < dz ? kq : dz - 1) * m + jc];
      rc[u] = mask_f64(cv, kq < dz && vj);
    }
#pragma unroll
    for (int u = 0; u < kZPass; ++u) {
      const int64_t t = t0 + zt + kZRows * u;
      rz[u] = mask_f64((double)xv[u] - mz, vk && t < n_eff);
    }
  };
  load(0);
  for (int64_t k0 = 0; k0 < dz; k0 += RK) {
#pragma unroll
    for (int u = 0; u < kZPass; ++u) Zs[zk][zt + kZRows * u] = rz[u];
#pragma unroll
    for (int u = 0; u < RK / 4; ++u) Cs[ck + 4 * u][cj] = rc[u];
    __syncthreads();
    if (k0 + RK < dz) load(k0 + RK);
#pragma unroll
    for (int kk = 0; kk < RK; kk += 4) {
      double a[XB], b[2];
#pragma unroll
      for (int x = 0; x < XB; ++x) a[x] = Zs[kk + lk][wi * (RT / 2) + x * 16 + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) b[y] = Cs[kk + lk][wj * 32 + y * 16 + li];
#pragma unroll
      for (int x = 0; x < XB; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
  // Y at this lane's outputs: every load issued before the first store (clamped addresses)
  float yin[XB][2][4];
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    const int64_t j = j0 + wj * 32 + y * 16 + li;
    const int64_t offy = colmap[j < m ? j : 0];
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t t = t0 + wi * (RT / 2) + x * 16 + lk + 4 * r;     // f64 D layout
        yin[x][y][r] = X[offy + (t < n_eff ? t : n_eff - 1) * ldx];
      }
  }
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    const int64_t j = j0 + wj * 32 + y * 16 + li;
    const double muy = mu[j < m ? j : 0];
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t t = t0 + wi * (RT / 2) + x * 16 + lk + 4 * r;
        if (t < n_eff && j < m) E[t * lde + j] = (TOut)(((double)yin[x][y][r] - muy) - acc[x][y][r]);
      }
  }
}

}  // namespace vl
