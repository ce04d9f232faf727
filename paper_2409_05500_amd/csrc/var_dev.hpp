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

template <class TOut>
__device__ inline void var_residual_tile_f64(
    const float* __restrict__ X, int64_t ldx, const int64_t* __restrict__ colmap,
    const double* __restrict__ mu, int64_t m, int p, int64_t n_eff,
    const double* __restrict__ Coef, TOut* __restrict__ E, int64_t lde, int64_t t0, int64_t j0) {
  __shared__ double Zs[16][64 + 1];
  __shared__ double Cs[16][64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
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

}  // namespace vl
