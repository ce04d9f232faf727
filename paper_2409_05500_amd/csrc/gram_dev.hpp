// Block-wide centred Gram tiles on gfx950 MFMA, shared by the single-problem kernels (split-K
// partials) and the batched kernels (one tile of one problem per block).
#pragma once
#include "common.hpp"

namespace vl {

// ------------------------------------------------------------------------------------------
// Centred TN Gram tile:  out[i * ldo + j] = scale * sum_{kb <= t < ke} (A(t,i) - muA[i])
// (with `mirror`, also out[j * ldo + i]: the other triangle of a symmetric result)
// (B(t,j) - muB[j]) for i in [i0, i0 + 64), j in [j0, j0 + 64), with A(t,i) = A[mapA[i] +
// t * lda].  Block tile 64 x 64 (4 waves of 32 x 32, one v_mfma_f32_32x32x2f32 accumulator
// each), 32 samples per LDS stage.  kFlush > 0 adds the FP32 accumulator into FP64 registers
// every kFlush stages (FP32-accurate result); kFlush == 0 keeps a plain FP32 accumulator.
// ------------------------------------------------------------------------------------------
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kGT = 64;    // tile side
constexpr int kGK = 32;    // samples per stage
constexpr int kGLd = 65;   // LDS row stride (floats): odd to keep the two half-waves apart

template <int kFlush>
__device__ inline void gram_tile_f32(
    const float* __restrict__ A, int64_t lda, const int64_t* __restrict__ mapA,
    const double* __restrict__ muA, int64_t M, const float* __restrict__ B, int64_t ldb,
    const int64_t* __restrict__ mapB, const double* __restrict__ muB, int64_t N, int64_t i0,
    int64_t j0, int64_t kb, int64_t ke, double* __restrict__ out, int64_t ldo, double scale,
    bool mirror = false) {
  __shared__ float As[kGK * kGLd];
  __shared__ float Bs[kGK * kGLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // loader: column cc, rows rg + 4 r
  const int cc = tid & 63, rg = tid >> 6;
  const int64_t ia = i0 + cc, jb = j0 + cc;
  const bool va = ia < M, vb = jb < N;
  const float* pa = A + (va ? (mapA ? mapA[ia] : ia) : 0);
  const float* pb = B + (vb ? (mapB ? mapB[jb] : jb) : 0);
  const float ma = va ? (float)muA[ia] : 0.f;
  const float mb = vb ? (float)muB[jb] : 0.f;
  // Centring with the float-rounded mean leaves an offset d ~ 1e-8 |mu|; it changes the Gram
  // by K d_a d_b only, since the centred columns sum to zero.

  const int wi = wave >> 1, wj = wave & 1;
  f32x16 acc = {};
  double acc64[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc64[r] = 0.0;

  // register prefetch of the next stage overlaps its loads with this stage's MFMAs: the raw
  // values are held, and centred and masked when they are stored to LDS (an operation on a
  // loaded value right after its load would wait for it before the MFMAs)
  float ra[kGK / 4], rb[kGK / 4];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < kGK / 4; ++r) {
      const int64_t t = k0 + rg + 4 * r;
      const int64_t tc = t < ke ? t : ke - 1;     // clamped, in bounds; padding masked below
      ra[r] = pa[tc * lda];
      rb[r] = pb[tc * ldb];
    }
  };
  load(kb);
  int stage = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += kGK, ++stage) {
#pragma unroll
    for (int r = 0; r < kGK / 4; ++r) {
      const bool in = k0 + rg + 4 * r < ke;
      As[(rg + 4 * r) * kGLd + cc] = mask_f32(ra[r] - ma, va && in);
      Bs[(rg + 4 * r) * kGLd + cc] = mask_f32(rb[r] - mb, vb && in);
    }
    __syncthreads();
    if (k0 + kGK < ke) load(k0 + kGK);
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 2) {
      const float a = As[(kk + (lane >> 5)) * kGLd + wi * 32 + (lane & 31)];
      const float b = Bs[(kk + (lane >> 5)) * kGLd + wj * 32 + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
    if (kFlush > 0 && (stage % kFlush) == kFlush - 1) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        acc64[r] += (double)acc[r];
        acc[r] = 0.f;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) acc64[r] += (double)acc[r];

  // D layout of 32x32x2: lane l, reg r -> row 8*(r/4) + 4*(l/32) + r%4, column l%32
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t i = i0 + wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int64_t j = j0 + wj * 32 + (lane & 31);
    if (i < M && j < N) {
      out[i * ldo + j] = scale * acc64[r];
      if (mirror) out[j * ldo + i] = scale * acc64[r];
    }
  }
}

// ------------------------------------------------------------------------------------------
// BF16 variant (the low-precision Gram that iterative refinement repairs): the centred FP32
// values staged in LDS are rounded to BF16 (nearest, ties to even) when read; the products of
// two BF16 values are exact in FP32; v_mfma_f32_32x32x8bf16_1k (lane l holds A[l % 32][4 (l /
// 32) + 0..3] and B[4 (l / 32) + 0..3][l % 32]; the output layout of the FP32 32x32 MFMA); FP32
// partial sums added into FP64 every 4 stages (128 samples).
// ------------------------------------------------------------------------------------------
typedef short s16x4 __attribute__((ext_vector_type(4)));

__device__ inline short to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ inline void gram_tile_bf16(
    const float* __restrict__ A, int64_t lda, const int64_t* __restrict__ mapA,
    const double* __restrict__ muA, int64_t M, const float* __restrict__ B, int64_t ldb,
    const int64_t* __restrict__ mapB, const double* __restrict__ muB, int64_t N, int64_t i0,
    int64_t j0, int64_t kb, int64_t ke, double* __restrict__ out, int64_t ldo, double scale) {
  __shared__ float As[kGK * kGLd];
  __shared__ float Bs[kGK * kGLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cc = tid & 63, rg = tid >> 6;
  const int64_t ia = i0 + cc, jb = j0 + cc;
  const bool va = ia < M, vb = jb < N;
  const float* pa = A + (va ? (mapA ? mapA[ia] : ia) : 0);
  const float* pb = B + (vb ? (mapB ? mapB[jb] : jb) : 0);
  const float ma = va ? (float)muA[ia] : 0.f;
  const float mb = vb ? (float)muB[jb] : 0.f;
  const int wi = wave >> 1, wj = wave & 1;
  f32x16 acc = {};
  double acc64[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc64[r] = 0.0;
  float ra[kGK / 4], rb[kGK / 4];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < kGK / 4; ++r) {
      const int64_t t = k0 + rg + 4 * r;
      const bool in = t < ke;
      const int64_t tc = in ? t : ke - 1;         // clamped, in bounds; padding masked below
      ra[r] = mask_f32(pa[tc * lda] - ma, va && in);
      rb[r] = mask_f32(pb[tc * ldb] - mb, vb && in);
    }
  };
  load(kb);
  int stage = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += kGK, ++stage) {
#pragma unroll
    for (int r = 0; r < kGK / 4; ++r) {
      As[(rg + 4 * r) * kGLd + cc] = ra[r];
      Bs[(rg + 4 * r) * kGLd + cc] = rb[r];
    }
    __syncthreads();
    if (k0 + kGK < ke) load(k0 + kGK);
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 8) {
      s16x4 a, b;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = kk + 4 * (lane >> 5) + q;
        a[q] = to_bf16(As[k * kGLd + wi * 32 + (lane & 31)]);
        b[q] = to_bf16(Bs[k * kGLd + wj * 32 + (lane & 31)]);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
    if ((stage & 3) == 3) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        acc64[r] += (double)acc[r];
        acc[r] = 0.f;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    acc64[r] += (double)acc[r];
    const int64_t i = i0 + wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int64_t j = j0 + wj * 32 + (lane & 31);
    if (i < M && j < N) out[i * ldo + j] = scale * acc64[r];
  }
}

// ------------------------------------------------------------------------------------------
// FP64 variant: same tiling, v_mfma_f64_16x16x4f64.  FP32 inputs are widened when read from
// LDS, so every product is exact and the sum is FP64 throughout.  Wave tile 32 x 32 = 2 x 2
// blocks of 16 x 16; 16 samples per LDS stage.
// ------------------------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kGK64 = 32;

__device__ inline void gram_tile_f64(
    const float* __restrict__ A, int64_t lda, const int64_t* __restrict__ mapA,
    const double* __restrict__ muA, int64_t M, const float* __restrict__ B, int64_t ldb,
    const int64_t* __restrict__ mapB, const double* __restrict__ muB, int64_t N, int64_t i0,
    int64_t j0, int64_t kb, int64_t ke, double* __restrict__ out, int64_t ldo, double scale,
    bool mirror = false) {
  __shared__ float As[kGK64 * kGLd];
  __shared__ float Bs[kGK64 * kGLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cc = tid & 63, rg = tid >> 6;
  const int64_t ia = i0 + cc, jb = j0 + cc;
  const bool va = ia < M, vb = jb < N;
  const float* pa = A + (va ? (mapA ? mapA[ia] : ia) : 0);
  const float* pb = B + (vb ? (mapB ? mapB[jb] : jb) : 0);
  const int wi = wave >> 1, wj = wave & 1;
  // 16 x 16 blocks wholly in the padding (edge tiles) are skipped (wave-uniform tests)
  const bool live_a[2] = {i0 + wi * 32 < M, i0 + wi * 32 + 16 < M};
  const bool live_b[2] = {j0 + wj * 32 < N, j0 + wj * 32 + 16 < N};
  // the means are subtracted after widening (in FP64), per operand column of this lane
  double mua[2], mub[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int64_t ii = i0 + wi * 32 + q * 16 + (lane & 15);
    const int64_t jj = j0 + wj * 32 + q * 16 + (lane & 15);
    mua[q] = ii < M ? muA[ii] : 0.0;
    mub[q] = jj < N ? muB[jj] : 0.0;
  }
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  float ra[kGK64 / 4], rb[kGK64 / 4];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < kGK64 / 4; ++r) {
      const int64_t t = k0 + rg + 4 * r;
      const bool in = t < ke;
      // a plain conditional load (no arithmetic on the value here, so no wait per load)
      ra[r] = (va && in) ? pa[t * lda] : 0.f;
      rb[r] = (vb && in) ? pb[t * ldb] : 0.f;
    }
  };
  load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kGK64) {
    // raw values; rows past the end of the split are zeroed again after centring below
#pragma unroll
    for (int r = 0; r < kGK64 / 4; ++r) {
      As[(rg + 4 * r) * kGLd + cc] = ra[r];
      Bs[(rg + 4 * r) * kGLd + cc] = rb[r];
    }
    __syncthreads();
    if (k0 + kGK64 < ke) load(k0 + kGK64);
#pragma unroll
    for (int kk = 0; kk < kGK64; kk += 4) {
      if (!(live_a[0] && live_b[0])) break;
      const bool in = k0 + kk + (lane >> 4) < ke;
      double av[2], bv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double ra = (double)As[(kk + (lane >> 4)) * kGLd + wi * 32 + q * 16 + (lane & 15)];
        const double rb = (double)Bs[(kk + (lane >> 4)) * kGLd + wj * 32 + q * 16 + (lane & 15)];
        av[q] = in ? ra - mua[q] : 0.0;
        bv[q] = in ? rb - mub[q] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          if (live_a[a] && live_b[b])
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of 16x16x4 f64: lane l, reg r -> row l/16 + 4 r, column l%16
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wi * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int64_t j = j0 + wj * 32 + b * 16 + (lane & 15);
        if (i < M && j < N) {
          out[i * ldo + j] = scale * acc[a][b][r];
          if (mirror) out[j * ldo + i] = scale * acc[a][b][r];
        }
      }
}

}  // namespace vl
