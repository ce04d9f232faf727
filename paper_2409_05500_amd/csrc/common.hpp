// Shared device/host helpers of the gfx950 VarLiNGAM library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "varlingam.h"

namespace vl {

constexpr int kWave = 64;

// ------------------------------------------------------------------------------------------
// Entropy-approximation constants (Hyvarinen 1998 maximum-entropy approximation with
// G1 = log cosh, G2 = u exp(-u^2/2); literal published values).
// ------------------------------------------------------------------------------------------
constexpr double kK1 = 79.047;
constexpr double kK2 = 7.4129;
constexpr double kGamma = 0.37457;
constexpr double kHGauss = 1.4189385332046727418;  // (1 + ln 2 pi) / 2
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kLog2e = 1.44269504088896340736;
// Sample values are pre-scaled, w = c u with c = sqrt(log2(e) / 2), so that
//   exp(-u^2/2) = exp2(-w^2)   and   exp(-2|u|) = exp2(kTScale |w|),  kTScale = -2 log2(e) / c.
constexpr double kWScale = 0.84932180028801904272;   // sqrt(log2(e)/2)
constexpr double kTScale = -3.39728720115207617089;  // -2 log2(e) / kWScale

// 1 - rho^2 below this is a degenerate (collinear) pair.
constexpr double kMinOneMinusRho2 = 1e-12;

// ------------------------------------------------------------------------------------------
// Device status word: the first error wins; VL_OK is written by a reset kernel per call.
// ------------------------------------------------------------------------------------------
__device__ inline void raise_status(int32_t* st, int code) {
  if (st) atomicCAS(reinterpret_cast<int*>(st), 0, code);
}

__global__ void reset_status_kernel(int32_t* st);

// ------------------------------------------------------------------------------------------
// Workspace carving: consecutive 256-byte aligned slices of the caller's buffer.  The same
// sequence of take() calls run with base == nullptr only measures the total.
// ------------------------------------------------------------------------------------------
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += bytes;
    return p;
  }
};

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Launch-error check used after every kernel launch by the host code.
#define VL_LAUNCH_CHECK()                               \
  do {                                                  \
    if (hipGetLastError() != hipSuccess) return VL_ERR_HIP; \
  } while (0)

// ------------------------------------------------------------------------------------------
// Wave-wide reductions (64 lanes) built on DPP row operations and the gfx950 permlane swaps.
// ------------------------------------------------------------------------------------------
template <class T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, kWave);
  return v;
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, kWave);
  return v;
}

// DPP control words (row = 16 lanes).
constexpr int kDppQuadXor1 = 0xB1;    // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;    // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane l of each 8-lane half-row reads lane 7 - l
constexpr int kDppRowMirror = 0x140;  // lane l of each 16-lane row reads lane 15 - l

template <int kCtrl>
__device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xF, 0xF, false));
}

// One butterfly reduce-scatter level on a pair of register arrays.  `upper` says whether
// this lane is the partner holding the second half; afterwards the lane keeps the half it
// owns, summed with its partner's copy.
template <int kCtrl>
__device__ inline float rs_level_dpp(float keep_lo, float keep_hi, bool upper) {
  float send = upper ? keep_lo : keep_hi;
  float keep = upper ? keep_hi : keep_lo;
  return keep + dpp_mov<kCtrl>(send);
}

// Reduce-scatter of 64 values held by every lane of a wave: on return lane l holds
// sum over all 64 lanes of v[l].  v is destroyed.  Lane pairing per level:
// 32 (permlane32 swap), 16 (permlane16 swap), 8 (row mirror), 4 (half-row mirror),
// 2 and 1 (quad permutes).  Every level pairs lanes that hold the same value set.
__device__ inline float wave_reduce_scatter64(float (&v)[64]) {
  const int lane = threadIdx.x & 63;
  // level 32: lanes < 32 keep v[0..31], lanes >= 32 keep v[32..63]
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[k]), __float_as_uint(v[k + 32]),
                                              false, false);
    v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  // level 16 on v[0..31]
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[k]), __float_as_uint(v[k + 16]),
                                              false, false);
    v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = rs_level_dpp<kDppRowMirror>(v[k], v[k + 8], b3);
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = rs_level_dpp<kDppHalfMirror>(v[k], v[k + 4], b2);
#pragma unroll
  for (int k = 0; k < 2; ++k) v[k] = rs_level_dpp<kDppQuadXor2>(v[k], v[k + 2], b1);
  v[0] = rs_level_dpp<kDppQuadXor1>(v[0], v[1], b0);
  return v[0];
}

// The FP64 form of wave_reduce_scatter64 (same levels and lane pairing; each double moves as
// its two 32-bit halves).
template <int kCtrl>
__device__ inline double dpp_mov_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int kCtrl>
__device__ inline double rs_level_dpp_d(double keep_lo, double keep_hi, bool upper) {
  const double send = upper ? keep_lo : keep_hi;
  const double keep = upper ? keep_hi : keep_lo;
  return keep + dpp_mov_d<kCtrl>(send);
}

// One permlane swap level on doubles: lanes of the lower group keep a (summed with the
// partner's a), lanes of the upper group keep b.
template <bool k32>
__device__ inline double swap_level_d(double a, double b) {
  const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
  const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
  auto swap = [](unsigned x, unsigned y) {
    if constexpr (k32)
      return __builtin_amdgcn_permlane32_swap(x, y, false, false);
    else
      return __builtin_amdgcn_permlane16_swap(x, y, false, false);
  };
  const auto lo = swap((unsigned)ua, (unsigned)ub);
  const auto hi = swap((unsigned)(ua >> 32), (unsigned)(ub >> 32));
  auto make = [](unsigned l, unsigned h) {
    return __longlong_as_double((long long)(((unsigned long long)h << 32) | l));
  };
  return make(lo[0], hi[0]) + make(lo[1], hi[1]);
}

__device__ inline double wave_reduce_scatter64_d(double (&v)[64]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < 32; ++k) v[k] = swap_level_d<true>(v[k], v[k + 32]);
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = swap_level_d<false>(v[k], v[k + 16]);
  const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = rs_level_dpp_d<kDppRowMirror>(v[k], v[k + 8], b3);
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = rs_level_dpp_d<kDppHalfMirror>(v[k], v[k + 4], b2);
#pragma unroll
  for (int k = 0; k < 2; ++k) v[k] = rs_level_dpp_d<kDppQuadXor2>(v[k], v[k + 2], b1);
  return rs_level_dpp_d<kDppQuadXor1>(v[0], v[1], b0);
}

// Reduce-scatter of 16 values held by every lane: on return lane l holds the sum over all 64
// lanes of v[l >> 2] (the four lanes of a quad hold the same sum).  v is destroyed.  Levels as
// in wave_reduce_scatter64 down to the half-row mirror (index bits 3..0 = lane bits 5..2); the
// lanes of a quad then hold the same index over complementary lane sets and are summed.
__device__ inline float wave_reduce_scatter16(float (&v)[16]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[k]), __float_as_uint(v[k + 8]),
                                              false, false);
    v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[k]), __float_as_uint(v[k + 4]),
                                              false, false);
    v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  const bool b3 = lane & 8, b2 = lane & 4;
#pragma unroll
  for (int k = 0; k < 2; ++k) v[k] = rs_level_dpp<kDppRowMirror>(v[k], v[k + 2], b3);
  float s = rs_level_dpp<kDppHalfMirror>(v[0], v[1], b2);
  s += dpp_mov<kDppQuadXor2>(s);
  s += dpp_mov<kDppQuadXor1>(s);
  return s;
}

// Exponent e with |v| < 2^e for every value of a set whose largest magnitude is mx (0 for mx = 0;
// a non-finite mx, which the callers' finiteness checks report, gives 0 as well).
__device__ __forceinline__ int32_t exponent_of(double mx) {
  int ex = 0;
  if (mx > 0.0 && mx < INFINITY) frexp(mx, &ex);
  return ex;
}

// v if keep, else +0.0, by masking the bits.  The mask is made opaque to the optimiser (an
// empty asm statement on the mask, which no load feeds): otherwise it proves the masked value
// dead and branches around the load that produces it, with a wait per load.
__device__ __attribute__((always_inline)) inline double mask_f64(double v, bool keep) {
  unsigned long long mk = 0ull - (unsigned long long)keep;
  asm volatile("" : "+v"(mk));
  return __longlong_as_double((long long)((unsigned long long)__double_as_longlong(v) & mk));
}

__device__ __attribute__((always_inline)) inline float mask_f32(float v, bool keep) {
  unsigned mk = 0u - (unsigned)keep;
  asm volatile("" : "+v"(mk));
  return __uint_as_float(__float_as_uint(v) & mk);
}

}  // namespace vl
