// Single-wave lookup-only ordering body (Alg. 1 main loop with Eq. 3), shared by the
// single-problem kernel and the batched kernels.
#pragma once
#include <math.h>

#include "common.hpp"

namespace vl {

// ------------------------------------------------------------------------------------------
// Single-wave form for m <= 64 R.  Phase 0: all waves of the block form M0 (this reads every
// row of S once, which also brings S into this CU's L2 for the sequential phase).  Phase 1:
// wave 0 alone runs the m steps with M in registers (lane l owns variables l + 64 r) and wave-
// wide minima by DPP / permlane butterflies: no barriers inside the sequential loop.
// ------------------------------------------------------------------------------------------
template <int kCtrl>
__device__ inline double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  // mov_dpp writes a fresh register (no zeroed "old" operand to set up); the mirror and quad
  // permutations used here give every lane a source lane, so bound_ctrl changes nothing
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, kCtrl, 0xF, 0xF, true),
                          __builtin_amdgcn_mov_dpp(lo, kCtrl, 0xF, 0xF, true));
}

template <class T>
__device__ inline T partner16(T v) {
  static_assert(sizeof(T) == 4, "32-bit");
  const unsigned u = __builtin_bit_cast(unsigned, v);
  auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  return __builtin_bit_cast(T, ((threadIdx.x >> 4) & 1) ? (unsigned)r[0] : (unsigned)r[1]);
}

template <class T>
__device__ inline T partner32(T v) {
  static_assert(sizeof(T) == 4, "32-bit");
  const unsigned u = __builtin_bit_cast(unsigned, v);
  auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  return __builtin_bit_cast(T, ((threadIdx.x >> 5) & 1) ? (unsigned)r[0] : (unsigned)r[1]);
}

__device__ inline double partner16_f64(double v) {
  return __hiloint2double(partner16(__double2hiint(v)), partner16(__double2loint(v)));
}
__device__ inline double partner32_f64(double v) {
  return __hiloint2double(partner32(__double2hiint(v)), partner32(__double2loint(v)));
}

// wave-wide minimum (every lane gets it); the lane pairings mirror-in-row, mirror-in-half-row,
// quad xor 2, quad xor 1, xor 16, xor 32 together cover all 64 lanes
__device__ inline double wave_min_f64(double v) {
  v = fmin(v, dpp_f64<kDppRowMirror>(v));
  v = fmin(v, dpp_f64<kDppHalfMirror>(v));
  v = fmin(v, dpp_f64<kDppQuadXor2>(v));
  v = fmin(v, dpp_f64<kDppQuadXor1>(v));
  v = fmin(v, partner16_f64(v));
  v = fmin(v, partner32_f64(v));
  return v;
}

__device__ inline int wave_min_i32(int v) {
  v = min(v, __builtin_amdgcn_mov_dpp(v, kDppRowMirror, 0xF, 0xF, true));
  v = min(v, __builtin_amdgcn_mov_dpp(v, kDppHalfMirror, 0xF, 0xF, true));
  v = min(v, __builtin_amdgcn_mov_dpp(v, kDppQuadXor2, 0xF, 0xF, true));
  v = min(v, __builtin_amdgcn_mov_dpp(v, kDppQuadXor1, 0xF, 0xF, true));
  v = min(v, partner16(v));
  v = min(v, partner32(v));
  return v;
}

template <int R, int kThreads>
__device__ inline void order_wave_block(const double* __restrict__ S, int64_t m,
                                        int32_t* __restrict__ order, double* __restrict__ margin,
                                        int32_t* st) {
  __shared__ double M0s[64 * R];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bool bad = false;
  // several rows per wave at once, every load of them issued before the sums (clamped
  // in-bounds addresses; the padding is skipped in the sums)
  constexpr int kRows = R <= 4 ? 4 : (R <= 8 ? 2 : 1);
  for (int64_t row0 = (int64_t)wave * kRows; row0 < m; row0 += (int64_t)(kThreads / 64) * kRows) {
    double v[kRows][R];
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      const int64_t row = row0 + q < m ? row0 + q : m - 1;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t j = lane + 64 * r;
        v[q][r] = S[row * m + (j < m ? j : m - 1)];
      }
    }
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      const int64_t row = row0 + q;
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t j = lane + 64 * r;
        const bool in = j < m && row < m;
        bad |= in && !isfinite(v[q][r]);
        if (in && j != row && v[q][r] < 0.0) s += v[q][r] * v[q][r];
      }
      s = wave_sum_d(s);
      if (lane == 0 && row < m) M0s[row] = isfinite(s) ? s : INFINITY;
    }
  }
  if (bad) raise_status(st, VL_ERR_NONFINITE);
  __syncthreads();
  if (wave == 0) {
  // Removed and padding entries hold NaN: fmin passes over NaN, and NaN equals nothing, so
  // they never win a minimum nor the index search even when every live M is +inf (a row of S
  // with a non-finite entry, which raised VL_ERR_NONFINITE).  Each step: m1 = wave min over
  // the live entries; i1 = lowest index holding m1; the loads of row i1 are issued at once
  // and the second minimum (the margin) is reduced while they are in flight.
  const double inf = INFINITY, gone = __builtin_nan("");
  double Mv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + 64 * r;
    Mv[r] = i < m ? M0s[i] : gone;
  }
  const int64_t last = m - 1;
  for (int64_t k = 0; k < m; ++k) {
    double lm = Mv[0];
#pragma unroll
    for (int r = 1; r < R; ++r) lm = fmin(lm, Mv[r]);
    const double m1 = wave_min_f64(lm);
    int li = 0x7fffffff;
#pragma unroll
    for (int r = R - 1; r >= 0; --r)
      if (Mv[r] == m1) li = lane + 64 * r;
    const int i1 = wave_min_i32(li);
    // row i1 of S (indices clamped into the matrix; padding entries stay NaN)
    const double* rowp = S + (int64_t)(i1 < m ? i1 : last) * m;
    double v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = lane + 64 * r;
      v[r] = rowp[i < m ? i : last];
    }
    // remove the winner, then the margin from the remaining minimum
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (lane + 64 * r == i1) Mv[r] = gone;
    double l2 = Mv[0];
#pragma unroll
    for (int r = 1; r < R; ++r) l2 = fmin(l2, Mv[r]);
    const double m2 = wave_min_f64(l2);    // NaN when no live entry is left
    if (lane == 0) {
      order[k] = i1;
      margin[k] = (m2 == inf || m2 != m2) ? inf : m2 - m1;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double pos = v[r] > 0.0 && v[r] < inf ? v[r] : 0.0;
      Mv[r] -= pos * pos;            // +inf stays +inf, NaN stays NaN
    }
  }
  }
  __syncthreads();
}

}  // namespace vl
