// Single-wave lookup-only ordering body (Alg. 1 main loop with Eq. 3), shared by the
// single-problem kernel and the batched kernels.
#pragma once
#include <math.h>

#include "common.hpp"

namespace vl {

// ------------------------------------------------------------------------------------------
// Single-wave form for m <= 64 R.  Phase 0: all waves of the block form M0 (this reads every
// row of S once, which also brings S into this CU's L2 for the sequential phase).  Phase 1:
// wave 0 alone runs the m steps with M in registers and wave-wide minima by DPP / permlane
// butterflies: no barriers inside the sequential loop.  The live set shrinks by one a step, so
// the loop runs in stages of R, R - 1, ..., 1 slots a lane (halving above 8): whenever the live
// entries fit in the next stage's slots they are packed into them through LDS, each slot
// carrying its variable's index.  The packing keeps the indices increasing in (slot, lane)
// order; ties are broken by the index itself, so the result does not depend on the layout.
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

// v_min_f64 as written.  fmin() compiles to the same instruction preceded by a v_max_f64 x, x
// per operand (quieting a signalling NaN), one more dependent operation per reduction level;
// the only NaNs here are the quiet ones that mark removed entries, which v_min_f64 passes over.
__device__ __forceinline__ double min_quiet(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

__device__ inline double wave_min_quiet(double v) {
  v = min_quiet(v, dpp_f64<kDppRowMirror>(v));
  v = min_quiet(v, dpp_f64<kDppHalfMirror>(v));
  v = min_quiet(v, dpp_f64<kDppQuadXor2>(v));
  v = min_quiet(v, dpp_f64<kDppQuadXor1>(v));
  v = min_quiet(v, partner16_f64(v));
  v = min_quiet(v, partner32_f64(v));
  return v;
}

// minimum over a lane's R slots (a tree: log2 R dependent steps)
template <int R>
__device__ __forceinline__ double slots_min(const double (&x)[R]) {
  double t[R];
#pragma unroll
  for (int r = 0; r < R; ++r) t[r] = x[r];
#pragma unroll
  for (int s = 1; s < R; s *= 2)
#pragma unroll
    for (int r = 0; r + s < R; r += 2 * s) t[r] = min_quiet(t[r], t[r + s]);
  return t[0];
}

// lowest index among a lane's slots holding key (2^31 - 1 when none)
template <int R>
__device__ __forceinline__ int slots_index_of(const double (&x)[R], const int (&vid)[R],
                                              double key) {
  int t[R];
#pragma unroll
  for (int r = 0; r < R; ++r) t[r] = x[r] == key ? vid[r] : 0x7fffffff;
#pragma unroll
  for (int s = 1; s < R; s *= 2)
#pragma unroll
    for (int r = 0; r + s < R; r += 2 * s) t[r] = min(t[r], t[r + s]);
  return t[0];
}

constexpr int order_next_slots(int R) { return R > 8 ? R / 2 : R - 1; }

// Steps k .. while more entries are live than the next stage holds, with R slots a lane
// (Mv[r], vid[r]: the lane's entries and their variable indices; removed and empty slots hold
// NaN).  Removed and padding entries hold NaN: the minimum passes over NaN, and NaN equals
// nothing, so they never win a minimum nor the index search even when every live M is +inf (a
// row of S with a non-finite entry, which raised VL_ERR_NONFINITE).  Each step: m1 = wave min
// over the live entries; i1 = lowest index holding m1; the loads of row i1 are issued at once
// and the second minimum (the margin) is reduced while they are in flight.  sM, sI: LDS for
// the packing (64 R entries each).
template <int R>
__device__ __forceinline__ void order_stage(const double* __restrict__ S, int64_t m,
                                            int32_t* __restrict__ order,
                                            double* __restrict__ margin, double* sM, int* sI,
                                            double (&Mv)[R], int (&vid)[R], int64_t k) {
  const int lane = threadIdx.x & 63;
  const double inf = INFINITY, gone = __builtin_nan("");
  const int64_t last = m - 1;
  constexpr int RN = order_next_slots(R);
  const int64_t kend = RN > 0 ? m - 64 * RN : m;   // m - k entries are live at step k
  for (; k < kend; ++k) {
    const double m1 = wave_min_quiet(slots_min<R>(Mv));
    const int i1 = wave_min_i32(slots_index_of<R>(Mv, vid, m1));
    // row i1 of S at this lane's variables (every vid is a valid column)
    const double* rowp = S + (int64_t)(i1 < m ? i1 : last) * m;
    double v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = rowp[vid[r]];
    // remove the winner, then the margin from the remaining minimum
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (vid[r] == i1) Mv[r] = gone;
    const double m2 = wave_min_quiet(slots_min<R>(Mv));    // NaN when no live entry is left
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
  if constexpr (RN > 0) {
    // pack the live entries into RN slots: position = live entries before this one in (slot,
    // lane) order, from one ballot per slot (the wave writes, then reads, its own LDS)
    int base = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool live = Mv[r] == Mv[r];
      const unsigned long long mk = __ballot(live);
      const int pos = base + __builtin_popcountll(mk & ((1ull << lane) - 1ull));
      if (live) {
        sM[pos] = Mv[r];
        sI[pos] = vid[r];
      }
      base += __builtin_popcountll(mk);
    }
    double Mn[RN];
    int vn[RN];
#pragma unroll
    for (int r = 0; r < RN; ++r) {
      const int p = lane + 64 * r;
      Mn[r] = p < base ? sM[p] : gone;
      vn[r] = p < base ? sI[p] : 0;
    }
    order_stage<RN>(S, m, order, margin, sM, sI, Mn, vn, k);
  }
}

template <int R, int kThreads>
__device__ inline void order_wave_block(const double* __restrict__ S, int64_t m,
                                        int32_t* __restrict__ order, double* __restrict__ margin,
                                        int32_t* st) {
  __shared__ double M0s[64 * R];   // M0, then the packing buffer of the sequential phase
  __shared__ int vidS[64 * R];
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
    const double gone = __builtin_nan("");
    double Mv[R];
    int vid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + 64 * r;
      Mv[r] = i < m ? M0s[i] : gone;
      vid[r] = i < m ? i : 0;
    }
    order_stage<R>(S, m, order, margin, M0s, vidS, Mv, vid, 0);
  }
  __syncthreads();
}

}  // namespace vl
