// Lookup-only causal ordering (Alg. 1 main loop with Eq. 3) on gfx950.
//
// M_i = sum_{j in U, j != i} min(0, S[i][j])^2 over the candidates U.  Removing c from U lowers
// every M_i by min(0, S[i][c])^2 = max(0, S[c][i])^2 (S is antisymmetric), so after one O(m^2)
// initial pass each of the m steps costs O(m): an argmin (lowest index on exact ties) and an
// update that reads the contiguous row c of S.  The steps are sequential; one workgroup runs
// them all with M held in registers, so the only memory traffic per step is row c.
#include "order.hpp"
#include "profile.hpp"

#include <math.h>

namespace vl {

// M0[i] = sum_{j != i} min(0, S[i][j])^2, one wave per row, fixed summation order.
// A non-finite S entry raises VL_ERR_NONFINITE; its row's M becomes +inf so that every
// selection step still picks a valid index.
__global__ __launch_bounds__(256) void order_init_kernel(const double* __restrict__ S, int64_t m,
                                                         double* __restrict__ M0, int32_t* st) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= m) return;
  double s = 0.0;
  bool bad = false;
  for (int64_t j = lane; j < m; j += 64) {
    const double v = S[row * m + j];
    bad |= !isfinite(v);
    if (j != row && v < 0.0) s += v * v;
  }
  s = wave_sum_d(s);
  if (bad) raise_status(st, VL_ERR_NONFINITE);
  if (lane == 0) M0[row] = isfinite(s) ? s : INFINITY;
}

struct Best {
  double m1, m2;
  int i1;
};

__device__ inline Best combine(Best a, Best b) {
  const bool b_wins = b.m1 < a.m1 || (b.m1 == a.m1 && b.i1 < a.i1);
  Best r;
  if (b_wins) {
    r.m1 = b.m1;
    r.i1 = b.i1;
    r.m2 = fmin(a.m1, b.m2);
  } else {
    r.m1 = a.m1;
    r.i1 = a.i1;
    r.m2 = fmin(b.m1, a.m2);
  }
  return r;
}

template <int kThreads, int kPer>
__global__ __launch_bounds__(kThreads) void order_kernel(const double* __restrict__ S, int64_t m,
                                                         const double* __restrict__ M0,
                                                         int32_t* __restrict__ order,
                                                         double* __restrict__ margin) {
  constexpr int kWaves = kThreads / 64;
  __shared__ double sm1[kWaves], sm2[kWaves];
  __shared__ int si1[kWaves];
  __shared__ int s_c;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double inf = INFINITY;
  double Mv[kPer];
  bool alive[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int64_t i = tid + (int64_t)kThreads * r;
    alive[r] = i < m;
    Mv[r] = alive[r] ? M0[i] : inf;
  }
  for (int64_t k = 0; k < m; ++k) {
    Best b{inf, inf, 0x7fffffff};
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      if (alive[r]) b = combine(b, Best{Mv[r], inf, tid + kThreads * r});
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
      Best o;
      o.m1 = __shfl_xor(b.m1, s, 64);
      o.m2 = __shfl_xor(b.m2, s, 64);
      o.i1 = __shfl_xor(b.i1, s, 64);
      b = combine(b, o);
    }
    if (lane == 0) {
      sm1[wave] = b.m1;
      sm2[wave] = b.m2;
      si1[wave] = b.i1;
    }
    __syncthreads();
    if (tid == 0) {
      Best t{sm1[0], sm2[0], si1[0]};
      for (int w = 1; w < kWaves; ++w) t = combine(t, Best{sm1[w], sm2[w], si1[w]});
      s_c = t.i1;
      order[k] = t.i1;
      margin[k] = (t.m2 == inf) ? inf : t.m2 - t.m1;
    }
    __syncthreads();
    const int c = s_c;
    const double* row = S + (int64_t)c * m;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int64_t i = tid + (int64_t)kThreads * r;
      if (alive[r]) {
        if (i == c) {
          alive[r] = false;
        } else {
          const double v = row[i];
          if (v > 0.0 && v < INFINITY) Mv[r] -= v * v;
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Single-wave form for m <= 64 R.  Phase 0: all waves of the block form M0 (this reads every
// row of S once, which also brings S into this CU's L2 for the sequential phase).  Phase 1:
// wave 0 alone runs the m steps with M in registers (lane l owns variables l + 64 r) and wave-
// wide minima by DPP / permlane butterflies: no barriers inside the sequential loop.
// ------------------------------------------------------------------------------------------
template <int kCtrl>
__device__ inline double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, kCtrl, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(0, lo, kCtrl, 0xF, 0xF, false));
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
  v = min(v, __builtin_amdgcn_update_dpp(0, v, kDppRowMirror, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(0, v, kDppHalfMirror, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(0, v, kDppQuadXor2, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(0, v, kDppQuadXor1, 0xF, 0xF, false));
  v = min(v, partner16(v));
  v = min(v, partner32(v));
  return v;
}

template <int R, int kThreads>
__global__ __launch_bounds__(kThreads) void order_wave_kernel(const double* __restrict__ S, int64_t m,
                                                          int32_t* __restrict__ order,
                                                          double* __restrict__ margin,
                                                          int32_t* st) {
  __shared__ double M0s[64 * R];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bool bad = false;
  for (int64_t row = wave; row < m; row += kThreads / 64) {
    double s = 0.0;
    for (int64_t j = lane; j < m; j += 64) {
      const double v = S[row * m + j];
      bad |= !isfinite(v);
      if (j != row && v < 0.0) s += v * v;
    }
    s = wave_sum_d(s);
    if (lane == 0) M0s[row] = isfinite(s) ? s : INFINITY;
  }
  if (bad) raise_status(st, VL_ERR_NONFINITE);
  __syncthreads();
  if (wave != 0) return;

  // Removed and padding entries hold +inf: no per-entry flags in the loop.  Each step: m1 =
  // wave min; i1 = lowest index holding m1; the loads of row i1 are issued at once and the
  // second minimum (the margin) is reduced while they are in flight.
  const double inf = INFINITY;
  double Mv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + 64 * r;
    Mv[r] = i < m ? M0s[i] : inf;
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
    // row i1 of S (indices clamped into the matrix; padding entries stay +inf)
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
      if (lane + 64 * r == i1) Mv[r] = inf;
    double l2 = Mv[0];
#pragma unroll
    for (int r = 1; r < R; ++r) l2 = fmin(l2, Mv[r]);
    const double m2 = wave_min_f64(l2);
    if (lane == 0) {
      order[k] = i1;
      margin[k] = (m2 == inf) ? inf : m2 - m1;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double pos = v[r] > 0.0 && v[r] < inf ? v[r] : 0.0;
      Mv[r] -= pos * pos;            // +inf stays +inf
    }
  }
}

int run_order(const double* S, int64_t m, int32_t* order, double* margin, double* M0,
              int32_t* st, hipStream_t stream) {
  ProfileScope ps("order", stream);
  // 16 waves form M0 quickly; with 64 or more variables per lane the block is cut to 4 waves
  // so that the one sequential wave may hold them all in registers
#define VL_ORDER_WAVE(R) \
  order_wave_kernel<R, (R <= 16 ? 1024 : 256)><<<1, (R <= 16 ? 1024 : 256), 0, stream>>>( \
      S, m, order, margin, st)
  if (m <= 64) VL_ORDER_WAVE(1);
  else if (m <= 128) VL_ORDER_WAVE(2);
  else if (m <= 256) VL_ORDER_WAVE(4);
  else if (m <= 512) VL_ORDER_WAVE(8);
  else if (m <= 1024) VL_ORDER_WAVE(16);
  else if (m <= 2048) VL_ORDER_WAVE(32);
  else if (m <= 4096) VL_ORDER_WAVE(64);
  else {
    order_init_kernel<<<(unsigned)ceil_div(m, 4), 256, 0, stream>>>(S, m, M0, st);
    VL_LAUNCH_CHECK();
    order_kernel<1024, 16><<<1, 1024, 0, stream>>>(S, m, M0, order, margin);
  }
#undef VL_ORDER_WAVE
  VL_LAUNCH_CHECK();
  return VL_OK;
}

}  // namespace vl
