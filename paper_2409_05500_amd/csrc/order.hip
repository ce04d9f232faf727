// Lookup-only causal ordering (Alg. 1 main loop with Eq. 3) on gfx950.
//
// M_i = sum_{j in U, j != i} min(0, S[i][j])^2 over the candidates U.  Removing c from U lowers
// every M_i by min(0, S[i][c])^2 = max(0, S[c][i])^2 (S is antisymmetric), so after one O(m^2)
// initial pass each of the m steps costs O(m): an argmin (lowest index on exact ties) and an
// update that reads the contiguous row c of S.  The steps are sequential; one workgroup runs
// them all with M held in registers, so the only memory traffic per step is row c.
#include "order.hpp"
#include "order_dev.hpp"
#include "profile.hpp"

#include <math.h>

namespace vl {

// M0[i] = sum_{j != i} min(0, S[i][j])^2, one wave per row, fixed summation order.
// A non-finite S entry raises VL_ERR_NONFINITE and its row's M becomes +inf; the selection
// keeps an explicit live mask, so every step still picks a variable not yet ordered.
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

template <int R, int kThreads>
__global__ __launch_bounds__(kThreads) void order_wave_kernel(const double* __restrict__ S, int64_t m,
                                                          int32_t* __restrict__ order,
                                                          double* __restrict__ margin,
                                                          int32_t* st) {
  order_wave_block<R, kThreads>(S, m, order, margin, st);
}

int run_order(const double* S, int64_t m, int32_t* order, double* margin, double* M0,
              int32_t* st, hipStream_t stream) {
  ProfileScope ps("order", stream);
  // 16 waves form M0 quickly; with more variables per lane the block is cut to 8 or 4 waves
  // so that the one sequential wave may hold them all in registers
#define VL_ORDER_WAVE(R) \
  order_wave_kernel<R, (R <= 8 ? 1024 : (R <= 16 ? 512 : 256))> \
      <<<1, (R <= 8 ? 1024 : (R <= 16 ? 512 : 256)), 0, stream>>>( \
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
