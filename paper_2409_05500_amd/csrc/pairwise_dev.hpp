// Device bodies of the pairwise-statistic precompute (Sec. 4.2 steps 1-2), shared by the
// single-problem kernels and the batched kernels.
#pragma once
#include <type_traits>

#include "common.hpp"

namespace vl {

// ------------------------------------------------------------------------------------------
// Stage 2a: standardise + transpose.  Block = 64 x 64 tile of E (t x i), staged through LDS.
// ------------------------------------------------------------------------------------------
// The blocks also clear zero[0 .. nzero) (the collinear-tile flags and list count of the
// pairwise precompute; nullptr for none), block `blk` of `nblk` taking a grid-stride share.
__device__ inline void standardize_tile(
    const float* __restrict__ E, int64_t lde, int64_t n_eff, int64_t m,
    const double* __restrict__ mu, const double* __restrict__ cov, float* __restrict__ Xs,
    int64_t n_pad, int64_t m_pad, int32_t* st, int64_t t0, int64_t i0,
    int32_t* __restrict__ zero = nullptr, int64_t nzero = 0, int64_t blk = 0, int64_t nblk = 1) {
  __shared__ float tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  if (zero)
    for (int64_t e = blk * blockDim.x + threadIdx.x; e < nzero; e += nblk * blockDim.x) zero[e] = 0;
  const int64_t i = i0 + tx;
  double mui = 0.0, inv = 0.0;
  if (i < m) {
    const double var = cov[i * m + i];
    if (!(var > 0.0)) raise_status(st, VL_ERR_DEGENERATE);
    mui = mu[i];
    inv = var > 0.0 ? 1.0 / sqrt(var) : 0.0;
  }
  for (int r = ty; r < 64; r += 4) {
    const int64_t t = t0 + r;
    float v = 0.f;
    if (i < m && t < n_eff) v = (float)(((double)E[t * lde + i] - mui) * inv);
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t iv = i0 + r, t = t0 + tx;
    if (iv < m_pad && t < n_pad) Xs[iv * n_pad + t] = tile[tx][r];  // rows >= m get zeros
  }
}

// ------------------------------------------------------------------------------------------
// Stage 2b: moments of the standardised columns -> Hx.  One NT-thread block per variable; accurate
// library exp/log (O(mn) work, not on the critical path).
// ------------------------------------------------------------------------------------------
template <int NT>
__device__ inline void hx_block(const float* __restrict__ Xs, int64_t n_pad, int64_t n_eff,
                                double* __restrict__ Hx, double* __restrict__ momx, int64_t i) {
  constexpr int kW = NT / 64;
  __shared__ double ra[kW], rb[kW];
  const float* x = Xs + i * n_pad;
  double sa = 0.0, sb = 0.0;
  auto term = [&](float u) {
    const float a = fabsf(u);
    sa += (double)(a + log1pf(expf(-2.f * a)) - (float)kLn2);
    sb += (double)(u * expf(-0.5f * u * u));
  };
  int64_t t = threadIdx.x;
  for (; t + 7 * NT < n_eff; t += 8 * NT) {  // eight loads in flight, summed in order
    float u[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) u[q] = x[t + q * NT];
#pragma unroll
    for (int q = 0; q < 8; ++q) term(u[q]);
  }
  for (; t < n_eff; t += NT) term(x[t]);
  sa = wave_sum_d(sa);
  sb = wave_sum_d(sb);
  if ((threadIdx.x & 63) == 0) {
    ra[threadIdx.x >> 6] = sa;
    rb[threadIdx.x >> 6] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double A = 0.0, B = 0.0;
#pragma unroll
    for (int w = 0; w < kW; ++w) {
      A += ra[w];
      B += rb[w];
    }
    A /= (double)n_eff;
    B /= (double)n_eff;
    Hx[i] = kHGauss - kK1 * (A - kGamma) * (A - kGamma) - kK2 * B * B;
    if (momx) {
      momx[2 * i] = A;
      momx[2 * i + 1] = B;
    }
  }
}

// ------------------------------------------------------------------------------------------
// Micro-tiles: kT x kT variable blocks {I, J} with bi <= bj, numbered row by row.
// ------------------------------------------------------------------------------------------
constexpr int kT = 4;

__device__ inline void tile_coords(int64_t k, int nt, int& bi, int& bj) {
  // upper-triangular tiles in row-major order: row r starts at r*nt - r*(r-1)/2
  const double T = (double)nt;
  const double disc = (2.0 * T + 1.0) * (2.0 * T + 1.0) - 8.0 * (double)k;
  int r = (int)(((2.0 * T + 1.0) - sqrt(disc > 0.0 ? disc : 0.0)) * 0.5);
  if (r < 0) r = 0;
  if (r > nt - 1) r = nt - 1;
  auto start = [nt](int q) { return (int64_t)q * nt - (int64_t)q * (q - 1) / 2; };
  while (r > 0 && start(r) > k) --r;
  while (r < nt - 1 && start(r + 1) <= k) ++r;
  bi = r;
  bj = r + (int)(k - start(r));
}

// A pair with sqrt(1 - rho^2) below kCollinearS is near-collinear: its Eq. 1 residual
// x_i - rho x_j cancels to a small fraction of the data, and forming it from the FP32 rounded
// standardised columns would amplify their rounding by 1 / sqrt(1 - rho^2).  The coefficient
// stage lists the micro-tiles that hold such a pair; after the FP32 moment kernel (which runs
// every tile) the collinear kernel recomputes their items, standardising and forming the
// residual in FP64 from E itself, and overwrites their partials.
// List layout (int32): flag[tiles] (1 = listed), then count, then the listed tile indices; the
// flags and the count are cleared by the standardisation stage.
constexpr double kCollinearS = 0.25;

__device__ inline void list_collinear_tile(int32_t* __restrict__ clist, int nt, int64_t tiles,
                                           int64_t i, int64_t j) {
  const int64_t a = (i < j ? i : j) / kT, b = (i < j ? j : i) / kT;
  const int64_t tile = a * nt - a * (a - 1) / 2 + (b - a);
  if (atomicExch(&clist[tile], 1) == 0) {
    const int k = atomicAdd(&clist[tiles], 1);
    clist[tiles + 1 + k] = (int32_t)tile;
  }
}

// ------------------------------------------------------------------------------------------
// Stage 3: scaled pair coefficients (a, b) for i, j < m_pad; zero on the diagonal / padding.
// A near-collinear pair lists its micro-tile in clist.
// ------------------------------------------------------------------------------------------
__device__ inline void pair_coef_elem(const double* __restrict__ cov, int64_t m, int64_t m_pad,
                                      float2* __restrict__ coef, int nt, int64_t tiles,
                                      int32_t* __restrict__ clist, int32_t* st, int64_t e) {
  if (e >= m_pad * m_pad) return;
  const int64_t i = e / m_pad, j = e % m_pad;
  float2 c = make_float2(0.f, 0.f);
  if (i < m && j < m && i != j) {
    const double vi = cov[i * m + i], vj = cov[j * m + j];
    const double rho = cov[i * m + j] / sqrt(vi * vj);
    const double omr = 1.0 - rho * rho;
    if (!(omr >= kCollinearS * kCollinearS)) list_collinear_tile(clist, nt, tiles, i, j);
    if (!(omr >= kMinOneMinusRho2)) {
      raise_status(st, VL_ERR_DEGENERATE);
    } else {
      const double s = sqrt(omr);
      c = make_float2((float)(kWScale / s), (float)(kWScale * rho / s));
    }
  }
  coef[e] = c;
}

// ------------------------------------------------------------------------------------------
// Stage 4: the pairwise-moment kernel.
//
// Work item = (micro-tile of kT x kT variables {I, J} with bi <= bj, sample chunk).  One wave
// per item; lanes run over samples (2 consecutive samples per lane per step, float2 loads of
// the variable-major Xs; pairs outermost within a step), the kT*kT pair coefficients are
// wave-uniform (scalar registers).
// Per pair, sample and direction (w = c u):
//     q = w*w;  e = exp2(-q)  (= exp(-u^2/2));        Bacc += w * e
//     t = exp2(kTScale * |w|) (= exp(-2|u|));         P    *= (1 + t)
//     Uacc += |w|
// log cosh u = |u| + ln(1 + exp(-2|u|)) - ln 2, so the logarithm is taken once per 64
// samples of a lane from the running product P (each factor lies in (1, 2], P <= 2^64):
//     Uacc += c ln2 (log2 P - count),  P = 1
// which leaves Uacc = c * sum log cosh u exactly in real arithmetic.  Zero-padded samples
// give w = 0, t = 1, factor 2: they add exactly 0 to Uacc and Bacc.
// Two transcendentals and seven other VALU operations per (pair, sample, direction); the
// compensated variant adds three per sum (Kahan), 13 in all.
//
// At the end the 2 x 2 x kT x kT wave sums are formed by a reduce-scatter (lane l ends with
// value l) and written to per-chunk FP32 partials part{U,B}[chunk][row][col].
// ------------------------------------------------------------------------------------------
static_assert(2 * 2 * kT * kT == 64, "reduce-scatter expects 64 values per lane");

__device__ __forceinline__ void moment_step(float w, float& U, float& P, float& B) {
  const float q = w * w;
  const float e = __builtin_amdgcn_exp2f(-q);
  B = fmaf(w, e, B);
  const float aw = fabsf(w);
  const float t = __builtin_amdgcn_exp2f(aw * (float)kTScale);
  P = fmaf(P, t, P);
  U += aw;
}

// Kahan accumulation s += x: the true sum is s - c.
__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
  const float y = x - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

// The moment accumulators of one (pair, direction), fed w = c u sample by sample: U sums |w|
// (and at each flush the log term of the running product P), B sums w e.  Plain FP32 sums
// (Comp = false), or Kahan-compensated ones (Comp = true): the compensation terms cU, cB keep
// a lane's sums within a few units of their last place whatever the sample count, where a
// plain running sum's rounding grows with it.
template <bool Comp>
struct MomentAcc;

template <>
struct MomentAcc<false> {
  float U, P, B;
  __device__ __forceinline__ void init() {
    U = 0.f;
    P = 1.f;
    B = 0.f;
  }
  __device__ __forceinline__ void step(float w) {
    const float q = w * w;
    const float e = __builtin_amdgcn_exp2f(-q);
    B = fmaf(w, e, B);
    const float aw = fabsf(w);
    const float t = __builtin_amdgcn_exp2f(aw * (float)kTScale);
    P = fmaf(P, t, P);
    U += aw;
  }
  __device__ __forceinline__ void flush(float cnt, float cln2) {
    U = fmaf(__builtin_amdgcn_logf(P) - cnt, cln2, U);
    P = 1.f;
  }
  __device__ __forceinline__ float u() const { return U; }
  __device__ __forceinline__ float b() const { return B; }
};

template <>
struct MomentAcc<true> {
  float U, cU, P, B, cB;
  __device__ __forceinline__ void init() {
    U = cU = B = cB = 0.f;
    P = 1.f;
  }
  __device__ __forceinline__ void step(float w) {
    const float q = w * w;
    const float e = __builtin_amdgcn_exp2f(-q);
    const float yb = fmaf(w, e, -cB);      // the product enters with one rounding
    const float tb = B + yb;
    cB = (tb - B) - yb;
    B = tb;
    const float aw = fabsf(w);
    const float t = __builtin_amdgcn_exp2f(aw * (float)kTScale);
    P = fmaf(P, t, P);
    kahan_add(U, cU, aw);
  }
  __device__ __forceinline__ void flush(float cnt, float cln2) {
    const float y = fmaf(__builtin_amdgcn_logf(P) - cnt, cln2, -cU);
    const float t = U + y;
    cU = (t - U) - y;
    U = t;
    P = 1.f;
  }
  __device__ __forceinline__ double u() const { return (double)U - (double)cU; }
  __device__ __forceinline__ double b() const { return (double)B - (double)cB; }
};

// Writes the 2 x 2 x kT x kT wave sums of one item: a reduce-scatter (lane l ends with value
// l), then the chunk partials part{U,B}[chunk][row][col] of the valid ordered pairs.  FP32
// partials take the plain sums (FP32 reduce-scatter); FP64 partials the compensated ones
// (each lane's exact value U - cU in FP64, FP64 reduce-scatter).
template <class TP, bool Comp>
__device__ __forceinline__ void write_moment_partials(MomentAcc<Comp> (&acc)[2][kT][kT],
                                                      int64_t i0, int64_t j0, int64_t m,
                                                      int64_t chunk, TP* __restrict__ partU,
                                                      TP* __restrict__ partB) {
  static_assert(std::is_same<TP, double>::value == Comp, "FP64 partials with compensation");
  const int lane = threadIdx.x & 63;
  // value index v = kind*32 + d*16 + ii*4 + jj (kind 0: U, 1: B)
  TP v[64];
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int ii = 0; ii < kT; ++ii)
#pragma unroll
      for (int jj = 0; jj < kT; ++jj) {
        v[d * 16 + ii * 4 + jj] = acc[d][ii][jj].u();
        v[32 + d * 16 + ii * 4 + jj] = acc[d][ii][jj].b();
      }
  TP sum;
  if constexpr (Comp)
    sum = wave_reduce_scatter64_d(v);
  else
    sum = wave_reduce_scatter64(v);
  const int kind = lane >> 5, d = (lane >> 4) & 1, ii = (lane >> 2) & 3, jj = lane & 3;
  const int64_t i = i0 + ii, j = j0 + jj;
  if (i < m && j < m && i != j) {
    const int64_t row = d ? j : i, col = d ? i : j;
    TP* dst = kind ? partB : partU;
    dst[chunk * m * m + row * m + col] = sum;
  }
}

// One wave's work item (tile, chunk); item < items is the caller's check.  Always inlined:
// as a call its register use rises from 168 to 248 and the occupancy falls to 2 waves/SIMD.
__device__ __attribute__((always_inline)) inline void pairwise_moments_item(
    const float* __restrict__ Xs, int64_t n_pad, const float2* __restrict__ coef, int64_t m_pad,
    int64_t m, int nt, int64_t tiles, int chunk_len, int64_t item,
    float* __restrict__ partU, float* __restrict__ partB) {
  const int lane = threadIdx.x & 63;
  const int64_t chunk = item / tiles;
  const int64_t tile = item - chunk * tiles;
  int bi, bj;
  tile_coords(tile, nt, bi, bj);
  const int64_t i0 = (int64_t)bi * kT, j0 = (int64_t)bj * kT;

  float ca[kT][kT], cb[kT][kT];
#pragma unroll
  for (int ii = 0; ii < kT; ++ii)
#pragma unroll
    for (int jj = 0; jj < kT; ++jj) {
      // read-only for this kernel: the constant address space lets these wave-uniform loads
      // be scalar loads into SGPRs whatever the pointer's provenance
      typedef const __attribute__((address_space(4))) float* const_f32p;
      const const_f32p cp = (const_f32p)(uintptr_t)coef;
      const int64_t ci = 2 * ((i0 + ii) * m_pad + j0 + jj);
      const float2 c = make_float2(cp[ci], cp[ci + 1]);
      ca[ii][jj] = c.x;
      cb[ii][jj] = c.y;
    }

  float U[2][kT][kT], P[2][kT][kT], B[2][kT][kT];
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int ii = 0; ii < kT; ++ii)
#pragma unroll
      for (int jj = 0; jj < kT; ++jj) {
        U[d][ii][jj] = 0.f;
        P[d][ii][jj] = 1.f;
        B[d][ii][jj] = 0.f;
      }

  // uniform row bases (scalar registers) and one 32-bit per-lane sample offset; 2 consecutive
  // samples per lane per step keep the live state at 168 VGPRs (3 waves per SIMD)
  const uint32_t tb = (uint32_t)(chunk * chunk_len) + 2u * (uint32_t)lane;
  const float* xi_r[kT];
  const float* xj_r[kT];
#pragma unroll
  for (int k = 0; k < kT; ++k) {
    xi_r[k] = Xs + (i0 + k) * n_pad;
    xj_r[k] = Xs + (j0 + k) * n_pad;
  }
  const float cln2 = (float)(kWScale * kLn2);
  const int steps = chunk_len / 128;                // 2 samples per lane per step
  int since_flush = 0;
  for (int s = 0; s < steps; ++s) {
    float2 xi[kT], xj[kT];
#pragma unroll
    for (int k = 0; k < kT; ++k) {
      const uint32_t o = tb + 128u * (uint32_t)s;
      xi[k] = *reinterpret_cast<const float2*>(xi_r[k] + o);
      xj[k] = *reinterpret_cast<const float2*>(xj_r[k] + o);
    }
#pragma unroll
    for (int ii = 0; ii < kT; ++ii) {
#pragma unroll
      for (int jj = 0; jj < kT; ++jj) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float xv = e ? xi[ii].y : xi[ii].x;
          const float yv = e ? xj[jj].y : xj[jj].x;
          const float w0 = fmaf(xv, ca[ii][jj], -(yv * cb[ii][jj]));
          const float w1 = fmaf(yv, ca[ii][jj], -(xv * cb[ii][jj]));
          moment_step(w0, U[0][ii][jj], P[0][ii][jj], B[0][ii][jj]);
          moment_step(w1, U[1][ii][jj], P[1][ii][jj], B[1][ii][jj]);
        }
      }
    }
    since_flush += 2;
    if (since_flush == 64 || s == steps - 1) {
      const float cnt = (float)since_flush;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int ii = 0; ii < kT; ++ii)
#pragma unroll
          for (int jj = 0; jj < kT; ++jj) {
            U[d][ii][jj] = fmaf(__builtin_amdgcn_logf(P[d][ii][jj]) - cnt, cln2, U[d][ii][jj]);
            P[d][ii][jj] = 1.f;
          }
      since_flush = 0;
    }
  }

  // value index v = kind*32 + d*16 + ii*4 + jj (kind 0: U, 1: B)
  float v[64];
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int ii = 0; ii < kT; ++ii)
#pragma unroll
      for (int jj = 0; jj < kT; ++jj) {
        v[d * 16 + ii * 4 + jj] = U[d][ii][jj];
        v[32 + d * 16 + ii * 4 + jj] = B[d][ii][jj];
      }
  const float sum = wave_reduce_scatter64(v);
  const int kind = lane >> 5, d = (lane >> 4) & 1, ii = (lane >> 2) & 3, jj = lane & 3;
  const int64_t i = i0 + ii, j = j0 + jj;
  if (i < m && j < m && i != j) {
    const int64_t row = d ? j : i, col = d ? i : j;
    float* dst = kind ? partB : partU;
    dst[chunk * m * m + row * m + col] = sum;
  }
}

// The same work item with Kahan-compensated sums and FP64 partials (231 VGPRs, 2 waves per
// SIMD).  A separate body: folding both forms into one template changed the schedule the
// compiler chose for the plain one (6% slower).
__device__ __attribute__((always_inline)) inline void pairwise_moments_item_comp(
    const float* __restrict__ Xs, int64_t n_pad, const float2* __restrict__ coef, int64_t m_pad,
    int64_t m, int nt, int64_t tiles, int chunk_len, int64_t item,
    double* __restrict__ partU, double* __restrict__ partB) {
  constexpr bool Comp = true;
  const int lane = threadIdx.x & 63;
  const int64_t chunk = item / tiles;
  const int64_t tile = item - chunk * tiles;
  int bi, bj;
  tile_coords(tile, nt, bi, bj);
  const int64_t i0 = (int64_t)bi * kT, j0 = (int64_t)bj * kT;

  float ca[kT][kT], cb[kT][kT];
#pragma unroll
  for (int ii = 0; ii < kT; ++ii)
#pragma unroll
    for (int jj = 0; jj < kT; ++jj) {
      // read-only for this kernel: the constant address space lets these wave-uniform loads
      // be scalar loads into SGPRs whatever the pointer's provenance
      typedef const __attribute__((address_space(4))) float* const_f32p;
      const const_f32p cp = (const_f32p)(uintptr_t)coef;
      const int64_t ci = 2 * ((i0 + ii) * m_pad + j0 + jj);
      const float2 c = make_float2(cp[ci], cp[ci + 1]);
      ca[ii][jj] = c.x;
      cb[ii][jj] = c.y;
    }

  MomentAcc<Comp> acc[2][kT][kT];
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int ii = 0; ii < kT; ++ii)
#pragma unroll
      for (int jj = 0; jj < kT; ++jj) acc[d][ii][jj].init();

  // uniform row bases (scalar registers) and one 32-bit per-lane sample offset; 2 consecutive
  // samples per lane per step keep the live state at 168 VGPRs (3 waves per SIMD)
  const uint32_t tb = (uint32_t)(chunk * chunk_len) + 2u * (uint32_t)lane;
  const float* xi_r[kT];
  const float* xj_r[kT];
#pragma unroll
  for (int k = 0; k < kT; ++k) {
    xi_r[k] = Xs + (i0 + k) * n_pad;
    xj_r[k] = Xs + (j0 + k) * n_pad;
  }
  const float cln2 = (float)(kWScale * kLn2);
  const int steps = chunk_len / 128;                // 2 samples per lane per step
  int since_flush = 0;
  for (int s = 0; s < steps; ++s) {
    float2 xi[kT], xj[kT];
#pragma unroll
    for (int k = 0; k < kT; ++k) {
      const uint32_t o = tb + 128u * (uint32_t)s;
      xi[k] = *reinterpret_cast<const float2*>(xi_r[k] + o);
      xj[k] = *reinterpret_cast<const float2*>(xj_r[k] + o);
    }
#pragma unroll
    for (int ii = 0; ii < kT; ++ii) {
#pragma unroll
      for (int jj = 0; jj < kT; ++jj) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float xv = e ? xi[ii].y : xi[ii].x;
          const float yv = e ? xj[jj].y : xj[jj].x;
          const float w0 = fmaf(xv, ca[ii][jj], -(yv * cb[ii][jj]));
          const float w1 = fmaf(yv, ca[ii][jj], -(xv * cb[ii][jj]));
          acc[0][ii][jj].step(w0);
          acc[1][ii][jj].step(w1);
        }
      }
    }
    since_flush += 2;
    if (since_flush == 64 || s == steps - 1) {
      const float cnt = (float)since_flush;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int ii = 0; ii < kT; ++ii)
#pragma unroll
          for (int jj = 0; jj < kT; ++jj) acc[d][ii][jj].flush(cnt, cln2);
      since_flush = 0;
    }
  }
  (void)lane;
  write_moment_partials(acc, i0, j0, m, chunk, partU, partB);
}

// The same item, (tile, chunk), for a listed micro-tile.  Lanes run over samples, one per step.  Each sample of the tile's 2 kT variables
// is standardised in FP64 from E (x = (e - mu) / sd, population moments), the residuals of
// both directions are formed in FP64, d = x_i - rho x_j, and only the scaled residual
// w = d c / sqrt(1 - rho^2) is rounded to FP32: its relative error is then that of one
// rounding, as for a well-conditioned pair.  The moment terms are the fast item's.
template <class TP>
__device__ inline void pairwise_collinear_item(
    const float* __restrict__ E, int64_t lde, int64_t n_eff, const double* __restrict__ mu,
    const double* __restrict__ cov, int64_t m, int nt, int chunk_len, int64_t tile,
    int64_t chunk, TP* __restrict__ partU, TP* __restrict__ partB) {
  constexpr bool Comp = std::is_same<TP, double>::value;
  const int lane = threadIdx.x & 63;
  int bi, bj;
  tile_coords(tile, nt, bi, bj);
  const int64_t i0 = (int64_t)bi * kT, j0 = (int64_t)bj * kT;
  double mi[kT], si[kT], mj[kT], sj[kT];
  int64_t ci[kT], cj[kT];
#pragma unroll
  for (int k = 0; k < kT; ++k) {
    const bool oi = i0 + k < m, oj = j0 + k < m;
    ci[k] = oi ? i0 + k : m - 1;
    cj[k] = oj ? j0 + k : m - 1;
    mi[k] = mu[ci[k]];
    mj[k] = mu[cj[k]];
    si[k] = oi ? 1.0 / sqrt(cov[ci[k] * m + ci[k]]) : 0.0;   // padding variables: x = 0
    sj[k] = oj ? 1.0 / sqrt(cov[cj[k] * m + cj[k]]) : 0.0;
  }
  double rho[kT][kT], kc[kT][kT];
#pragma unroll
  for (int ii = 0; ii < kT; ++ii)
#pragma unroll
    for (int jj = 0; jj < kT; ++jj) {
      const int64_t i = i0 + ii, j = j0 + jj;
      rho[ii][jj] = 0.0;
      kc[ii][jj] = 0.0;
      if (i < m && j < m && i != j) {
        const double r = cov[i * m + j] / sqrt(cov[i * m + i] * cov[j * m + j]);
        const double omr = 1.0 - r * r;
        rho[ii][jj] = r;
        kc[ii][jj] = omr >= kMinOneMinusRho2 ? kWScale / sqrt(omr) : 0.0;  // else: raised
      }
    }

  MomentAcc<Comp> acc[2][kT][kT];
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int ii = 0; ii < kT; ++ii)
#pragma unroll
      for (int jj = 0; jj < kT; ++jj) acc[d][ii][jj].init();
  const float cln2 = (float)(kWScale * kLn2);
  const int steps = chunk_len / 64;
  int since_flush = 0;
  for (int s = 0; s < steps; ++s) {
    const int64_t t = chunk * chunk_len + (int64_t)s * 64 + lane;
    const bool ot = t < n_eff;
    const int64_t tc = ot ? t : n_eff - 1;           // clamped row; padding samples give 0
    double xi[kT], xj[kT];
#pragma unroll
    for (int k = 0; k < kT; ++k) {
      xi[k] = mask_f64(((double)E[tc * lde + ci[k]] - mi[k]) * si[k], ot);
      xj[k] = mask_f64(((double)E[tc * lde + cj[k]] - mj[k]) * sj[k], ot);
    }
#pragma unroll
    for (int ii = 0; ii < kT; ++ii)
#pragma unroll
      for (int jj = 0; jj < kT; ++jj) {
        const float w0 = (float)(fma(-rho[ii][jj], xj[jj], xi[ii]) * kc[ii][jj]);
        const float w1 = (float)(fma(-rho[ii][jj], xi[ii], xj[jj]) * kc[ii][jj]);
        acc[0][ii][jj].step(w0);
        acc[1][ii][jj].step(w1);
      }
    since_flush += 1;
    if (since_flush == 64 || s == steps - 1) {
      const float cnt = (float)since_flush;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int ii = 0; ii < kT; ++ii)
#pragma unroll
          for (int jj = 0; jj < kT; ++jj) acc[d][ii][jj].flush(cnt, cln2);
      since_flush = 0;
    }
  }
  write_moment_partials(acc, i0, j0, m, chunk, partU, partB);
}

// ------------------------------------------------------------------------------------------
// Stage 5: FP64 combine.  Hr[i][j] from the chunk partials (fixed order), then S.
// ------------------------------------------------------------------------------------------
template <class TP>
__device__ inline void combine_hr_elem(const TP* __restrict__ partU,
                                       const TP* __restrict__ partB, int nc, int64_t m,
                                       int64_t n_eff, double* __restrict__ Hr,
                                       double* __restrict__ mom, int64_t e) {
  if (e >= m * m) return;
  const int64_t i = e / m, j = e % m;
  if (i == j) {
    Hr[e] = 0.0;
    if (mom) mom[2 * e] = mom[2 * e + 1] = 0.0;
    return;
  }
  double su = 0.0, sb = 0.0;
  for (int c = 0; c < nc; ++c) {
    su += (double)partU[(int64_t)c * m * m + e];
    sb += (double)partB[(int64_t)c * m * m + e];
  }
  const double A = su / (kWScale * (double)n_eff);
  const double B = sb / (kWScale * (double)n_eff);
  Hr[e] = kHGauss - kK1 * (A - kGamma) * (A - kGamma) - kK2 * B * B;
  if (mom) {
    mom[2 * e] = A;
    mom[2 * e + 1] = B;
  }
}

__device__ inline void score_elem(const double* __restrict__ Hx, const double* __restrict__ Hr,
                                  int64_t m, double* __restrict__ S, int64_t e) {
  if (e >= m * m) return;
  const int64_t i = e / m, j = e % m;
  // the same two sums in both orders -> S[j][i] == -S[i][j] bit for bit
  S[e] = i == j ? 0.0 : (Hx[j] + Hr[i * m + j]) - (Hx[i] + Hr[j * m + i]);
}

}  // namespace vl
