// Certified ordering: Alg. 1 (with Eq. 3) on the FP32-moment score matrix, where every step
// whose decision the scores' error bound cannot settle is re-decided on scores recomputed in
// FP64.
//
// With |S_ij - S*_ij| <= eps_ij (S* the exact scores), M_i = sum_{j in U} min(0, S_ij)^2
// differs from M*_i by at most
//     EM_i = sum_{j in U, S_ij < eps_ij} eps_ij (2 |min(0, S_ij)| + eps_ij).
// The pick c = argmin M is certainly within `tie` of the exact minimum when
//     M_c + EM_c - (M_i - EM_i) <= tie   for every other candidate i.
// A step where that fails lists c and every i that breaks it.  Those variables' rows (and so
// their columns) of S are recomputed in FP64 from E: standardised in FP64, rho_ij = mean(x_i
// x_j), both Eq. 1 residuals, the Eq. 2 moments and H in FP64; their entries then have
// eps = 0.  The ordering is rerun until no step is in doubt.  Each round refines at least one
// new row (a step in doubt always has an unrefined candidate: among refined rows the bound is
// exact), so it ends after at most m rounds; one or two are typical.
#include <math.h>

#include <vector>

#include "certify.hpp"
#include "order_dev.hpp"
#include "profile.hpp"

namespace vl {

// ------------------------------------------------------------------------------------------
// FP64 column statistics and the variable-major standardised copy X64[i][t] (m x n_eff).
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void cert_colstats_kernel(const float* __restrict__ E,
                                                            int64_t lde, int64_t n_eff,
                                                            int64_t m, double* __restrict__ mu,
                                                            double* __restrict__ inv_sd,
                                                            int32_t* st) {
  const int64_t i = blockIdx.x;
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < n_eff; t += 256) s += (double)E[t * lde + i];
  s = wave_sum_d(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double mean = ((red[0] + red[1]) + red[2] + red[3]) / (double)n_eff;
  __syncthreads();
  double v = 0.0;
  for (int64_t t = threadIdx.x; t < n_eff; t += 256) {
    const double d = (double)E[t * lde + i] - mean;
    v += d * d;
  }
  v = wave_sum_d(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double var = ((red[0] + red[1]) + red[2] + red[3]) / (double)n_eff;
    if (!(var > 0.0)) raise_status(st, VL_ERR_DEGENERATE);
    mu[i] = mean;
    inv_sd[i] = var > 0.0 ? 1.0 / sqrt(var) : 0.0;
  }
}

__global__ __launch_bounds__(256) void cert_standardize_kernel(
    const float* __restrict__ E, int64_t lde, int64_t n_eff, int64_t m,
    const double* __restrict__ mu, const double* __restrict__ inv_sd, double* __restrict__ X64) {
  __shared__ double tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t t0 = (int64_t)blockIdx.x * 64, i0 = (int64_t)blockIdx.y * 64;
  const int64_t i = i0 + tx;
  for (int r = ty; r < 64; r += 4) {
    const int64_t t = t0 + r;
    tile[r][tx] = (i < m && t < n_eff) ? ((double)E[t * lde + i] - mu[i]) * inv_sd[i] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t iv = i0 + r, t = t0 + tx;
    if (iv < m && t < n_eff) X64[iv * n_eff + t] = tile[tx][r];
  }
}

// Moments of one standardised sample u: log cosh u (overflow-free) and u exp(-u^2/2), FP64.
__device__ inline void moments64(double u, double& a, double& b) {
  const double au = fabs(u);
  a += au + log1p(exp(-2.0 * au)) - kLn2;
  b += u * exp(-0.5 * u * u);
}

__device__ inline double entropy64(double A, double B) {
  return kHGauss - kK1 * (A - kGamma) * (A - kGamma) - kK2 * B * B;
}

// Hx64[i] = H(x_i) in FP64; one workgroup per variable.
__global__ __launch_bounds__(256) void cert_hx_kernel(const double* __restrict__ X64,
                                                      int64_t n_eff, double* __restrict__ Hx) {
  const int64_t i = blockIdx.x;
  __shared__ double ra[4], rb[4];
  double a = 0.0, b = 0.0;
  for (int64_t t = threadIdx.x; t < n_eff; t += 256) moments64(X64[i * n_eff + t], a, b);
  a = wave_sum_d(a);
  b = wave_sum_d(b);
  if ((threadIdx.x & 63) == 0) {
    ra[threadIdx.x >> 6] = a;
    rb[threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double A = (((ra[0] + ra[1]) + ra[2]) + ra[3]) / (double)n_eff;
    const double B = (((rb[0] + rb[1]) + rb[2]) + rb[3]) / (double)n_eff;
    Hx[i] = entropy64(A, B);
  }
}

// One wave per (listed row i, partner j): S[i][j] and S[j][i] in FP64.  A pair of two listed
// rows is formed once (by the smaller row).
__global__ __launch_bounds__(256) void cert_refine_kernel(const double* __restrict__ X64,
                                                          int64_t n_eff, int64_t m,
                                                          const double* __restrict__ Hx,
                                                          const int32_t* __restrict__ list,
                                                          int64_t count,
                                                          const int32_t* __restrict__ listed,
                                                          double* __restrict__ S, int32_t* st) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= count * m) return;
  const int64_t i = list[w / m], j = w % m;
  if (j == i || (listed[j] && j < i)) return;
  const double* xi = X64 + i * n_eff;
  const double* xj = X64 + j * n_eff;
  double r = 0.0;
  for (int64_t t = lane; t < n_eff; t += 64) r += xi[t] * xj[t];
  const double rho = wave_sum_d(r) / (double)n_eff;
  const double omr = 1.0 - rho * rho;
  if (!(omr >= kMinOneMinusRho2)) {
    if (lane == 0) raise_status(st, VL_ERR_DEGENERATE);
    return;
  }
  const double inv_s = 1.0 / sqrt(omr);
  double a0 = 0.0, b0 = 0.0, a1 = 0.0, b1 = 0.0;
  for (int64_t t = lane; t < n_eff; t += 64) {
    moments64((xi[t] - rho * xj[t]) * inv_s, a0, b0);
    moments64((xj[t] - rho * xi[t]) * inv_s, a1, b1);
  }
  a0 = wave_sum_d(a0);
  b0 = wave_sum_d(b0);
  a1 = wave_sum_d(a1);
  b1 = wave_sum_d(b1);
  if (lane == 0) {
    const double n = (double)n_eff;
    const double hr_ij = entropy64(a0 / n, b0 / n), hr_ji = entropy64(a1 / n, b1 / n);
    const double s = (Hx[j] + hr_ij) - (Hx[i] + hr_ji);
    S[i * m + j] = s;
    S[j * m + i] = -s;
  }
}

__global__ void cert_mark_kernel(const int32_t* __restrict__ list, int64_t count,
                                 int32_t* __restrict__ refined, int32_t* __restrict__ listed) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) {
    refined[list[e]] = 1;
    listed[list[e]] = 0;
  }
}

// ------------------------------------------------------------------------------------------
// Alg. 1 with error bounds: one wave, lane l holding variables l + 64 r (as the plain
// single-wave ordering).  Variables in doubt are collected in registers and written at the
// end as a list in index order (deterministic), with listed[i] = 1 and *count.
// ------------------------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(256) void cert_order_kernel(
    const double* __restrict__ S, int64_t m, const int32_t* __restrict__ refined, double eps,
    double tie, int32_t* __restrict__ order, double* __restrict__ margin,
    int32_t* __restrict__ list, int32_t* __restrict__ listed, int32_t* __restrict__ count) {
  __shared__ double M0s[64 * R], EM0s[64 * R];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // phase 0: M and its bound from scratch, one row per wave at a time
  for (int64_t row = wave; row < m; row += 4) {
    const bool rr = refined[row] != 0;
    double s = 0.0, e = 0.0;
    for (int64_t j = lane; j < m; j += 64) {
      if (j == row) continue;
      const double v = S[row * m + j];
      const double ej = (rr || refined[j]) ? 0.0 : eps;
      if (v < 0.0) s += v * v;
      if (v < ej) e += ej * (2.0 * fabs(fmin(v, 0.0)) + ej);
    }
    s = wave_sum_d(s);
    e = wave_sum_d(e);
    if (lane == 0) {
      M0s[row] = s;
      EM0s[row] = e;
    }
  }
  __syncthreads();
  if (wave != 0) return;
  const double inf = INFINITY, gone = __builtin_nan("");
  double Mv[R], EMv[R];
  bool ref[R], doubt[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = lane + 64 * r;
    Mv[r] = i < m ? M0s[i] : gone;
    EMv[r] = i < m ? EM0s[i] : 0.0;
    ref[r] = i < m ? refined[i] != 0 : true;
    doubt[r] = false;
  }
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
    // the pick's own bound, then every candidate that could still be the exact minimum
    double le = inf;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (lane + 64 * r == i1) le = EMv[r];
    const double e1 = wave_min_f64(le);
    const double thr = m1 + e1 - tie;
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool c = lane + 64 * r != i1 && Mv[r] - EMv[r] < thr;   // NaN (gone) is false
      any |= c;
      if (c && !ref[r]) doubt[r] = true;
    }
    if (__builtin_amdgcn_ballot_w64(any)) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (lane + 64 * r == i1 && !ref[r]) doubt[r] = true;
    }
    const int64_t last = m - 1;
    const double* rowp = S + (int64_t)(i1 < m ? i1 : last) * m;
    const bool ref1 = refined[i1 < m ? i1 : last] != 0;
    double v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = lane + 64 * r;
      v[r] = rowp[i < m ? i : last];
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (lane + 64 * r == i1) Mv[r] = gone;
    double l2 = Mv[0];
#pragma unroll
    for (int r = 1; r < R; ++r) l2 = fmin(l2, Mv[r]);
    const double m2 = wave_min_f64(l2);
    if (lane == 0) {
      order[k] = i1;
      margin[k] = (m2 == inf || m2 != m2) ? inf : m2 - m1;
    }
    // removing i1: M_i loses min(0, S_i,i1)^2 = max(0, S_i1,i)^2, its bound that entry's share
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double sij = -v[r];                            // S[i][i1]
      const double pos = v[r] > 0.0 && v[r] < inf ? v[r] : 0.0;
      Mv[r] -= pos * pos;
      const double ej = (ref[r] || ref1) ? 0.0 : eps;
      if (sij < ej) EMv[r] -= ej * (2.0 * fabs(fmin(sij, 0.0)) + ej);
      EMv[r] = fmax(EMv[r], 0.0);
    }
  }
  // the variables in doubt, in index order
  int base = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t b = __builtin_amdgcn_ballot_w64(doubt[r]);
    const int64_t i = lane + 64 * r;
    if (doubt[r]) {
      const int pos = base + __builtin_popcountll(b & ((1ull << lane) - 1ull));
      list[pos] = (int32_t)i;
      listed[i] = 1;
    }
    base += __builtin_popcountll(b);
  }
  if (lane == 0) *count = base;
}

// ------------------------------------------------------------------------------------------
size_t cert_ws_bytes(int64_t n_eff, int64_t m, void* base, CertWs* out) {
  Carver c(base);
  CertWs w;
  w.mu = c.take<double>(m);
  w.inv_sd = c.take<double>(m);
  w.Hx = c.take<double>(m);
  w.X64 = c.take<double>(m * n_eff);
  w.refined = c.take<int32_t>(m);
  w.listed = c.take<int32_t>(m);
  w.list = c.take<int32_t>(m);
  w.count = c.take<int32_t>(1);
  if (out) *out = w;
  return c.used;
}

__global__ void cert_clear_kernel(int32_t* __restrict__ a, int32_t* __restrict__ b, int64_t m) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) a[e] = b[e] = 0;
}

int run_order_certified(const float* E, int64_t n_eff, int64_t m, int64_t lde, double* S,
                        double eps, int32_t* order, double* margin, int32_t* refined_out,
                        int64_t* n_refined, int64_t* rounds, const CertWs& w, int32_t* st,
                        hipStream_t stream) {
  ProfileScope ps("certify", stream);
  cert_colstats_kernel<<<(unsigned)m, 256, 0, stream>>>(E, lde, n_eff, m, w.mu, w.inv_sd, st);
  VL_LAUNCH_CHECK();
  dim3 g((unsigned)ceil_div(n_eff, 64), (unsigned)ceil_div(m, 64));
  cert_standardize_kernel<<<g, 256, 0, stream>>>(E, lde, n_eff, m, w.mu, w.inv_sd, w.X64);
  VL_LAUNCH_CHECK();
  cert_hx_kernel<<<(unsigned)m, 256, 0, stream>>>(w.X64, n_eff, w.Hx);
  VL_LAUNCH_CHECK();
  cert_clear_kernel<<<(unsigned)ceil_div(m, 256), 256, 0, stream>>>(w.refined, w.listed, m);
  VL_LAUNCH_CHECK();
  const double tie = 1e-9;
  int64_t total = 0, r = 0;
  for (;; ++r) {
#define VL_CERT_ORDER(RR)                                                                   \
  cert_order_kernel<RR><<<1, 256, 0, stream>>>(S, m, w.refined, eps, tie, order, margin,     \
                                               w.list, w.listed, w.count)
    if (m <= 64) VL_CERT_ORDER(1);
    else if (m <= 128) VL_CERT_ORDER(2);
    else if (m <= 256) VL_CERT_ORDER(4);
    else if (m <= 512) VL_CERT_ORDER(8);
    else if (m <= 1024) VL_CERT_ORDER(16);
    else if (m <= 2048) VL_CERT_ORDER(32);
    else VL_CERT_ORDER(64);
#undef VL_CERT_ORDER
    VL_LAUNCH_CHECK();
    int32_t cnt = 0;
    if (hipMemcpyAsync(&cnt, w.count, sizeof(int32_t), hipMemcpyDeviceToHost, stream) !=
            hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return VL_ERR_HIP;
    if (cnt == 0 || r >= m) break;
    cert_refine_kernel<<<(unsigned)ceil_div((int64_t)cnt * m, 4), 256, 0, stream>>>(
        w.X64, n_eff, m, w.Hx, w.list, cnt, w.listed, S, st);
    VL_LAUNCH_CHECK();
    cert_mark_kernel<<<(unsigned)ceil_div(cnt, 256), 256, 0, stream>>>(w.list, cnt, w.refined,
                                                                      w.listed);
    VL_LAUNCH_CHECK();
    total += cnt;
  }
  if (refined_out &&
      hipMemcpyAsync(refined_out, w.refined, m * sizeof(int32_t), hipMemcpyDeviceToDevice,
                     stream) != hipSuccess)
    return VL_ERR_HIP;
  if (n_refined) *n_refined = total;
  if (rounds) *rounds = r + 1;
  return VL_OK;
}

}  // namespace vl
