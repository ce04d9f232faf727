// The original iterative DirectLiNGAM ordering (Sec. 3 steps 1-5), the search that the
// heuristic's one-time precompute replaces.  Each step scores every ordered pair of the
// remaining variables on the current data (the pairwise stage of the heuristic path, on the
// current columns), picks the variable with the smallest aggregate M_i = sum_j min(0, S_ij)^2
// (Eq. 3; lowest index on exact ties), then replaces every remaining column by its residual on
// the pick, computed from the standardised columns (Sec. 3 step 5):
//     x_j <- (x_j - mu_j)/s_j - rho_jc (x_c - mu_c)/s_c,
// and drops the pick.  The current columns stay in ascending original order (a compacting
// copy), so the lowest current index is the lowest original index.  One pairwise pass per step:
// sum_u u^2 n = O(m^3 n) sample-evals in all.  The loop is launched from the host without
// synchronisation: the pick stays on the device.
#include "iterative.hpp"
#include "order.hpp"
#include "pairwise.hpp"
#include "profile.hpp"

#include <algorithm>

namespace vl {

__global__ void iter_init_kernel(int32_t* __restrict__ idx, int64_t m) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) idx[e] = (int32_t)e;
}

constexpr int kIterMaxM = 4096;

// M_i over the u current columns, the pick c (smallest M, lowest index on ties) and the margin
// (second-smallest M minus the smallest; +inf with one column left).  One workgroup.
__global__ __launch_bounds__(256) void iter_select_kernel(const double* __restrict__ S, int64_t u,
                                                          const int32_t* __restrict__ idx,
                                                          int64_t k, int32_t* __restrict__ order,
                                                          double* __restrict__ margin,
                                                          int32_t* __restrict__ pick) {
  __shared__ double Mv[kIterMaxM];
  __shared__ double rv[256];
  __shared__ int ri[256];
  const int tid = threadIdx.x;
  if (u == 1) {
    if (tid == 0) {
      order[k] = idx[0];
      margin[k] = INFINITY;
      *pick = 0;
    }
    return;
  }
  // S is antisymmetric bit for bit (S_ji = -S_ij), so min(0, S_ij)^2 = max(0, S_ji)^2: the
  // same sum in the same order, read along columns (consecutive threads, consecutive words)
  // (16 loads in flight, then summed in j order)
  constexpr int kL = 16;
  for (int64_t i = tid; i < u; i += 256) {
    double s = 0.0;
    int64_t j = 0;
    for (; j + kL <= u; j += kL) {
      double v[kL];
#pragma unroll
      for (int q = 0; q < kL; ++q) v[q] = S[(j + q) * u + i];
#pragma unroll
      for (int q = 0; q < kL; ++q)
        if (j + q != i && v[q] > 0.0) s += v[q] * v[q];
    }
    for (; j < u; ++j) {
      const double v = S[j * u + i];
      if (j != i && v > 0.0) s += v * v;
    }
    Mv[i] = s;
  }
  __syncthreads();
  // smallest M, lowest index on ties
  double bv = INFINITY;
  int bi = 0x7fffffff;
  for (int64_t i = tid; i < u; i += 256)
    if (Mv[i] < bv || (Mv[i] == bv && (int)i < bi)) {
      bv = Mv[i];
      bi = (int)i;
    }
  rv[tid] = bv;
  ri[tid] = bi;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      const double ov = rv[tid + h];
      const int oi = ri[tid + h];
      if (ov < rv[tid] || (ov == rv[tid] && oi < ri[tid])) {
        rv[tid] = ov;
        ri[tid] = oi;
      }
    }
    __syncthreads();
  }
  const double m1 = rv[0];
  const int c = ri[0];
  __syncthreads();
  // second smallest
  double b2 = INFINITY;
  for (int64_t i = tid; i < u; i += 256)
    if ((int)i != c) b2 = fmin(b2, Mv[i]);
  rv[tid] = b2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) rv[tid] = fmin(rv[tid], rv[tid + h]);
    __syncthreads();
  }
  if (tid == 0) {
    order[k] = idx[c < u ? c : 0];
    margin[k] = rv[0] - m1;
    *pick = c < u ? c : 0;
  }
}

// Column j' of the next data: the standardised x_j minus rho_jc times the standardised x_c,
// with j = j' + (j' >= c); FP64 arithmetic, FP32 storage.
__global__ void iter_refine_kernel(const float* __restrict__ Ek, int64_t ldk, int64_t n_eff,
                                   int64_t u, const double* __restrict__ mu,
                                   const double* __restrict__ Cov,
                                   const int32_t* __restrict__ pick,
                                   const int32_t* __restrict__ idx_in,
                                   int32_t* __restrict__ idx_out, float* __restrict__ En,
                                   int64_t ldn) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t w = u - 1;
  if (e >= n_eff * w) return;
  const int64_t t = e / w, jp = e % w;
  const int64_t c = *pick;
  const int64_t j = jp + (jp >= c ? 1 : 0);
  const double sj = sqrt(Cov[j * u + j]), sc = sqrt(Cov[c * u + c]);
  const double rho = Cov[j * u + c] / (sj * sc);
  const double v = ((double)Ek[t * ldk + j] - mu[j]) / sj -
                   rho * (((double)Ek[t * ldk + c] - mu[c]) / sc);
  En[t * ldn + jp] = (float)v;
  if (t == 0) idx_out[jp] = idx_in[j];
}

// Hybrid finish: the remaining variables' lookup order, mapped to original indices.
__global__ void iter_map_kernel(const int32_t* __restrict__ osub,
                                const int32_t* __restrict__ idx, int64_t u,
                                int32_t* __restrict__ order) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= u) return;
  int32_t v = osub[r];
  v = v < 0 ? 0 : (v >= u ? (int32_t)u - 1 : v);
  order[r] = idx[v];
}

size_t iter_ws_bytes(int64_t n_eff, int64_t m, void* base, IterWs* out) {
  Carver c(base);
  IterWs w;
  w.D[0] = c.take<float>(n_eff * m);
  w.D[1] = c.take<float>(n_eff * m);
  w.idx[0] = c.take<int32_t>(m);
  w.idx[1] = c.take<int32_t>(m);
  w.pick = c.take<int32_t>(1);
  w.Hx = c.take<double>(m);
  w.Hr = c.take<double>(m * m);
  w.S = c.take<double>(m * m);
  w.Cov = c.take<double>(m * m);
  size_t pw = 0;
  for (int64_t u = 2; u <= m; ++u)
    pw = std::max(pw, pairwise_ws_bytes(plan_pairwise(n_eff, u), nullptr, nullptr));
  w.pw = c.take<char>(pw);
  w.osub = c.take<int32_t>(m);
  w.M0 = c.take<double>(m);
  if (out) *out = w;
  return c.used;
}

int run_order_iterative(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec,
                        int64_t k_exact, int32_t* order, double* margin, const IterWs& w,
                        int32_t* st, hipStream_t stream) {
  if (m > kIterMaxM) return VL_ERR_SHAPE;
  ProfileScope ps("iterative", stream);
  iter_init_kernel<<<(unsigned)ceil_div(m, (int64_t)256), 256, 0, stream>>>(w.idx[0], m);
  VL_LAUNCH_CHECK();
  const float* cur = E;
  int64_t ldc = lde;
  for (int64_t k = 0; k < m; ++k) {
    const int64_t u = m - k;
    const int32_t* idx_in = w.idx[k & 1];
    PairwiseWs pw;
    if (u >= 2) {
      const PairwisePlan p = plan_pairwise(n_eff, u);
      pairwise_ws_bytes(p, w.pw, &pw);
      int rc = run_pairwise(p, pw, cur, ldc, prec, w.Hx, w.Hr, w.S, w.Cov, nullptr, st, stream);
      if (rc) return rc;
      if (k == k_exact) {             // hybrid: the heuristic orders the remaining variables
        rc = run_order(w.S, u, w.osub, margin + k, w.M0, st, stream);
        if (rc) return rc;
        iter_map_kernel<<<(unsigned)ceil_div(u, (int64_t)256), 256, 0, stream>>>(
            w.osub, idx_in, u, order + k);
        VL_LAUNCH_CHECK();
        return VL_OK;
      }
    }
    iter_select_kernel<<<1, 256, 0, stream>>>(w.S, u, idx_in, k, order, margin, w.pick);
    VL_LAUNCH_CHECK();
    if (u >= 2) {
      float* next = w.D[k & 1];
      iter_refine_kernel<<<(unsigned)ceil_div(n_eff * (u - 1), (int64_t)256), 256, 0, stream>>>(
          cur, ldc, n_eff, u, pw.mu, w.Cov, w.pick, idx_in, w.idx[(k + 1) & 1], next, m);
      VL_LAUNCH_CHECK();
      cur = next;
      ldc = m;
    }
  }
  return VL_OK;
}

}  // namespace vl
