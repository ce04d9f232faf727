// Ensembles of the fit.
//
// Residual bootstrap of the VAR of Sec. 2.1: resample b starts from the first p observed rows
// and continues x*(t) = c + sum_{tau=1..p} M_tau x*(t - tau) + e(idx_b[t - p]) with the fit's
// residual rows drawn with replacement (the draws are an input).  One workgroup runs one
// resample; the last p + 1 rows sit in an LDS ring, the lag matrices are read transposed
// (M_tau^T, so the threads of a wave read consecutive doubles), the recursion runs in FP64 from
// the FP32 rows it stored (the series is the batched fit's FP32 input).
//
// Aggregation over K fits of one dataset (rolling windows, resamples): edge probabilities
// P0[i][j] = #{k : |B0_k[i][j]| > threshold} / K', the same for every B_tau, and the order
// precedence P_order[i][j] = #{k : j precedes i in order_k} / K', over the K' problems whose
// status is VL_OK.  Integer counts divided once: exact and order-independent.
#include "ensemble.hpp"
#include "profile.hpp"

namespace vl {
namespace {

// Mt[(tau-1) m m + k m + i] = M[(tau-1) m m + i m + k]
__global__ void sim_transpose_kernel(const double* __restrict__ M, int64_t m, int p,
                                     double* __restrict__ Mt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)p * m * m) return;
  const int64_t tau1 = e / (m * m), rem = e % (m * m), i = rem / m, k = rem % m;
  Mt[tau1 * m * m + k * m + i] = M[e];
}

__global__ __launch_bounds__(256) void var_simulate_kernel(
    const double* __restrict__ Mt, const double* __restrict__ c, int64_t m, int p,
    const float* __restrict__ X0, int64_t ldx0, const float* __restrict__ E, int64_t n_e,
    int64_t lde, const int32_t* __restrict__ idx, int64_t T, float* __restrict__ Xout,
    int64_t ldxo, int64_t sstride, int32_t* st) {
  extern __shared__ float ring[];  // (p + 1) x m: row t in slot t mod (p + 1)
  const int64_t b = blockIdx.x;
  float* Xb = Xout + b * sstride;
  const int32_t* ib = idx + b * T;
  const int slots = p + 1;
  for (int64_t e = threadIdx.x; e < (int64_t)p * m; e += 256) {
    const int64_t r = e / m, i = e % m;
    const float v = X0[r * ldx0 + i];
    Xb[r * ldxo + i] = v;
    ring[r * m + i] = v;
  }
  __syncthreads();
  for (int64_t t = p; t < p + T; ++t) {
    int64_t j = ib[t - p];
    if (j < 0 || j >= n_e) {
      if (threadIdx.x == 0) raise_status(st, VL_ERR_INVALID_ARG);
      j = j < 0 ? 0 : n_e - 1;
    }
    const float* e = E + j * lde;
    float* out = ring + (t % slots) * m;
    for (int64_t i = threadIdx.x; i < m; i += 256) {
      double acc = c[i] + (double)e[i];
      for (int tau = 1; tau <= p; ++tau) {
        const float* xr = ring + ((t - tau) % slots) * m;
        const double* Mtt = Mt + (int64_t)(tau - 1) * m * m + i;
        double s0 = 0.0, s1 = 0.0;
        int64_t k = 0;
        for (; k + 2 <= m; k += 2) {
          s0 += Mtt[k * m] * (double)xr[k];
          s1 += Mtt[(k + 1) * m] * (double)xr[k + 1];
        }
        if (k < m) s0 += Mtt[k * m] * (double)xr[k];
        acc += s0 + s1;
      }
      const float v = (float)acc;
      Xb[t * ldxo + i] = v;
      out[i] = v;
    }
    __syncthreads();
  }
}

// The same recursion with the lag matrices held in registers: thread (tau, part, i) keeps
// M_tau[i][part kSC .. part kSC + kSC - 1] and forms that slice of the dot product from the LDS
// ring (every lane of a wave reads the same ring word: a broadcast); thread i then adds the
// p * parts partial sums in a fixed order.  Used when m p ceil(m / kSC) <= kSimThreads.
constexpr int kSC = 64;
constexpr int kSimThreads = 512;

__global__ __launch_bounds__(kSimThreads) void var_simulate_reg_kernel(
    const double* __restrict__ M, const double* __restrict__ c, int m, int p,
    const float* __restrict__ X0, int64_t ldx0, const float* __restrict__ E, int64_t n_e,
    int64_t lde, const int32_t* __restrict__ idx, int64_t T, float* __restrict__ Xout,
    int64_t ldxo, int64_t sstride, int32_t* st) {
  extern __shared__ double sim_lds[];
  const int tid = threadIdx.x;
  const int parts = (m + kSC - 1) / kSC;
  const int groups = p * parts;                      // (tau, part) pairs
  double* partial = sim_lds;                         // groups x m
  float* ring = reinterpret_cast<float*>(sim_lds + (int64_t)groups * m);  // (p+1) m + kSC
  const int slots = p + 1;
  const int64_t b = blockIdx.x;
  float* Xb = Xout + b * sstride;
  const int32_t* ib = idx + b * T;
  const bool active = tid < groups * m;
  const int g = active ? tid / m : 0, i = active ? tid % m : 0;
  const int tau = g / parts + 1, k0 = (g % parts) * kSC;
  double mr[kSC];
#pragma unroll
  for (int u = 0; u < kSC; ++u)
    mr[u] = active && k0 + u < m ? M[(int64_t)(tau - 1) * m * m + (int64_t)i * m + k0 + u] : 0.0;
  for (int e = tid; e < slots * m + kSC; e += kSimThreads) ring[e] = 0.0f;
  __syncthreads();
  for (int e = tid; e < p * m; e += kSimThreads) {
    const int r = e / m, j = e % m;
    const float v = X0[(int64_t)r * ldx0 + j];
    Xb[(int64_t)r * ldxo + j] = v;
    ring[r * m + j] = v;
  }
  __syncthreads();
  for (int64_t t = p; t < p + T; ++t) {
    if (active) {
      const float* xr = ring + ((t - tau) % slots) * m + k0;
      double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < kSC; ++u) s[u & 3] += mr[u] * (double)xr[u];
      partial[tid] = (s[0] + s[1]) + (s[2] + s[3]);
    }
    __syncthreads();
    if (tid < m) {
      int64_t j = ib[t - p];
      if (j < 0 || j >= n_e) {
        raise_status(st, VL_ERR_INVALID_ARG);
        j = j < 0 ? 0 : n_e - 1;
      }
      double acc = c[tid] + (double)E[j * lde + tid];
      for (int q = 0; q < groups; ++q) acc += partial[q * m + tid];
      const float v = (float)acc;
      Xb[t * ldxo + tid] = v;
      ring[(t % slots) * m + tid] = v;
    }
    __syncthreads();
  }
}

// pos[k m + order_k[r]] = r (clamped indices; the orders of failed problems are never read)
__global__ void order_positions_kernel(const int32_t* __restrict__ orders, int64_t K, int64_t m,
                                       int32_t* __restrict__ pos) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * m) return;
  const int64_t k = e / m, r = e % m;
  int v = orders[e];
  v = v < 0 ? 0 : (v >= m ? (int)m - 1 : v);
  pos[k * m + v] = (int32_t)r;
}

// One thread per output entry: [0, m^2) P0, [m^2, (p+1) m^2) P_tau, [(p+1) m^2, (p+2) m^2)
// P_order.
__global__ void edge_frequency_kernel(const int32_t* __restrict__ pos,
                                      const double* __restrict__ B0s,
                                      const double* __restrict__ Bls, int64_t K, int64_t m,
                                      int p, double thr, const int32_t* __restrict__ pst,
                                      double* __restrict__ P0, double* __restrict__ Pl,
                                      double* __restrict__ Po, int32_t* __restrict__ count) {
  const int64_t mm = m * m;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (p + 2) * mm) return;
  int64_t hits = 0, used = 0;
  if (e < mm) {
    for (int64_t k = 0; k < K; ++k) {
      if (pst && pst[k] != 0) continue;
      ++used;
      hits += fabs(B0s[k * mm + e]) > thr ? 1 : 0;
    }
    P0[e] = used ? (double)hits / (double)used : 0.0;
  } else if (e < (p + 1) * mm) {
    const int64_t f = e - mm;
    for (int64_t k = 0; k < K; ++k) {
      if (pst && pst[k] != 0) continue;
      ++used;
      hits += fabs(Bls[k * p * mm + f]) > thr ? 1 : 0;
    }
    Pl[f] = used ? (double)hits / (double)used : 0.0;
  } else {
    const int64_t f = e - (p + 1) * mm, i = f / m, j = f % m;
    for (int64_t k = 0; k < K; ++k) {
      if (pst && pst[k] != 0) continue;
      ++used;
      hits += pos[k * m + j] < pos[k * m + i] ? 1 : 0;
    }
    Po[f] = used ? (double)hits / (double)used : 0.0;
  }
  if (e == 0) *count = (int32_t)used;
}

}  // namespace

size_t sim_ws_bytes(int64_t m, int p) {
  Carver c(nullptr);
  c.take<double>((size_t)p * m * m);
  return c.used;
}

int run_var_simulate(const double* M, const double* intercept, int64_t m, int p, const float* X0,
                     int64_t ldx0, const float* E, int64_t n_e, int64_t lde, const int32_t* idx,
                     int64_t R, int64_t T, float* Xout, int64_t ldxo, int64_t series_stride,
                     void* ws, int32_t* st, hipStream_t stream) {
  ProfileScope ps("simulate", stream);
  Carver c(ws);
  double* Mt = c.take<double>((size_t)p * m * m);
  const int64_t nm = (int64_t)p * m * m;
  sim_transpose_kernel<<<(unsigned)ceil_div(nm, 256), 256, 0, stream>>>(M, m, p, Mt);
  VL_LAUNCH_CHECK();
  const int64_t groups = (int64_t)p * ceil_div(m, kSC);
  if (groups * m <= kSimThreads) {
    const size_t lds = (size_t)groups * m * sizeof(double) + ((size_t)(p + 1) * m + kSC) * 4;
    var_simulate_reg_kernel<<<(unsigned)R, kSimThreads, lds, stream>>>(
        M, intercept, (int)m, p, X0, ldx0, E, n_e, lde, idx, T, Xout, ldxo, series_stride, st);
    VL_LAUNCH_CHECK();
    return VL_OK;
  }
  const size_t lds = (size_t)(p + 1) * m * sizeof(float);
  var_simulate_kernel<<<(unsigned)R, 256, lds, stream>>>(Mt, intercept, m, p, X0, ldx0, E, n_e,
                                                         lde, idx, T, Xout, ldxo, series_stride,
                                                         st);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

size_t freq_ws_bytes(int64_t K, int64_t m) {
  Carver c(nullptr);
  c.take<int32_t>((size_t)K * m);
  return c.used;
}

int run_edge_frequency(const int32_t* orders, const double* B0s, const double* Blags, int64_t K,
                       int64_t m, int p, double threshold, const int32_t* problem_status,
                       double* P0, double* Plag, double* P_order, int32_t* count, void* ws,
                       int32_t* st, hipStream_t stream) {
  (void)st;
  Carver c(ws);
  int32_t* pos = c.take<int32_t>((size_t)K * m);
  order_positions_kernel<<<(unsigned)ceil_div(K * m, 256), 256, 0, stream>>>(orders, K, m, pos);
  VL_LAUNCH_CHECK();
  const int64_t tot = (int64_t)(p + 2) * m * m;
  edge_frequency_kernel<<<(unsigned)ceil_div(tot, 256), 256, 0, stream>>>(
      pos, B0s, Blags, K, m, p, threshold, problem_status, P0, Plag, P_order, count);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

}  // namespace vl
