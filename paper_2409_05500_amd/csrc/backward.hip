// Gradient of the pairwise score with respect to the residuals: dL/dE for L = <G, S(E)> with an
// m x m cotangent G (the differentiable form of the precompute of Sec. 4.2 steps 1-2 / Eq. 1-2).
//
// Chain (x = standardised columns, rho_ij = mean x_i x_j, s = sqrt(1 - rho^2),
// u_ij = (x_i - rho x_j)/s, A/B the two entropy moments, Hr = H(nu) - k1 (A-gamma)^2 - k2 B^2):
//   dL/dHr_ij = G_ij - G_ji,             dL/dHx_i = sum_k G_ki - sum_k G_ik
//   alpha_ij = dL/dA_ij = -2 k1 (A_ij - gamma) (G_ij - G_ji),  beta_ij = -2 k2 B_ij (G_ij - G_ji)
//   g_ij(t) = dL/du_ij(t) = (alpha_ij tanh u + beta_ij (1 - u^2) e^{-u^2/2}) / n
//   dx_i(t) += (g_ij(t) - rho_ij g_ji(t)) / s_ij                        (u depends on x_i, x_j)
//   R_ij = dL/drho_ij = sum_t g_ij (rho u_ij / s^2 - x_j / s) + g_ji (rho u_ji / s^2 - x_i / s)
//        = -(1/s^2) sum_t (g_ij u_ji + g_ji u_ij)          (rho u_ij / s^2 - x_j / s = -u_ji / s^2)
//   dx_i(t) += sum_j R_ij x_j(t) / n                                     (rho = mean x_i x_j)
//   dx_i(t) += (alpha^x_i tanh x_i + beta^x_i (1 - x_i^2) e^{-x_i^2/2}) / n   (the Hx term)
//   dE_i(t) = (dx_i(t) - mean dx_i - x_i(t) mean(dx_i x_i)) / sd_i      (standardisation)
//
// The per-sample terms are recomputed (nothing of size m^2 n is stored).  The transcendental
// pass is owner-computes: one wave owns 4 variables and a 128-sample chunk and visits every
// partner block, so each dx_i(t) is summed in registers in a fixed order (no atomics); the
// pair's R contribution of that chunk is reduced across the wave and written per chunk.
#include "backward.hpp"
#include "profile.hpp"

namespace vl {

constexpr int kBT = 4;        // variables per wave (owner block)
constexpr int kBSpl = 2;      // samples per lane (67 VGPRs: many waves hide the trans latency)
constexpr int kBChunk = 64 * kBSpl;

// Per ordered pair (i, j), i != j, the wave-uniform constants of the transcendental pass:
//   (a, b)      w0 = a x_i - b x_j = c u_ij,  w1 = a x_j - b x_i = c u_ji
//   rho         dx_i += G0 - rho G1  with G0 = g_ij / s, G1 = g_ji / s
//   per direction d (0: u_ij with alpha_ij, beta_ij; 1: u_ji with alpha_ji, beta_ji), with
//   A = alpha / (n s), B = beta / (n s):  G = A tanh u + B (1 - u^2) e^{-u^2/2}
//      = 2A r - A + (B - B q / c^2) e,   q = w^2, e = exp2(-q), r = 1 / (1 + e^{-2u})
//   stored as (2A, -A, B, -B / c^2).
struct BwdPair {
  float a, b, rho, pad;
  float a2[2], na[2], bb[2], bq[2];
};
static_assert(sizeof(BwdPair) == 48, "BwdPair is read with scalar loads");

__device__ inline void pair_geometry(const double* __restrict__ cov, int64_t m, int64_t i,
                                     int64_t j, double& rho, double& s) {
  rho = cov[i * m + j] / sqrt(cov[i * m + i] * cov[j * m + j]);
  s = sqrt(fmax(1.0 - rho * rho, kMinOneMinusRho2));
}

__global__ void bwd_pair_kernel(const double* __restrict__ cov, const double* __restrict__ mom,
                                const double* __restrict__ G, int64_t m, int64_t m_pad,
                                int64_t n_eff, BwdPair* __restrict__ bp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m_pad * m_pad) return;
  const int64_t i = e / m_pad, j = e % m_pad;
  BwdPair p = {};
  if (i < m && j < m && i != j) {
    double rho, s;
    pair_geometry(cov, m, i, j, rho, s);
    const double gh = G[i * m + j] - G[j * m + i];            // dL/dHr_ij = -dL/dHr_ji
    const double k = 1.0 / ((double)n_eff * s);
    const double A[2] = {mom[2 * (i * m + j)], mom[2 * (j * m + i)]};
    const double B[2] = {mom[2 * (i * m + j) + 1], mom[2 * (j * m + i) + 1]};
    const double dh[2] = {gh, -gh};
    p.a = (float)(kWScale / s);
    p.b = (float)(kWScale * rho / s);
    p.rho = (float)rho;
    for (int d = 0; d < 2; ++d) {
      const double al = -2.0 * kK1 * (A[d] - kGamma) * dh[d] * k;
      const double be = -2.0 * kK2 * B[d] * dh[d] * k;
      p.a2[d] = (float)(2.0 * al);
      p.na[d] = (float)(-al);
      p.bb[d] = (float)be;
      p.bq[d] = (float)(-be / (kWScale * kWScale));
    }
  }
  bp[j * m_pad + i] = p;
}

// Hx-term coefficients per variable: (alpha^x_i, beta^x_i) / n
__global__ void bwd_var_kernel(const double* __restrict__ momx, const double* __restrict__ G,
                               int64_t m, int64_t m_pad, int64_t n_eff,
                               float2* __restrict__ vx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m_pad) return;
  float2 v = make_float2(0.f, 0.f);
  if (i < m) {
    double c = 0.0;
    for (int64_t k = 0; k < m; ++k) c += G[k * m + i] - G[i * m + k];
    const double inv_n = 1.0 / (double)n_eff;
    v.x = (float)(-2.0 * kK1 * (momx[2 * i] - kGamma) * c * inv_n);
    v.y = (float)(-2.0 * kK2 * momx[2 * i + 1] * c * inv_n);
  }
  vx[i] = v;
}

// One direction's pre-scaled dL/du from w = c u (constants as stored in BwdPair):
//   2A r - A + (B + Bq q) e,  r = 1 / (1 + exp2(kTScale w)) (exact limits 0 and 1 for large |w|)
__device__ __forceinline__ float dir_grad(float w, float a2, float na, float bb, float bq) {
  const float q = w * w;
  const float e = __builtin_amdgcn_exp2f(-q);
  const float t = __builtin_amdgcn_exp2f(w * (float)kTScale);
  const float r = __builtin_amdgcn_rcpf(1.f + t);
  return fmaf(a2, r, fmaf(fmaf(q, bq, bb), e, na));
}

// One wave per (block I of 4 variables, 128-sample chunk); lane l holds samples
// chunk * 128 + 2 l + [0, 2).  The wave walks every partner j (runtime loop, next partner's
// samples prefetched), and for the 4 pairs (i, j), i in I: dx_i += g_ij / s - rho g_ji / s and
// the chunk's R partial of (i, j) is summed across the wave.  Output: dx (m_pad x n_pad,
// variable-major FP32: direct and Hx terms) and Rp[chunk][i][j] for j > i.
// Pair constants are stored transposed, bp[j * m_pad + i], so the 4 pairs of one step are
// contiguous (wave-uniform scalar loads).
__global__ __launch_bounds__(256) void bwd_owner_kernel(
    const float* __restrict__ Xs, int64_t n_pad, const BwdPair* __restrict__ bp,
    const float2* __restrict__ vx, int64_t m_pad, int64_t m, int nt, int64_t nchunk,
    float* __restrict__ dx, float* __restrict__ Rp) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * 4 + wave;
  if (item >= (int64_t)nt * nchunk) return;
  const int64_t chunk = item / nt;
  const int bi = (int)(item - chunk * nt);
  const int64_t i0 = (int64_t)bi * kBT;
  const int64_t tb = chunk * kBChunk + kBSpl * lane;

  // dL/dx_i(t) is summed in FP64: the Hx term and the sum of the pair terms nearly cancel
  // (each pair term follows Hr_ij - Hx_i, a small difference), so FP32 partial sums would
  // carry rounding at many times the scale of the result.
  float xi[kBT][kBSpl], xj[kBSpl];
  double acc[kBT][kBSpl];
  static_assert(kBSpl == 2, "float2 loads and stores");
  auto load_x = [&](const float* src, int64_t row, float* dst) {
    const float2 f = *reinterpret_cast<const float2*>(src + row * n_pad + tb);
    dst[0] = f.x;
    dst[1] = f.y;
  };
#pragma unroll
  for (int ii = 0; ii < kBT; ++ii) {
    load_x(Xs, i0 + ii, xi[ii]);
    // Hx term: the standardised column's own entropy moments
    const float2 cx = vx[i0 + ii];
#pragma unroll
    for (int e = 0; e < kBSpl; ++e)
      acc[ii][e] = (double)dir_grad(xi[ii][e] * (float)kWScale, 2.f * cx.x, -cx.x, cx.y,
                                    cx.y * (float)(-1.0 / (kWScale * kWScale)));
  }
  load_x(Xs, 0, xj);

  for (int64_t j = 0; j < m; ++j) {
    float xn[kBSpl];
    load_x(Xs, j + 1 < m_pad ? j + 1 : j, xn);      // prefetch the next partner
    const BwdPair* c4 = bp + j * m_pad + i0;
    float rs[kBT];
#pragma unroll
    for (int ii = 0; ii < kBT; ++ii) {
      const BwdPair c = c4[ii];
      float r = 0.f;
#pragma unroll
      for (int e = 0; e < kBSpl; ++e) {
        const float x = xi[ii][e], y = xj[e];
        const float w0 = fmaf(x, c.a, -(y * c.b));      // c u_ij
        const float w1 = fmaf(y, c.a, -(x * c.b));      // c u_ji
        const float g0 = dir_grad(w0, c.a2[0], c.na[0], c.bb[0], c.bq[0]);   // g_ij / s
        const float g1 = dir_grad(w1, c.a2[1], c.na[1], c.bb[1], c.bq[1]);   // g_ji / s
        acc[ii][e] += (double)fmaf(-c.rho, g1, g0);
        // rho chain: (g_ij / s)(c u_ji) + (g_ji / s)(c u_ij), = -R_ij c / s summed over t
        r = fmaf(g0, w1, fmaf(g1, w0, r));
      }
      rs[ii] = r;
    }
#pragma unroll
    for (int ii = 0; ii < kBT; ++ii) rs[ii] = wave_sum(rs[ii]);
    if (lane < kBT) {
      float v = rs[0];
#pragma unroll
      for (int ii = 1; ii < kBT; ++ii) v = lane == ii ? rs[ii] : v;
      if (i0 + lane < j) Rp[(chunk * m + i0 + lane) * m + j] = v;    // j > i: one copy
    }
#pragma unroll
    for (int e = 0; e < kBSpl; ++e) xj[e] = xn[e];
  }
#pragma unroll
  for (int ii = 0; ii < kBT; ++ii)
    *reinterpret_cast<float2*>(dx + (i0 + ii) * n_pad + tb) =
        make_float2((float)acc[ii][0], (float)acc[ii][1]);
}

// R[i][j] = R[j][i] = -(sum over chunks of Rp[c][i][j], i < j) / (c s n)  (FP64 sum), the
// factor 1/n of d rho / d x included; stored as FP32 for the R x product.  One thread per
// i <= j (coalesced reads along j); diagonal and padding 0.
__global__ void bwd_r_combine_kernel(const float* __restrict__ Rp, int64_t nchunk,
                                     const double* __restrict__ cov, int64_t m, int64_t m_pad,
                                     int64_t n_eff, float* __restrict__ Rf) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m_pad * m_pad) return;
  const int64_t i = e / m_pad, j = e % m_pad;
  if (i > j) return;
  double v = 0.0;
  if (j < m && i != j) {
    double sum = 0.0;
    for (int64_t c = 0; c < nchunk; ++c) sum += (double)Rp[c * m * m + i * m + j];
    double rho, s;
    pair_geometry(cov, m, i, j, rho, s);
    v = -sum / (kWScale * s * (double)n_eff);
  }
  Rf[i * m_pad + j] = (float)v;
  Rf[j * m_pad + i] = (float)v;
}

// dx[i][t] += sum_j Rf[i][j] Xs[j][t]: 64 (i) x 64 (t) tiles, FP32 MFMA 32x32x2, K = m_pad.
typedef float f32x16 __attribute__((ext_vector_type(16)));
__global__ __launch_bounds__(256) void bwd_rx_kernel(const float* __restrict__ Rf,
                                                     const float* __restrict__ Xs, int64_t m_pad,
                                                     int64_t n_pad, float* __restrict__ dx) {
  __shared__ float Rs[32][64 + 1];   // [j][i]
  __shared__ float Xl[32][64 + 1];   // [j][t]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wt = wave & 1;
  const int64_t i0 = (int64_t)blockIdx.y * 64, t0 = (int64_t)blockIdx.x * 64;
  f32x16 acc = {};
  for (int64_t k0 = 0; k0 < m_pad; k0 += 32) {
    {
      const int kk = tid & 31, ii = tid >> 5;     // 32 j x 8 i per pass
      // clamped in-bounds addresses, padding masked after the loads (no branch per load)
      float rv[8], xv[8];
      const int tt = tid & 63, kr = tid >> 6;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t i = i0 + ii + 8 * r, j = k0 + kk;
        rv[r] = Rf[(i < m_pad ? i : m_pad - 1) * m_pad + (j < m_pad ? j : m_pad - 1)];
        const int64_t j2 = k0 + kr + 4 * r, t = t0 + tt;
        xv[r] = Xs[(j2 < m_pad ? j2 : m_pad - 1) * n_pad + (t < n_pad ? t : n_pad - 1)];
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t i = i0 + ii + 8 * r, j = k0 + kk;
        Rs[kk][ii + 8 * r] = mask_f32(rv[r], i < m_pad && j < m_pad);
        const int64_t j2 = k0 + kr + 4 * r, t = t0 + tt;
        Xl[kr + 4 * r][tt] = mask_f32(xv[r], j2 < m_pad && t < n_pad);
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 32; kk += 2) {
      const float a = Rs[kk + (lane >> 5)][wi * 32 + (lane & 31)];
      const float b = Xl[kk + (lane >> 5)][wt * 32 + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t i = i0 + wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int64_t t = t0 + wt * 32 + (lane & 31);
    if (i < m_pad && t < n_pad) dx[i * n_pad + t] += acc[r];
  }
}

// Per variable: sums over valid samples of dx and dx * x (FP64), one block per variable.
__global__ __launch_bounds__(256) void bwd_colsum_kernel(const float* __restrict__ dx,
                                                         const float* __restrict__ Xs,
                                                         int64_t n_pad, int64_t n_eff,
                                                         double* __restrict__ sums) {
  __shared__ double r1[4], r2[4];
  const int64_t i = blockIdx.x;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t t = threadIdx.x; t < n_eff; t += 256) {
    const double d = dx[i * n_pad + t];
    s1 += d;
    s2 += d * (double)Xs[i * n_pad + t];
  }
  s1 = wave_sum_d(s1);
  s2 = wave_sum_d(s2);
  if ((threadIdx.x & 63) == 0) {
    r1[threadIdx.x >> 6] = s1;
    r2[threadIdx.x >> 6] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sums[2 * i] = ((r1[0] + r1[1]) + r1[2]) + r1[3];
    sums[2 * i + 1] = ((r2[0] + r2[1]) + r2[2]) + r2[3];
  }
}

// dE[t][i] = (dx_i(t) - mean dx_i - x_i(t) mean(dx_i x_i)) / sd_i, transposed to sample-major.
__global__ __launch_bounds__(256) void bwd_std_kernel(const float* __restrict__ dx,
                                                      const float* __restrict__ Xs,
                                                      const double* __restrict__ sums,
                                                      const double* __restrict__ cov, int64_t m,
                                                      int64_t n_pad, int64_t n_eff,
                                                      float* __restrict__ dE, int64_t ldde) {
  __shared__ float tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t t0 = (int64_t)blockIdx.x * 64, i0 = (int64_t)blockIdx.y * 64;
  // read along t (variable-major), write along i (sample-major)
  for (int r = ty; r < 64; r += 4) {
    const int64_t i = i0 + r, t = t0 + tx;
    float v = 0.f;
    if (i < m && t < n_eff) {
      const double inv_n = 1.0 / (double)n_eff;
      const double d = dx[i * n_pad + t], x = Xs[i * n_pad + t];
      v = (float)((d - sums[2 * i] * inv_n - x * sums[2 * i + 1] * inv_n) /
                  sqrt(cov[i * m + i]));
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t t = t0 + r, i = i0 + tx;
    if (i < m && t < n_eff) dE[t * ldde + i] = tile[tx][r];
  }
}

BwdPlan plan_backward(int64_t n_eff, int64_t m) {
  BwdPlan b;
  b.fwd = plan_pairwise(n_eff, m);
  b.nt = (int)ceil_div(m, kBT);
  b.m_pad = (int64_t)b.nt * kBT;
  b.nchunk = ceil_div(n_eff, kBChunk);
  b.n_pad = b.nchunk * kBChunk;
  return b;
}

size_t bwd_ws_bytes(const BwdPlan& b, void* base, BwdWs* out) {
  Carver c(base);
  BwdWs w;
  const size_t fwd = pairwise_ws_bytes(b.fwd, nullptr, nullptr);
  char* fbase = c.take<char>(fwd);
  if (base) pairwise_ws_bytes(b.fwd, fbase, &w.fwd);
  const int64_t m = b.fwd.m;
  w.Hx = c.take<double>(m);
  w.Hr = c.take<double>(m * m);
  w.S = c.take<double>(m * m);
  w.cov = c.take<double>(m * m);
  w.mom = c.take<double>(2 * m * m);
  w.Xs = c.take<float>(b.m_pad * b.n_pad);
  w.bp = c.take<BwdPair>(b.m_pad * b.m_pad);
  w.vx = c.take<float2>(b.m_pad);
  w.dx = c.take<float>(b.m_pad * b.n_pad);
  w.Rp = c.take<float>((size_t)b.nchunk * m * m);
  w.Rf = c.take<float>(b.m_pad * b.m_pad);
  w.sums = c.take<double>(2 * m);
  if (out) *out = w;
  return c.used;
}

int run_backward(const BwdPlan& b, const BwdWs& w, const float* E, int64_t lde, int prec,
                 const double* saved, const double* G, float* dE, int64_t ldde, int32_t* st,
                 hipStream_t stream) {
  const int64_t m = b.fwd.m, n_eff = b.fwd.n_eff;
  int rc = VL_OK;
  // the forward's statistics: the saved block [A,B per ordered pair | A,B per variable |
  // covariance | means], else recomputed here
  const double *mom = w.mom, *momx = w.fwd.momx, *cov = w.cov, *mu = w.fwd.mu;
  if (saved) {
    mom = saved;
    momx = saved + 2 * m * m;
    cov = saved + 2 * m * m + 2 * m;
    mu = saved + 3 * m * m + 2 * m;
  } else {
    rc = run_pairwise(b.fwd, w.fwd, E, lde, prec, w.Hx, w.Hr, w.S, w.cov, w.mom, st, stream);
    if (rc) return rc;
  }
  {
    ProfileScope ps("backward_prep", stream);
    // standardised variable-major copy in this pass's chunking (zero padded)
    rc = standardize_to(E, lde, n_eff, m, mu, cov, w.Xs, b.n_pad, b.m_pad, st, stream);
    if (rc) return rc;
    bwd_pair_kernel<<<(unsigned)ceil_div(b.m_pad * b.m_pad, 256), 256, 0, stream>>>(
        cov, mom, G, m, b.m_pad, n_eff, w.bp);
    VL_LAUNCH_CHECK();
    bwd_var_kernel<<<(unsigned)ceil_div(b.m_pad, 256), 256, 0, stream>>>(momx, G, m, b.m_pad,
                                                                        n_eff, w.vx);
    VL_LAUNCH_CHECK();
  }
  {
    ProfileScope ps("backward_owner", stream);
    const int64_t items = (int64_t)b.nt * b.nchunk;
    bwd_owner_kernel<<<(unsigned)ceil_div(items, 4), 256, 0, stream>>>(
        w.Xs, b.n_pad, w.bp, w.vx, b.m_pad, m, b.nt, b.nchunk, w.dx, w.Rp);
    VL_LAUNCH_CHECK();
  }
  {
    ProfileScope ps("backward_tail", stream);
    bwd_r_combine_kernel<<<(unsigned)ceil_div(b.m_pad * b.m_pad, 256), 256, 0, stream>>>(
        w.Rp, b.nchunk, cov, m, b.m_pad, n_eff, w.Rf);
    VL_LAUNCH_CHECK();
    dim3 grx((unsigned)ceil_div(b.n_pad, 64), (unsigned)ceil_div(b.m_pad, 64));
    bwd_rx_kernel<<<grx, 256, 0, stream>>>(w.Rf, w.Xs, b.m_pad, b.n_pad, w.dx);
    VL_LAUNCH_CHECK();
    bwd_colsum_kernel<<<(unsigned)m, 256, 0, stream>>>(w.dx, w.Xs, b.n_pad, n_eff, w.sums);
    VL_LAUNCH_CHECK();
    dim3 gs((unsigned)ceil_div(n_eff, 64), (unsigned)ceil_div(m, 64));
    bwd_std_kernel<<<gs, 256, 0, stream>>>(w.dx, w.Xs, w.sums, cov, m, b.n_pad, n_eff, dE,
                                           ldde);
    VL_LAUNCH_CHECK();
  }
  return VL_OK;
}

}  // namespace vl
