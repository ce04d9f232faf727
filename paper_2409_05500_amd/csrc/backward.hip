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
// pass evaluates each pair once: a workgroup takes one 128-sample chunk and a row a of the
// 32 x 32 tiles of variable pairs (blocks a <= b of 32 variables); each wave keeps its own 4
// rows of block a in registers over the row and visits the 4-row blocks of b in a rotation
// that gives every block of b to one wave per round, whose sums go through LDS.  Each pair adds
// its two terms to dx_i and dx_j and its chunk's R partial; the sums of block b from row a are
// written as one partial per (row, variable) and summed in a fixed order afterwards, so the
// result is deterministic with no atomics.
#include <algorithm>
#include <type_traits>

#include "backward.hpp"
#include "profile.hpp"

namespace vl {

// 8 waves: three workgroups share a CU (76 VGPRs), so one workgroup's round barrier overlaps
// the others' work (16 waves at one workgroup per CU: 15% slower)
constexpr int kTW = 8;              // waves per workgroup of the pair-tile pass
constexpr int kTT = 4;              // variables per wave block
constexpr int kTK = kTW * kTT;      // 32 variables per tile side
constexpr int kBSpl = 2;            // samples per lane
constexpr int kBChunk = 64 * kBSpl;
constexpr int64_t kPdBytes = int64_t(2) << 30;   // per-partner-block sums of one window
constexpr double kExpMinusHalf = 0.60653065971263342360;   // e^{-1/2}

// Per ordered pair (i, j), i != j, the wave-uniform constants of the transcendental pass:
//   (a, b)      w0 = a x_i - b x_j = c u_ij,  w1 = a x_j - b x_i = c u_ji
//   rho         dx_i += G0 - rho G1  with G0 = g_ij / s, G1 = g_ji / s
//   per direction d (0: u_ij with alpha_ij, beta_ij; 1: u_ji with alpha_ji, beta_ji), with
//   A = alpha / (n s), B = beta / (n s):  G = A tanh u + B (1 - u^2) e^{-u^2/2}
//      = 2A r - A + Bq h exp2(-h),   h = w^2 - c^2,  r = 1 / (1 + e^{-2u}),
//   since c^2 = log2(e) / 2 makes exp2(-w^2) = e^{-1/2} exp2(-h) and B (1 - u^2) = -B h / c^2:
//   stored as (2A, -A, Bq = -B e^{-1/2} / c^2).
struct BwdPair {
  float a, b, rho;
  float a2[2], na[2], bq[2];
};
static_assert(sizeof(BwdPair) == 36, "BwdPair is read with scalar loads");

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
      p.bq[d] = (float)(-be * kExpMinusHalf / (kWScale * kWScale));
    }
  }
  bp[j * m_pad + i] = p;
}

// Hx-term coefficients per variable: (alpha^x_i, beta^x_i) / n.  One wave per variable: its
// lanes stride over k for sum_k G_ki - G_ik (FP64), then a wave sum.
__global__ __launch_bounds__(256) void bwd_var_kernel(const double* __restrict__ momx,
                                                      const double* __restrict__ G, int64_t m,
                                                      int64_t m_pad, int64_t n_eff,
                                                      float2* __restrict__ vx) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= m_pad) return;
  double c = 0.0;
  if (i < m)
    for (int64_t k = lane; k < m; k += 64) c += G[k * m + i] - G[i * m + k];
  c = wave_sum_d(c);
  if (lane != 0) return;
  float2 v = make_float2(0.f, 0.f);
  if (i < m) {
    const double inv_n = 1.0 / (double)n_eff;
    v.x = (float)(-2.0 * kK1 * (momx[2 * i] - kGamma) * c * inv_n);
    v.y = (float)(-2.0 * kK2 * momx[2 * i + 1] * c * inv_n);
  }
  vx[i] = v;
}

// One direction's pre-scaled dL/du from w = c u (constants as stored in BwdPair):
//   2A r - A + Bq h exp2(-h),  h = w^2 - c^2 (one rounding),  r = 1 / (1 + exp2(kTScale w))
//   (exact limits 0 and 1 for large |w|)
__device__ __forceinline__ float dir_grad(float w, float a2, float na, float bq) {
  const float h = fmaf(w, w, -(float)(kWScale * kWScale));
  const float e = __builtin_amdgcn_exp2f(-h);
  const float t = __builtin_amdgcn_exp2f(w * (float)kTScale);
  const float r = __builtin_amdgcn_rcpf(1.f + t);
  return fmaf(a2, r, fmaf(bq * h, e, na));
}

// A lane's kBSpl consecutive samples: FP32 loads and stores, FP64 LDS sums.
typedef std::conditional_t<kBSpl == 2, double2, double> SlotT;
static_assert(kBSpl == 1 || kBSpl == 2, "one or two samples per lane");
__device__ __forceinline__ void load_spl(const float* p, float* dst) {
  if constexpr (kBSpl == 2) {
    const float2 f = *reinterpret_cast<const float2*>(p);
    dst[0] = f.x;
    dst[1] = f.y;
  } else {
    dst[0] = *p;
  }
}
__device__ __forceinline__ void store_spl(float* p, const double* v) {
  if constexpr (kBSpl == 2)
    *reinterpret_cast<float2*>(p) = make_float2((float)v[0], (float)v[1]);
  else
    *p = (float)v[0];
}
__device__ __forceinline__ void slot_add(double2& s, const double* v) {
  s.x += v[0];
  s.y += v[1];
}
__device__ __forceinline__ void slot_add(double& s, const double* v) { s += v[0]; }
__device__ __forceinline__ void slot_get(const double2& s, double* v) {
  v[0] = s.x;
  v[1] = s.y;
}
__device__ __forceinline__ void slot_get(double s, double* v) { v[0] = s; }

// Both terms of the pair (i, j) at one sample (x = x_i(t), y = x_j(t), constants of the
// ordered pair (i, j)): dx_i += g_ij / s - rho g_ji / s, dx_j += g_ji / s - rho g_ij / s, and
// the rho chain's (g_ij / s)(c u_ji) + (g_ji / s)(c u_ij) (= -R_ij c / s summed over t).
__device__ __forceinline__ void pair_terms(const BwdPair& c, float x, float y, double& ai,
                                           double& aj, float& r) {
  const float w0 = fmaf(x, c.a, -(y * c.b));      // c u_ij
  const float w1 = fmaf(y, c.a, -(x * c.b));      // c u_ji
  const float g0 = dir_grad(w0, c.a2[0], c.na[0], c.bq[0]);   // g_ij / s
  const float g1 = dir_grad(w1, c.a2[1], c.na[1], c.bq[1]);   // g_ji / s
  // dL/dx_i(t) is summed in FP64: the Hx term and the sum of the pair terms nearly cancel
  // (each pair term follows Hr_ij - Hx_i, a small difference), so FP32 partial sums would
  // carry rounding at many times the scale of the result.
  ai += (double)fmaf(-c.rho, g1, g0);
  aj += (double)fmaf(-c.rho, g0, g1);
  r = fmaf(g0, w1, fmaf(g1, w0, r));
}

// Row of Pd holding partial p (p <= v / 32) of variable v: the partials of one variable are
// consecutive, block B of variables holding B + 1 partials per variable.
__host__ __device__ inline int64_t pd_row(int64_t v, int64_t p) {
  const int64_t B = v / kTK, r = v - B * kTK;
  return kTK * B * (B + 1) / 2 + r * (B + 1) + p;
}
__host__ __device__ inline int64_t pd_rows(int64_t nblk) { return kTK * nblk * (nblk + 1) / 2; }

// One workgroup (8 waves) per (row a of the 32-variable blocks, 128-sample chunk); rows in
// increasing a (the longest first).  The workgroup visits the tiles (a, b), b = a .. P - 1.
// Lane l holds samples chunk * 128 + 2 l + [0, 2).  Wave w owns rows a * 32 + 4 w + [0, 4), their
// sums in registers over the whole row of tiles.  In round r of a tile it takes the rows
// b * 32 + 4 y + [0, 4), y = (w + r) mod 8: within a round every y has one wave, so the partner
// sums are added to LDS rows with one writer, and a barrier orders the rounds.  Off-diagonal
// tiles run 8 rounds; the diagonal tile (b = a) runs the pairs inside the own block (round 0)
// and the rotations 1..4 (rotation 4 by waves 0..3 only), so each unordered pair is visited
// once.  After a tile, each wave moves its 4 LDS rows out: into its own sums (b = a) or to the
// partial a of the variables of b.  The launch covers chunks [chunk0, chunk0 + nchunk) (a window
// of the samples); outputs, FP32, with t - chunk0 * 128 as the column (row stride ldp):
// partial a of each variable of blocks a .. P - 1 (rows pd_row; for block a the own sums with
// the Hx term), and Rp[chunk][i][j] for each pair, i < j < m.  Pair constants are stored
// transposed, bp[j * m_pad + i], so the 4 own rows of one partner are contiguous (scalar loads).
__global__ __launch_bounds__(kTW * 64) void bwd_tile_kernel(
    const float* __restrict__ Xs, int64_t n_pad, const BwdPair* __restrict__ bp,
    const float2* __restrict__ vx, int64_t m_pad, int64_t m, int P, int64_t chunk0,
    int64_t nchunk, float* __restrict__ Pd, int64_t ldp, float* __restrict__ Rp) {
  __shared__ SlotT slot[kTK][64];     // sums of the rows of block b: [row][lane] (32 KB)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int a = (int)((int64_t)blockIdx.x / nchunk);
  const int64_t chunk = chunk0 + ((int64_t)blockIdx.x - (int64_t)a * nchunk);
  const int64_t ia0 = (int64_t)a * kTK + kTT * wave;
  const int64_t tb = chunk * kBChunk + kBSpl * lane;
  float* const pd = Pd + (tb - chunk0 * kBChunk);     // this lane's column of the window
  auto load_x = [&](int64_t row, float* dst) { load_spl(Xs + row * n_pad + tb, dst); };
  float xa[kTT][kBSpl];
  double acc[kTT][kBSpl];
#pragma unroll
  for (int ii = 0; ii < kTT; ++ii) {
    load_x(ia0 + ii, xa[ii]);
    // Hx term: the column's own entropy moments
    const float2 cx = vx[ia0 + ii];
#pragma unroll
    for (int e = 0; e < kBSpl; ++e)
      acc[ii][e] = (double)dir_grad(xa[ii][e] * (float)kWScale, 2.f * cx.x, -cx.x,
                                    cx.y * (float)(-kExpMinusHalf / (kWScale * kWScale)));
    slot[kTT * wave + ii][lane] = SlotT{};
  }

  for (int b = a; b < P; ++b) {
    __syncthreads();     // the LDS rows are clear
    const bool diag = b == a;
    const int nround = diag ? kTW / 2 + 1 : kTW;
    for (int r = 0; r < nround; ++r) {
      const int y = (wave + r) & (kTW - 1);
      const bool self = diag && r == 0;
      const bool active = !diag || r < kTW / 2 || wave < kTW / 2;
      if (active) {
        const int64_t ib0 = (int64_t)b * kTK + kTT * y;
        float rs[kTT * kTT];   // rho-chain partial of pair (ii, jj) at index 4 ii + jj
#pragma unroll
        for (int k = 0; k < kTT * kTT; ++k) rs[k] = 0.f;
        if (self) {
          // pairs inside the own block, ii < jj: both sides are own rows
#pragma unroll
          for (int jj = 1; jj < kTT; ++jj) {
            const BwdPair* c4 = bp + (ia0 + jj) * m_pad + ia0;
#pragma unroll
            for (int ii = 0; ii < jj; ++ii) {
              const BwdPair c = c4[ii];
#pragma unroll
              for (int e = 0; e < kBSpl; ++e)
                pair_terms(c, xa[ii][e], xa[jj][e], acc[ii][e], acc[jj][e], rs[kTT * ii + jj]);
            }
          }
        } else {
          float xb[kTT][kBSpl];
          double accb[kTT][kBSpl];
#pragma unroll
          for (int jj = 0; jj < kTT; ++jj) {
            load_x(ib0 + jj, xb[jj]);
#pragma unroll
            for (int e = 0; e < kBSpl; ++e) accb[jj][e] = 0.0;
          }
#pragma unroll
          for (int jj = 0; jj < kTT; ++jj) {
            const BwdPair* c4 = bp + (ib0 + jj) * m_pad + ia0;
#pragma unroll
            for (int ii = 0; ii < kTT; ++ii) {
              const BwdPair c = c4[ii];
#pragma unroll
              for (int e = 0; e < kBSpl; ++e)
                pair_terms(c, xa[ii][e], xb[jj][e], acc[ii][e], accb[jj][e], rs[kTT * ii + jj]);
            }
          }
#pragma unroll
          for (int jj = 0; jj < kTT; ++jj) {
            SlotT sv = slot[kTT * y + jj][lane];
            slot_add(sv, accb[jj]);
            slot[kTT * y + jj][lane] = sv;
          }
        }
        const float v = wave_reduce_scatter16(rs);   // sum over the chunk of pair lane >> 2
        if ((lane & 3) == 0) {
          const int p = lane >> 2, ii = p / kTT, jj = p % kTT;
          const int64_t i = ia0 + ii, j = ib0 + jj;
          if (i < m && j < m && (!self || ii < jj)) {
            const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
            Rp[(chunk * m + lo) * m + hi] = v;
          }
        }
      }
      __syncthreads();
    }
    // this wave's 4 LDS rows: into the own sums (b = a) or out as partial a of block b
#pragma unroll
    for (int jj = 0; jj < kTT; ++jj) {
      const SlotT sv = slot[kTT * wave + jj][lane];
      double v[kBSpl];
      slot_get(sv, v);
      if (diag) {
#pragma unroll
        for (int e = 0; e < kBSpl; ++e) acc[jj][e] += v[e];
      } else {
        store_spl(pd + pd_row((int64_t)b * kTK + kTT * wave + jj, a) * ldp, v);
      }
      slot[kTT * wave + jj][lane] = SlotT{};
    }
  }
#pragma unroll
  for (int ii = 0; ii < kTT; ++ii) store_spl(pd + pd_row(ia0 + ii, a) * ldp, acc[ii]);
}

// One window of the samples, columns [t0, t0 + nw) of dx: dx[v][t0 + t] = sum over the partials
// p = 0 .. v / 32 (in order) of row pd_row(v, p) of Pd (row stride ldp), in FP64; 4 consecutive
// samples a thread (nw, ldp, t0 and n_pad multiples of 4).
__global__ void bwd_reduce_kernel(const float* __restrict__ Pd, int64_t m_pad, int64_t ldp,
                                  int64_t nw, int64_t t0, int64_t n_pad,
                                  float* __restrict__ dx) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nq = nw / 4;
  if (q >= m_pad * nq) return;
  const int64_t v = q / nq, t = (q - v * nq) * 4;
  const int np = (int)(v / kTK) + 1;
  const float* src = Pd + pd_row(v, 0) * ldp + t;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  auto add = [&](const float4& x4) {
    s0 += x4.x;
    s1 += x4.y;
    s2 += x4.z;
    s3 += x4.w;
  };
  int p = 0;
  for (; p + 8 <= np; p += 8) {     // eight loads in flight, summed in order
    float4 x4[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x4[k] = *reinterpret_cast<const float4*>(src + (p + k) * ldp);
#pragma unroll
    for (int k = 0; k < 8; ++k) add(x4[k]);
  }
  for (; p < np; ++p) add(*reinterpret_cast<const float4*>(src + p * ldp));
  *reinterpret_cast<float4*>(dx + v * n_pad + t0 + t) =
      make_float4((float)s0, (float)s1, (float)s2, (float)s3);
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
  b.nblk = (int)ceil_div(m, kTK);
  b.m_pad = (int64_t)b.nblk * kTK;
  b.nchunk = ceil_div(n_eff, kBChunk);
  b.n_pad = b.nchunk * kBChunk;
  // sample windows of the pair pass, of equal length: its per-partner-block sums take at most
  // kPdBytes
  const int64_t per_chunk = pd_rows(b.nblk) * kBChunk * (int64_t)sizeof(float);
  const int64_t most = std::max<int64_t>(1, kPdBytes / per_chunk);
  b.win_chunks = b.nblk > 1 ? ceil_div(b.nchunk, ceil_div(b.nchunk, most)) : b.nchunk;
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
  // one block of variables: the tile pass writes dx directly
  w.Pd = b.nblk > 1 ? c.take<float>((size_t)pd_rows(b.nblk) * b.win_chunks * kBChunk) : w.dx;
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
    bwd_var_kernel<<<(unsigned)ceil_div(b.m_pad, 4), 256, 0, stream>>>(momx, G, m, b.m_pad,
                                                                      n_eff, w.vx);
    VL_LAUNCH_CHECK();
  }
  {
    // one block of variables: the tile pass writes dx directly (one window)
    const int64_t ldp = b.nblk > 1 ? b.win_chunks * kBChunk : b.n_pad;
    for (int64_t c0 = 0; c0 < b.nchunk; c0 += b.win_chunks) {
      const int64_t nc = std::min(b.win_chunks, b.nchunk - c0);
      {
        ProfileScope ps("backward_pairs", stream);
        bwd_tile_kernel<<<(unsigned)(b.nblk * nc), kTW * 64, 0, stream>>>(
            w.Xs, b.n_pad, w.bp, w.vx, b.m_pad, m, b.nblk, c0, nc, w.Pd, ldp, w.Rp);
        VL_LAUNCH_CHECK();
      }
      if (b.nblk > 1) {
        ProfileScope ps("backward_reduce", stream);
        const int64_t nq = b.m_pad * nc * kBChunk / 4;
        bwd_reduce_kernel<<<(unsigned)ceil_div(nq, 256), 256, 0, stream>>>(
            w.Pd, b.m_pad, ldp, nc * kBChunk, c0 * kBChunk, b.n_pad, w.dx);
        VL_LAUNCH_CHECK();
      }
    }
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
