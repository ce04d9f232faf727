// Adaptive-lasso pruning of B0 / B_tau, the step after the fit that the paper names but does
// not specify.  Variable i (position k of the causal order) is regressed with intercept on its
// k predecessors at lag 0 and on all m variables at lags 1..p (d = k + m p columns).  The
// unpruned coefficients b are that regression's least-squares solution, so column j is scaled
// by |b_j| (adaptive lasso, Zou 2006, exponent 1).  The lasso path is the LARS path with the
// lasso modification (Efron, Hastie, Johnstone and Tibshirani 2004, Sec. 2 and Sec. 3.1), and
// the knot minimising BIC = T ln(RSS / T) + df ln T (df = nonzero coefficients) is kept.
//
// Everything the path needs is in one FP64 matrix: the centred cross-products C of the
// m (p + 1) lag-embedded columns, shared by all m regressions.  One workgroup follows one
// variable's path on it.  Its state lives in a region of global memory of its own:
//   Gi   inverse of the (unsigned) Gram of the active columns, updated by bordering when a
//        column joins and by the Schur complement when one leaves (O(|A|^2) each).  The
//        rank-one parts of up to kPruneDefer borderings are kept as a thin factor and applied
//        together, so a joining column costs one read of Gi (to form G_A^{-1} b) and Gi is
//        rewritten once per kPruneDefer joins (and before a column leaves);
//   q    G_A^{-1} s, bordered along with Gi (recomputed from Gi after a column leaves);
//   c    correlations z~_j^T r with the current residual, updated by c -= gamma a;
//   beta the scaled coefficients, best the coefficients of the best knot so far.
// The correlation of an active column is set to s_j C after every step (the equiangular
// property), and the residual sum of squares follows from the correlations:
//   RSS = y^T y - sum_{j in A} beta_j (c0_j + c_j).
// Numerical rules, shared with the FP64 reference: a step must exceed 1e-12 of the full step
// C / A_A; a column whose Schur complement against the active ones is <= 1e-12 of its squared
// norm is excluded; the path ends once C <= 1e-12 C_0, at the least-squares fit, or after the
// step limit (8 d by default).  Ties go to the lowest design column.
#include "prune.hpp"
#include "gram.hpp"
#include "profile.hpp"
#include "var_fit.hpp"

namespace vl {
namespace {

constexpr int kPT = 512;            // threads per variable
constexpr int kU = 8;               // independent loads in flight per thread (row updates)
constexpr int kUD = 16;             // independent loads in flight per thread (dot products)
constexpr int kPW = kPT / kWave;
constexpr double kGammaRel = 1e-12;
constexpr double kCollinearRel = 1e-12;
constexpr double kStopRel = 1e-12;
constexpr int kNone = 0x7fffffff;

struct PruneArgs {
  const double* C;
  int64_t ldc, m, T, cap;
  int p;
  const int32_t* order;
  const double* B0;
  const double* Bl;
  double* regions;
  double* B0o;
  double* Blo;
  int32_t* info;
  int32_t* st;
};

// sum_k M[k ld + r] v[k] over k < n (a row of a column-major matrix times a vector), with kU
// loads in flight; a fixed summation order, so repeated calls give the same bits.
__device__ inline double col_dot(const double* __restrict__ M, int64_t ld, int r,
                                 const double* __restrict__ v, int n) {
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int k = 0;
  for (; k + kUD <= n; k += kUD) {
    double x[kUD];
#pragma unroll
    for (int u = 0; u < kUD; ++u) x[u] = M[(int64_t)(k + u) * ld + r];
#pragma unroll
    for (int u = 0; u < kUD; ++u) s[u & 3] += x[u] * v[k + u];
  }
  for (; k < n; ++k) s[0] += M[(int64_t)k * ld + r] * v[k];
  return (s[0] + s[1]) + (s[2] + s[3]);
}

// sum_r Cj[col[r] ld] w[r] over r < n (a gathered row of the covariance times a vector)
__device__ inline double gather_dot(const double* __restrict__ Cj, int64_t ld,
                                    const int* __restrict__ col, const double* __restrict__ w,
                                    int n) {
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int r = 0;
  for (; r + kUD <= n; r += kUD) {
    double x[kUD];
#pragma unroll
    for (int u = 0; u < kUD; ++u) x[u] = Cj[(int64_t)col[r + u] * ld];
#pragma unroll
    for (int u = 0; u < kUD; ++u) s[u & 3] += x[u] * w[r + u];
  }
  for (; r < n; ++r) s[0] += Cj[(int64_t)col[r] * ld] * w[r];
  return (s[0] + s[1]) + (s[2] + s[3]);
}

// Row x of a column-major matrix: M[y ld + x] += a f[y] for y < n, kU loads in flight.
__device__ inline void row_axpy(double* __restrict__ M, int64_t ld, int x, double a,
                                const double* __restrict__ f, int n) {
  int y = 0;
  for (; y + kU <= n; y += kU) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = M[(int64_t)(y + u) * ld + x];
#pragma unroll
    for (int u = 0; u < kU; ++u) M[(int64_t)(y + u) * ld + x] = v[u] + a * f[y + u];
  }
  for (; y < n; ++y) M[(int64_t)y * ld + x] += a * f[y];
}

// Workgroup sum, the same bits in every thread (lane 0 of each wave, waves in a fixed order).
__device__ inline double wg_sum(double v, double* red) {
  v = wave_sum_d(v);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int w = 1; w < kPW; ++w) s += red[w];
  return s;
}

__device__ inline void take_min(double& g, int& j, double g2, int j2) {
  if (g2 < g || (g2 == g && j2 < j)) {
    g = g2;
    j = j2;
  }
}

// Workgroup (value, index) minimum, lowest index on ties; exact, so the same in every thread.
__device__ inline void wg_argmin(double& g, int& j, double* rg, int* rj) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) take_min(g, j, __shfl_xor(g, s, kWave), __shfl_xor(j, s, kWave));
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) {
    rg[threadIdx.x / kWave] = g;
    rj[threadIdx.x / kWave] = j;
  }
  __syncthreads();
  g = rg[0];
  j = rj[0];
#pragma unroll
  for (int w = 1; w < kPW; ++w) take_min(g, j, rg[w], rj[w]);
}

// Values every thread of the workgroup holds alike (read back from LDS after a reduction),
// declared uniform so they live in scalar registers and branch without divergence.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t uni64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Workgroup sums of kPruneDefer values at once, the same bits in every thread.
__device__ inline void wg_sum_vec(double (&v)[kPruneDefer], double* red) {
#pragma unroll
  for (int q = 0; q < kPruneDefer; ++q) v[q] = wave_sum_d(v[q]);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
    for (int q = 0; q < kPruneDefer; ++q) red[q * kPW + threadIdx.x / kWave] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPruneDefer; ++q) {
    double s = red[q * kPW];
    for (int w = 1; w < kPW; ++w) s += red[q * kPW + w];
    v[q] = s;
  }
}

constexpr int kFC = 256;  // rows of the deferred factor staged in LDS per flush chunk

// Gi(x, y) += sum_q U_q[x] w_q U_q[y] for x, y < n: the deferred rank-one terms applied in one
// read and one write of Gi.  us: kPruneDefer x kFC doubles of LDS.
__device__ inline void flush_deferred(double* __restrict__ Gi, int64_t dA,
                                      const double* __restrict__ U, int64_t ldu,
                                      const double* __restrict__ w, int nU, int n,
                                      double* __restrict__ us) {
  for (int y0 = 0; y0 < n; y0 += kFC) {
    const int ny = min(kFC, n - y0);
    __syncthreads();
    for (int e = threadIdx.x; e < kPruneDefer * kFC; e += kPT) {
      const int q = e / kFC, yy = e % kFC;
      us[e] = q < nU && yy < ny ? U[(int64_t)q * ldu + y0 + yy] * w[q] : 0.0;
    }
    __syncthreads();
    for (int x = threadIdx.x; x < n; x += kPT) {
      double ux[kPruneDefer];
#pragma unroll
      for (int q = 0; q < kPruneDefer; ++q) ux[q] = q < nU ? U[(int64_t)q * ldu + x] : 0.0;
      constexpr int kF = 4;  // rows of Gi in flight per group (register budget)
      int yy = 0;
      for (; yy + kF <= ny; yy += kF) {
        double v[kF];
#pragma unroll
        for (int u = 0; u < kF; ++u) v[u] = Gi[(int64_t)(y0 + yy + u) * dA + x];
#pragma unroll
        for (int u = 0; u < kF; ++u) {
          double sum = 0.0;
#pragma unroll
          for (int q = 0; q < kPruneDefer; ++q) sum += ux[q] * us[q * kFC + yy + u];
          Gi[(int64_t)(y0 + yy + u) * dA + x] = v[u] + sum;
        }
      }
      for (; yy < ny; ++yy) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < kPruneDefer; ++q) sum += ux[q] * us[q * kFC + yy];
        Gi[(int64_t)(y0 + yy) * dA + x] += sum;
      }
    }
  }
  __syncthreads();
}

// permutation check of the order (one workgroup; m <= 4096)
__global__ __launch_bounds__(256) void prune_check_order_kernel(const int32_t* __restrict__ order,
                                                                int64_t m, int32_t* st) {
  __shared__ int seen[4096];
  for (int64_t e = threadIdx.x; e < m; e += 256) seen[e] = 0;
  __syncthreads();
  for (int64_t e = threadIdx.x; e < m; e += 256) {
    const int v = order[e];
    if (v < 0 || v >= m) raise_status(st, VL_ERR_INVALID_ARG);
    else atomicAdd(&seen[v], 1);
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < m; e += 256)
    if (seen[e] != 1) raise_status(st, VL_ERR_INVALID_ARG);
}

__global__ __launch_bounds__(kPT) void prune_lars_kernel(PruneArgs a) {
  __shared__ double red[kPW];
  __shared__ double rg[kPW];
  __shared__ int rj[kPW];
  __shared__ int slot;
  __shared__ double redv[kPruneDefer * kPW];
  __shared__ double wq[kPruneDefer];  // weights 1 / delta of the deferred terms
  __shared__ double us[kPruneDefer * kFC];
  const int t = threadIdx.x;
  const int64_t m = a.m, mp = m * a.p, ldc = a.ldc;
  const int64_t pos = m - 1 - (int64_t)blockIdx.x;  // the longest designs start first
  const int i = min(max(a.order[pos], 0), (int)m - 1);

  // this variable's region: after the regions of positions 0 .. pos-1
  double off = 0.0;
  for (int64_t k = t; k < pos; k += kPT) off += (double)prune_region_doubles(k + mp, a.cap);
  const int64_t base = uni64((int64_t)wg_sum(off, red));
  const int64_t d = pos + mp;
  const int64_t dA = prune_active_cap(d, a.cap);
  double* Gi = a.regions + base;
  double* sc = Gi + dA * dA;
  double* c0 = sc + d;
  double* c = c0 + d;
  double* av = c + d;
  double* beta = av + d;
  double* best = beta + d;
  double* sv = best + d;  // sign of each active slot
  double* qv = sv + d;    // G_A^{-1} s of the active slots
  double* dd = qv + d;    // direction of each active slot
  double* bv = dd + d;    // scaled direction, then the bordering column
  double* gn = bv + d;    // G_A^{-1} times the bordering column
  double* U = gn + d;     // deferred rank-one terms of Gi, kPruneDefer columns of d
  int* idx = reinterpret_cast<int*>(U + (int64_t)kPruneDefer * d);  // column of C per column
  int* state = idx + d;                       // 0 inactive, 1 active, 2 excluded
  int* act = state + d;                       // design column of each active slot
  int* ac = act + d;                          // its column of C

  // design columns: lag-0 predecessors in order, then (tau, k) for tau = 1..p, k = 0..m-1
  double g0 = INFINITY, nkeep = 0.0;
  int j0 = kNone;
  for (int64_t j = t; j < d; j += kPT) {
    int cj;
    double bj;
    if (j < pos) {
      const int v = min(max(a.order[j], 0), (int)m - 1);
      cj = v;
      bj = a.B0[(int64_t)i * m + v];
    } else {
      const int64_t jj = j - pos, tau = jj / m + 1, k = jj % m;
      cj = (int)(m * tau + k);
      bj = a.Bl[(tau - 1) * m * m + (int64_t)i * m + k];
    }
    const double s = fabs(bj);
    const double gjj = s * s * a.C[(int64_t)cj * ldc + cj];
    const double cj0 = s * a.C[(int64_t)cj * ldc + i];
    idx[j] = cj;
    sc[j] = s;
    c0[j] = cj0;
    c[j] = cj0;
    beta[j] = 0.0;
    best[j] = 0.0;
    const bool ok = s > 0.0 && gjj > 0.0;
    state[j] = ok ? 0 : 2;
    nkeep += s > 0.0 ? 1.0 : 0.0;
    if (ok) take_min(g0, j0, -fabs(cj0), (int)j);
  }
  const int64_t n_keep = uni((int)wg_sum(nkeep, red));
  wg_argmin(g0, j0, rg, rj);
  j0 = uni(j0);
  const double C0 = j0 == kNone ? 0.0 : -g0;
  const double T = (double)a.T, lnT = log(T);
  const double yy = a.C[(int64_t)i * ldc + i];
  double best_bic = T * log(yy / T);
  int best_knot = 0, best_df = 0, steps = 0, nA = 0;
  const int64_t cap = a.cap > 0 ? a.cap : 8 * n_keep;
  double Cc = C0;
  if (C0 > 0.0) {
    __syncthreads();
    if (t == 0) {
      const int cj = idx[j0];
      Gi[0] = 1.0 / (sc[j0] * sc[j0] * a.C[(int64_t)cj * ldc + cj]);
      act[0] = j0;
      ac[0] = cj;
      sv[0] = c[j0] >= 0.0 ? 1.0 : -1.0;
      qv[0] = sv[0] * Gi[0];
      state[j0] = 1;
    }
    nA = 1;
    __syncthreads();
  }

  // The inverse of the active Gram is Gi + sum_{q < nU} U_q wq[q] U_q^T: the rank-one parts of
  // the last nU borderings are kept as columns of U (zero in the rows of slots added after
  // them) and applied to Gi every kPruneDefer borderings, or before a column leaves.
  int nU = 0;
  while (nA > 0 && steps < cap) {
    // A_A = (s^T q)^(-1/2), direction dd = A_A q
    double part = 0.0;
    for (int r = t; r < nA; r += kPT) part += sv[r] * qv[r];
    const double AA = 1.0 / sqrt(wg_sum(part, red));
    for (int r = t; r < nA; r += kPT) {
      const double w = AA * qv[r];
      dd[r] = w;
      bv[r] = sc[act[r]] * w;
    }
    __syncthreads();
    // a = Z~^T u for the inactive columns, and the first of them to reach the active
    // correlation (gamma^)
    const double full = Cc / AA, tol = kGammaRel * full;
    double gh = INFINITY;
    int jh = kNone;
    for (int64_t j = t; j < d; j += kPT) {
      if (state[j] != 0) continue;
      const double aj = sc[j] * gather_dot(a.C + idx[j], ldc, ac, bv, nA), cj = c[j];
      av[j] = aj;
      double den = AA - aj;
      if (den != 0.0) {
        const double g = (Cc - cj) / den;
        if (isfinite(g) && g > tol) take_min(gh, jh, g, (int)j);
      }
      den = AA + aj;
      if (den != 0.0) {
        const double g = (Cc + cj) / den;
        if (isfinite(g) && g > tol) take_min(gh, jh, g, (int)j);
      }
    }
    wg_argmin(gh, jh, rg, rj);
    jh = uni(jh);
    // first active coefficient to change sign (gamma~)
    double gt = INFINITY;
    int lt = kNone;
    for (int r = t; r < nA; r += kPT) {
      const int l = act[r];
      if (beta[l] != 0.0 && dd[r] != 0.0) {
        const double g = -beta[l] / dd[r];
        if (g > tol) take_min(gt, lt, g, l);
      }
    }
    wg_argmin(gt, lt, rg, rj);
    lt = uni(lt);
    if (jh == kNone) gh = full;
    int event;
    double gamma;
    if (gt < gh) {
      event = -1;
      gamma = gt;
    } else if (jh != kNone) {
      event = 1;
      gamma = gh;
    } else {
      event = 0;
      gamma = full;
    }
    event = uni(event);
    // move along the direction
    for (int r = t; r < nA; r += kPT) beta[act[r]] += gamma * dd[r];
    for (int64_t j = t; j < d; j += kPT)
      if (state[j] == 0) c[j] -= gamma * av[j];
    Cc -= gamma * AA;
    for (int r = t; r < nA; r += kPT) c[act[r]] = sv[r] * Cc;
    __syncthreads();

    if (event == -1) {
      if (nU > 0) {
        flush_deferred(Gi, dA, U, d, wq, nU, nA, us);
        nU = 0;
      }
      // slot of the leaving column; swap it with the last slot, then take the Schur complement
      for (int r = t; r < nA; r += kPT)
        if (act[r] == lt) slot = r;
      __syncthreads();
      const int r0 = uni(slot), L = nA - 1;
      if (r0 != L) {
        for (int x = t; x < nA; x += kPT) {  // rows
          const double u = Gi[(int64_t)x * dA + r0];
          Gi[(int64_t)x * dA + r0] = Gi[(int64_t)x * dA + L];
          Gi[(int64_t)x * dA + L] = u;
        }
        __syncthreads();
        for (int x = t; x < nA; x += kPT) {  // columns
          const double u = Gi[(int64_t)r0 * dA + x];
          Gi[(int64_t)r0 * dA + x] = Gi[(int64_t)L * dA + x];
          Gi[(int64_t)L * dA + x] = u;
        }
        __syncthreads();
        if (t == 0) {
          const int ta = act[r0], tc = ac[r0];
          const double ts = sv[r0];
          act[r0] = act[L];
          ac[r0] = ac[L];
          sv[r0] = sv[L];
          act[L] = ta;
          ac[L] = tc;
          sv[L] = ts;
        }
      }
      __syncthreads();
      // row L of the inverse over the pivot, then Gi(x, y) -= Gi(x, L) Gi(L, y) / Gi(L, L)
      const double piv = Gi[(int64_t)L * dA + L];
      for (int y = t; y < L; y += kPT) dd[y] = Gi[(int64_t)y * dA + L] / piv;
      __syncthreads();
      for (int x = t; x < L; x += kPT) row_axpy(Gi, dA, x, -Gi[(int64_t)L * dA + x], dd, L);
      if (t == 0) {
        beta[lt] = 0.0;
        state[lt] = 0;
      }
      nA = L;
      __syncthreads();
      for (int r = t; r < nA; r += kPT) qv[r] = col_dot(Gi, dA, r, sv, nA);
      __syncthreads();
    } else if (event == 1) {
      // border the inverse with the joining column k (or exclude it when collinear)
      const int k = jh, ck = idx[k];
      const double sk = sc[k];
      for (int r = t; r < nA; r += kPT) bv[r] = sc[act[r]] * sk * a.C[(int64_t)ac[r] * ldc + ck];
      __syncthreads();
      // g = G_A^{-1} b = Gi b + sum_q U_q wq[q] (U_q^T b): one read of Gi
      double tv[kPruneDefer];
#pragma unroll
      for (int q = 0; q < kPruneDefer; ++q) tv[q] = 0.0;
      for (int r = t; r < nA; r += kPT) {
        const double br = bv[r];
#pragma unroll
        for (int q = 0; q < kPruneDefer; ++q)
          if (q < nU) tv[q] += U[(int64_t)q * d + r] * br;
      }
      wg_sum_vec(tv, redv);
#pragma unroll
      for (int q = 0; q < kPruneDefer; ++q) tv[q] = q < nU ? tv[q] * wq[q] : 0.0;
      double bg = 0.0;
      for (int r = t; r < nA; r += kPT) {
        double g = col_dot(Gi, dA, r, bv, nA);
#pragma unroll
        for (int q = 0; q < kPruneDefer; ++q)
          if (q < nU) g += U[(int64_t)q * d + r] * tv[q];
        gn[r] = g;
        bg += bv[r] * g;
      }
      const double gkk = sk * sk * a.C[(int64_t)ck * ldc + ck];
      const double delta = gkk - wg_sum(bg, red);
      if (delta <= kCollinearRel * gkk) {
        if (t == 0) state[k] = 2;
      } else {
        // border: G'^{-1} = [[Gi + g g^T / delta, -g / delta], [-g^T / delta, 1 / delta]]
        // (the g g^T / delta term deferred); q' = [q + g (g^T s - s_k) / delta,
        // (s_k - g^T s) / delta]
        const double rd = 1.0 / delta;
        const double sk1 = c[k] >= 0.0 ? 1.0 : -1.0;
        double gp = 0.0;
        for (int x = t; x < nA; x += kPT) gp += gn[x] * sv[x];
        const double gs = wg_sum(gp, red);
        for (int x = t; x < nA; x += kPT) {
          Gi[(int64_t)nA * dA + x] = -gn[x] * rd;
          Gi[(int64_t)x * dA + nA] = -gn[x] * rd;
          qv[x] += gn[x] * ((gs - sk1) * rd);
          U[(int64_t)nU * d + x] = gn[x];
        }
        if (t == 0) {
          Gi[(int64_t)nA * dA + nA] = rd;
          act[nA] = k;
          ac[nA] = ck;
          sv[nA] = sk1;
          qv[nA] = (sk1 - gs) * rd;
          state[k] = 1;
          for (int q = 0; q <= nU; ++q) U[(int64_t)q * d + nA] = 0.0;
          wq[nU] = rd;
        }
        ++nU;
        ++nA;
      }
      __syncthreads();
      if (nU == kPruneDefer) {
        flush_deferred(Gi, dA, U, d, wq, nU, nA, us);
        nU = 0;
      }
    }
    ++steps;
    // the knot: RSS from the correlations, df = nonzero coefficients
    double rp = 0.0, nz = 0.0;
    for (int r = t; r < nA; r += kPT) {
      const int l = act[r];
      rp += beta[l] * (c0[l] + c[l]);
      nz += beta[l] != 0.0 ? 1.0 : 0.0;
    }
    const double rss = yy - wg_sum(rp, red);
    const int df = (int)wg_sum(nz, red);
    const double bic = T * log(rss / T) + (double)df * lnT;
    if (bic < best_bic) {
      best_bic = bic;
      best_knot = steps;
      best_df = df;
      for (int64_t j = t; j < d; j += kPT) best[j] = beta[j];
    }
    __syncthreads();
    if (event == 0 || Cc <= kStopRel * C0) break;
  }

  // outputs: row i of B0 (predecessors only) and of every B_tau
  double* rowB0 = a.B0o + (int64_t)i * m;
  for (int64_t v = t; v < m; v += kPT) rowB0[v] = 0.0;
  __syncthreads();
  for (int64_t j = t; j < d; j += kPT) {
    const double v = best[j] * sc[j];
    if (j < pos) {
      rowB0[idx[j]] = v;
    } else {
      const int64_t jj = j - pos, tau = jj / m + 1, k = jj % m;
      a.Blo[(tau - 1) * m * m + (int64_t)i * m + k] = v;
    }
  }
  if (a.info && t == 0) {
    a.info[3 * i] = steps;
    a.info[3 * i + 1] = best_knot;
    a.info[3 * i + 2] = best_df;
  }
}

}  // namespace

size_t prune_ws_bytes(int64_t n, int64_t m, int p, int64_t cap, void* base, PruneWs* out) {
  Carver c(base);
  PruneWs w;
  const int64_t nc = m * (p + 1);
  w.colmap = c.take<int64_t>(nc);
  w.mu = c.take<double>(nc);
  w.C = c.take<double>(nc * nc);
  w.scratch = c.take<double>(lag_cov_scratch_doubles(n, m, p));
  int64_t tot = 0;
  for (int64_t k = 0; k < m; ++k) tot += prune_region_doubles(k + m * p, cap);
  w.regions = c.take<double>(tot);
  if (out) *out = w;
  return c.used;
}

int run_prune(int64_t n, int64_t m, int p, const PruneWs& w, const float* X, int64_t ldx,
              const int32_t* order, const double* B0, const double* Blag, int64_t cap,
              double* B0_out, double* Blag_out, int32_t* info, int32_t* st, hipStream_t stream) {
  ProfileScope ps("prune", stream);
  const int64_t nc = m * (p + 1);
  int rc = lag_covariance(n, m, p, X, ldx, w.colmap, w.mu, w.C, w.scratch, st, stream);
  if (rc) return rc;
  prune_check_order_kernel<<<1, 256, 0, stream>>>(order, m, st);
  VL_LAUNCH_CHECK();
  PruneArgs a;
  a.C = w.C;
  a.ldc = nc;
  a.m = m;
  a.T = n - p;
  a.cap = cap;
  a.p = p;
  a.order = order;
  a.B0 = B0;
  a.Bl = Blag;
  a.regions = w.regions;
  a.B0o = B0_out;
  a.Blo = Blag_out;
  a.info = info;
  a.st = st;
  prune_lars_kernel<<<(unsigned)m, kPT, 0, stream>>>(a);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

}  // namespace vl
