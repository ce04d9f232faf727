// Gradient of the pairwise score: launch plan and workspace layout.
#pragma once
#include "common.hpp"
#include "pairwise.hpp"

namespace vl {

struct BwdPair;   // per ordered pair constants of the transcendental pass (backward.hip)

struct BwdPlan {
  PairwisePlan fwd;        // forward recompute
  int nblk = 0;            // 32-variable blocks (tile sides of the pair pass)
  int64_t m_pad = 0;       // nblk * 32
  int64_t nchunk = 0;      // 128-sample chunks
  int64_t n_pad = 0;       // nchunk * 128
  int64_t win_chunks = 0;  // chunks per launch of the pair pass (bounds its partial sums)
};

struct BwdWs {
  PairwiseWs fwd;
  double* Hx = nullptr;    // forward outputs (m, m^2, m^2, m^2)
  double* Hr = nullptr;
  double* S = nullptr;
  double* cov = nullptr;
  double* mom = nullptr;   // 2 m^2: (A, B) per ordered pair
  float* Xs = nullptr;     // m_pad x n_pad standardised, variable-major, zero padded
  BwdPair* bp = nullptr;   // m_pad x m_pad
  float2* vx = nullptr;    // m_pad: Hx-term coefficients
  float* dx = nullptr;     // m_pad x n_pad: dL/dx
  float* Pd = nullptr;     // nblk x m_pad x (win_chunks * 128): dL/dx sums per partner block,
                           // one sample window (dx itself if nblk = 1)
  float* Rp = nullptr;     // nchunk x m x m: per-chunk dL/drho partials
  float* Rf = nullptr;     // m_pad x m_pad: dL/drho / n
  double* sums = nullptr;  // 2 m: sum dx, sum dx x
};

BwdPlan plan_backward(int64_t n_eff, int64_t m);
size_t bwd_ws_bytes(const BwdPlan& b, void* base, BwdWs* out);
// saved (nullable): the forward's statistics, [A,B per ordered pair (2 m^2) | A,B per
// variable (2 m) | covariance (m^2) | means (m)]; NULL recomputes them.
int run_backward(const BwdPlan& b, const BwdWs& w, const float* E, int64_t lde, int prec,
                 const double* saved, const double* G, float* dE, int64_t ldde, int32_t* st,
                 hipStream_t stream);

}  // namespace vl
