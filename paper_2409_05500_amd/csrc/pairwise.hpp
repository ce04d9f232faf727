// Pairwise-statistic precompute: launch plan and workspace layout.
#pragma once
#include "common.hpp"

namespace vl {

struct PairwisePlan {
  bool comp = false;      // compensated moment sums, FP64 partials
  bool sliced = false;    // covariance from int8 slices (VL_PREC_SLICED)
  int64_t m = 0, n_eff = 0;
  int nt = 0;             // micro-tiles per side (4 variables each)
  int64_t m_pad = 0;      // nt * 4
  int64_t tiles = 0;      // nt (nt + 1) / 2 upper-triangular micro-tiles
  int nc = 0;             // sample chunks
  int chunk_len = 0;      // samples per chunk, multiple of 128
  int64_t n_pad = 0;      // nc * chunk_len >= n_eff
  int64_t items = 0;      // tiles * nc (one wave each)
  int64_t blocks = 0;     // ceil(items / 4) rounded up to a multiple of 8
};

struct PairwiseWs {
  double* mu = nullptr;       // m column means
  double* cov = nullptr;      // m x m covariance when the caller passes none
  double* scratch = nullptr;  // split partials of the column sums / Gram
  float* Xs = nullptr;        // m_pad x n_pad standardised, variable-major
  float2* coef = nullptr;     // m_pad x m_pad pair coefficients
  float* partU = nullptr;     // nc x m x m (plain sums)
  float* partB = nullptr;     // nc x m x m
  double* partU64 = nullptr;  // nc x m x m (compensated sums; in place of partU, partB)
  double* partB64 = nullptr;
  double* momx = nullptr;     // 2 m: E[log cosh x_i], E[x_i exp(-x_i^2/2)]
  int32_t* clist = nullptr;   // 2 tiles + 1: near-collinear tile flags, count, list
  int8_t* slices = nullptr;   // sliced covariance: slice planes of E's columns (stage 1)
  int32_t* ex = nullptr;      // m exponents
};

PairwisePlan plan_pairwise(int64_t n_eff, int64_t m, bool compensated = false,
                           bool sliced = false);
size_t scratch_doubles(const PairwisePlan& p);
// Total workspace bytes; with base != nullptr also fills *out with the carved pointers.
size_t pairwise_ws_bytes(const PairwisePlan& p, void* base, PairwiseWs* out);
// Standardise E with the given means and covariance diagonal into the variable-major Xs
// (m_pad x n_pad, zero padded).  n_pad >= n_eff, m_pad >= m.
// The launch also clears zero[0 .. nzero) (nullptr: nothing).
int standardize_to(const float* E, int64_t lde, int64_t n_eff, int64_t m, const double* mu,
                   const double* cov, float* Xs, int64_t n_pad, int64_t m_pad, int32_t* st,
                   hipStream_t stream, int32_t* zero = nullptr, int64_t nzero = 0);
// mom (nullable): 2 m^2 doubles, (A, B) per ordered pair, for tests and the backward pass.
// prec: the covariance's arithmetic (VL_PREC_FP32 or another precision, possibly with the
// VL_PAIRWISE_COMPENSATED bit, which the plan also carries).
int run_pairwise(const PairwisePlan& p, const PairwiseWs& w, const float* E, int64_t lde,
                 int prec, double* Hx, double* Hr, double* S, double* Cov, double* mom,
                 int32_t* st, hipStream_t stream);

}  // namespace vl
