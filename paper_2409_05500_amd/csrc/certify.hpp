// Certified ordering: Alg. 1 with the near-ties re-decided on FP64 scores (declarations).
#pragma once
#include "common.hpp"

namespace vl {

struct CertWs {
  double* mu = nullptr;        // m column means (FP64)
  double* inv_sd = nullptr;    // m inverse population standard deviations
  double* Hx = nullptr;        // m FP64 H(x_i)
  double* X64 = nullptr;       // m x n_eff standardised columns, FP64, variable-major
  int32_t* refined = nullptr;  // m flags: row recomputed in FP64
  int32_t* listed = nullptr;   // m flags: in the current round's list
  int32_t* list = nullptr;     // m: the rows in doubt this round
  int32_t* count = nullptr;    // 1
};

size_t cert_ws_bytes(int64_t n_eff, int64_t m, void* base, CertWs* out);

// S (m x m, FP64, antisymmetric) is updated in place: the rows (and columns) in doubt are
// replaced by FP64 recomputations from E.  Synchronises `stream` once per round.
int run_order_certified(const float* E, int64_t n_eff, int64_t m, int64_t lde, double* S,
                        double eps, int32_t* order, double* margin, int32_t* refined_out,
                        int64_t* n_refined, int64_t* rounds, const CertWs& w, int32_t* st,
                        hipStream_t stream);

}  // namespace vl
