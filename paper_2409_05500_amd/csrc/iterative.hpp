// The original iterative DirectLiNGAM ordering (declarations).
#pragma once
#include "common.hpp"

namespace vl {

struct IterWs {
  float* D[2] = {nullptr, nullptr};      // current data, n_eff x m (ld m), ping-pong
  int32_t* idx[2] = {nullptr, nullptr};  // original index of each current column, ping-pong
  int32_t* pick = nullptr;               // current-column index of this step's pick
  double* Hx = nullptr;                  // m
  double* Hr = nullptr;                  // m x m
  double* S = nullptr;                   // m x m
  double* Cov = nullptr;                 // m x m
  void* pw = nullptr;                    // the pairwise stage's workspace (largest plan)
  int32_t* osub = nullptr;               // hybrid: order of the remaining variables (m)
  double* M0 = nullptr;                  // hybrid: the lookup ordering's scratch (m)
};

// Workspace bytes for n_eff samples of m variables; with base != nullptr also carves *out.
size_t iter_ws_bytes(int64_t n_eff, int64_t m, void* base, IterWs* out);

// order (m) and margin (m) of the iterative search on E (n_eff x m, ld lde).  After k_exact
// picks (k_exact >= m - 1: none) the rest is ordered by the heuristic: one pairwise precompute
// on the refined data of the remaining variables and the lookup-only selection.
int run_order_iterative(const float* E, int64_t n_eff, int64_t m, int64_t lde, int prec,
                        int64_t k_exact, int32_t* order, double* margin, const IterWs& w,
                        int32_t* st, hipStream_t stream);

}  // namespace vl
