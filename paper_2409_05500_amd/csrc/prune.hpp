// Adaptive-lasso pruning of B0 / B_tau (declarations).
#pragma once
#include "common.hpp"

namespace vl {

struct PruneWs {
  int64_t* colmap = nullptr;  // m (p+1) sample offsets of the lag-embedded columns
  double* mu = nullptr;       // their means
  double* C = nullptr;        // m (p+1) square centred cross-products
  double* scratch = nullptr;  // split partials of the covariance
  double* regions = nullptr;  // one LARS state region per variable
};

// Active-set capacity of a path over d columns with at most cap steps (cap 0: no limit).
__host__ __device__ inline int64_t prune_active_cap(int64_t d, int64_t cap) {
  return cap > 0 && cap + 1 < d ? cap + 1 : d;
}
// Rank-one updates of the inverse of the active Gram kept aside and applied together.
constexpr int kPruneDefer = 8;

// Doubles of the region of a variable with d design columns: the inverse of the active Gram
// (capacity^2), eleven FP64 vectors of d, the kPruneDefer deferred columns of d and four int32
// vectors of d.
__host__ __device__ inline int64_t prune_region_doubles(int64_t d, int64_t cap) {
  const int64_t a = prune_active_cap(d, cap);
  return round_up(a * a + (13 + kPruneDefer) * d, 32);
}

size_t prune_ws_bytes(int64_t n, int64_t m, int p, int64_t cap, void* base, PruneWs* out);
int run_prune(int64_t n, int64_t m, int p, const PruneWs& w, const float* X, int64_t ldx,
              const int32_t* order, const double* B0, const double* Blag, int64_t cap,
              double* B0_out, double* Blag_out, int32_t* info, int32_t* st, hipStream_t stream);

}  // namespace vl
