// Lookup-only ordering (declarations).
#pragma once
#include "common.hpp"

namespace vl {

constexpr int64_t kMaxOrderM = 16384;

// Enqueues the O(m^2) initial aggregate pass and the m sequential selection steps.
// M0: m doubles of scratch.  Non-finite S raises VL_ERR_NONFINITE.
int run_order(const double* S, int64_t m, int32_t* order, double* margin, double* M0,
              int32_t* st, hipStream_t stream);

}  // namespace vl
