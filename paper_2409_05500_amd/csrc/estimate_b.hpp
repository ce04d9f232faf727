// B0 / B_tau estimation (declarations).
#pragma once
#include "common.hpp"

namespace vl {

struct BWs {
  double* P = nullptr;     // m x m permuted covariance (destroyed by the factorisation)
  double* Linv = nullptr;  // m x m inverse of the factor
  double* chol = nullptr;  // factorisation scratch
};

size_t b_ws_bytes(int64_t m, void* base, BWs* out);
int run_estimate_b(const BWs& w, const double* Cov, const double* M, const int32_t* K, int64_t m,
                   int p, double* B0, double* Blag, int32_t* st, hipStream_t stream);

}  // namespace vl
