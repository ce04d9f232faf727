// Ensembles of the fit: VAR resampling for the residual bootstrap and edge-probability
// aggregation over many fits (declarations).
#pragma once
#include "common.hpp"

namespace vl {

// Largest m (p + 1) of a simulation: the last p + 1 rows of a resample live in LDS.
constexpr int64_t kSimMaxRing = 8192;

size_t sim_ws_bytes(int64_t m, int p);
int run_var_simulate(const double* M, const double* intercept, int64_t m, int p, const float* X0,
                     int64_t ldx0, const float* E, int64_t n_e, int64_t lde, const int32_t* idx,
                     int64_t R, int64_t T, float* Xout, int64_t ldxo, int64_t series_stride,
                     void* ws, int32_t* st, hipStream_t stream);

size_t freq_ws_bytes(int64_t K, int64_t m);
int run_edge_frequency(const int32_t* orders, const double* B0s, const double* Blags, int64_t K,
                       int64_t m, int p, double threshold, const int32_t* problem_status,
                       double* P0, double* Plag, double* P_order, int32_t* count, void* ws,
                       int32_t* st, hipStream_t stream);

}  // namespace vl
