// FP64-grade products from int8 slices (the VL_PREC_SLICED arithmetic): each operand vector is
// scaled by a power of two 2^e (|value| < 2^e) and written as six signed digits,
//   v 2^-e = d_0 2^-6 + d_1 2^-13 + ... + d_5 2^-41 + rest,   |d_k| <= 64,  |rest| <= 2^-42,
// so a dot product is a sum over digit pairs of exact int8 x int8 MFMA products, summed exactly
// in int32 and weighted by powers of two in FP64.  Pairs (i, j) with i + j <= 5 are kept; those
// with the same i + j share an int32 accumulator.  Per product term the error is below 2^-39 of
// 2^(e_a + e_b): 2^-41 from the two remainders, about 2^-39.7 from the dropped pairs.
// (Splitting floating-point data into small-integer slices so that a dot product runs exactly
// on integer matrix units is the Ozaki scheme.)
#pragma once
#include "common.hpp"

namespace vl {

constexpr int kSlices = 6;
constexpr int kSliceK = 32;        // K step of the int8 MFMA; slice rows are padded to it

// Slice plane layout, K-blocked: the digits of row r at K index k are at byte
//   s * plane + (k / 32) * R * 32 + r * 32 + (k mod 32),   plane = R * round_up(K, 32),
// zero beyond K.  The 32-byte records of consecutive rows for one K block are contiguous, so a
// wave's operand load (32 rows x 32 bytes) is one contiguous kilobyte.
struct SliceOp {
  const int8_t* D = nullptr;
  int64_t rows = 0;                // R
  int64_t plane = 0;               // bytes per plane
  const int32_t* e = nullptr;      // exponent of row r: e[r mod e_period] (e[r] if 0); null: 0
  int64_t e_period = 0;
};

// Slices of the lag-embedded columns: row h m + j (h < L) of the operand holds
// x_j(t0 + t - h) - mu[j] for t < K and 0 for K <= t < round_up(K, 32), scaled by 2^-e[h m + j]
// (e from colmeans' range exponents: every such value is below 2^e in magnitude).
// D: slice_bytes(L m, K) bytes.
int slice_columns(const float* X, int64_t ldx, int64_t m, int L, int64_t t0, int64_t K,
                  const double* mu, const int32_t* e, int8_t* D, hipStream_t stream);

// Slices of the rows of the VAR design, each design column k scaled by 2^-f[k] (every value
// below 1 in magnitude, so the rows need no exponent of their own): row t holds
// z_k(t) 2^-f[k], z_k(t) = X[colmap[m + k] + t ldx] - mu[m + k], k < dz.
// D: slice_bytes(n_eff, dz) bytes.
int slice_design(const float* X, int64_t ldx, const int64_t* colmap, const double* mu,
                 const int32_t* f, int64_t m, int64_t dz, int64_t n_eff, int8_t* D,
                 hipStream_t stream);

// Slices of the columns of a row-major FP64 K x N matrix, entry k scaled by 2^f[k] (f nullable):
// row j holds C[k N + j] 2^f[k], k < K, with its exponent in e[j].  D: slice_bytes(N, K) bytes.
// With the design slices above, sum_k z_k(t) C_kj = sum_k (z_k(t) 2^-f[k]) (C_kj 2^f[k]).
int slice_matrix_columns(const double* C, const int32_t* f, int64_t K, int64_t N, int8_t* D,
                         int32_t* e, hipStream_t stream);

// Split-K factor and partial size of slice_gram (splits * M * N doubles).
int slice_gram_splits(int64_t M, int64_t N, int64_t K, bool sym);

// C[i ldc + j] = scale * sum_{k < K} A_i(k) B_j(k) from the slices (FP64 result).  sym: B is A
// (M == N), the lower tiles are computed and C comes out exactly symmetric.
int slice_gram(const SliceOp& A, int64_t M, const SliceOp& B, int64_t N, int64_t K, double scale,
               double* C, int64_t ldc, double* part, hipStream_t stream, bool sym = false);

// The VAR residual from the slices of the design rows (A, n_eff rows) and of the coefficient
// columns (B, m rows), K = dz:  E[t lde + j] = (X[colmap[j] + t ldx] - mu[j]) - sum_k z_k(t) C_kj,
// rounded to TOut once.
template <class TOut>
int slice_residual(const SliceOp& A, int64_t n_eff, const SliceOp& B, int64_t m, int64_t dz,
                   const float* X, int64_t ldx, const int64_t* colmap, const double* mu, TOut* E,
                   int64_t lde, hipStream_t stream);

// Bytes of slice planes for R rows of K: kSlices * R * round_up(K, 32).
inline int64_t slice_ldk(int64_t K) { return round_up(K, kSliceK); }
inline int64_t slice_bytes(int64_t R, int64_t K) { return kSlices * R * slice_ldk(K); }

}  // namespace vl
