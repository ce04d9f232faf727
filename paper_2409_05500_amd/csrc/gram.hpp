// Column statistics and centred Gram matrices (declarations).
#pragma once
#include "common.hpp"

namespace vl {

// Row splits used by colmeans(); scratch must hold colmean_splits(K) * ncol doubles.
inline int colmean_splits(int64_t K) {
  int64_t s = K / 128;
  return (int)(s < 1 ? 1 : (s > 256 ? 256 : s));
}

// mean[c] = (1/K) sum_{t<K} A[map(c) + t*lda]  (FP64);  raises VL_ERR_NONFINITE on NaN/Inf.
// With rep: rep[h * rep_m + c] = mean[c] for c < rep_m and h < rep_blocks as well.
// With range_exp: range_exp[c] = e with |A(t, c) - mean[c mod centre_m]| < 2^e for every t < K
// (from the column's range; centre_m = 0: ncol), and scratch holds 3 splits ncol doubles;
// range_exp_own (with range_exp only): the same about the column's own mean.
int colmeans(const float* A, int64_t lda, const int64_t* colmap, int64_t ncol, int64_t K,
             double* mean, double* scratch, int32_t* st, hipStream_t stream,
             double* rep = nullptr, int64_t rep_m = 0, int64_t rep_blocks = 0,
             int32_t* range_exp = nullptr, int64_t centre_m = 0,
             int32_t* range_exp_own = nullptr);

// Split-K factor of gram_tn(); scratch must hold gram_splits(M,N,K) * M * N doubles.  About
// 1024 workgroups (four per CU): with M == N the tiles counted are the lower triangle's, which
// is all a symmetric Gram launches (a square non-symmetric one then gets the same splits).
inline int gram_splits(int64_t M, int64_t N, int64_t K) {
  const int64_t tm = ceil_div(M, 64);
  int64_t tiles = M == N ? tm * (tm + 1) / 2 : tm * ceil_div(N, 64);
  int64_t s = ceil_div(1024, tiles);
  int64_t smax = K / 256;
  if (smax < 1) smax = 1;
  if (s > smax) s = smax;
  if (s > 64) s = 64;
  return (int)(s < 1 ? 1 : s);
}

// Arithmetic of gram_tn():
//   kFp32        FP32 MFMA, FP32 accumulation over the whole split;
//   kFp32Flush64 FP32 MFMA partial sums over 128-sample blocks accumulated in FP64;
//   kFp64        FP64 MFMA on the widened FP32 inputs (exact products, FP64 sums);
//   kBf16        BF16 MFMA on the centred inputs rounded to BF16 (relative error 2^-9 per
//                input), FP32 partial sums added into FP64 every 128 samples.
enum class GramMode { kFp32, kFp32Flush64, kFp64, kBf16 };

// C[i*ldc + j] = scale * sum_{t<K} (A(t,i) - muA[i]) (B(t,j) - muB[j]),
//   A(t,i) = A[mapA[i] + t*lda] (mapA == nullptr: mapA[i] = i); likewise B.
// sym: B is the same operand as A (M == N): only the tiles on and below the diagonal are
// computed, and C comes out exactly symmetric.
int gram_tn(const float* A, int64_t lda, const int64_t* mapA, const double* muA, int64_t M,
            const float* B, int64_t ldb, const int64_t* mapB, const double* muB, int64_t N,
            int64_t K, GramMode mode, double scale, double* C, int64_t ldc, double* scratch,
            hipStream_t stream, bool sym = false);

// C[i*ldc + j] = scale * sum_{z < splits} P[z][i][j] (P: splits x M x N), in split order; sym
// (M == N): the lower triangle's sums, written to both triangles.
int sum_splits(const double* P, int splits, int64_t M, int64_t N, double scale, double* C,
               int64_t ldc, bool sym, hipStream_t stream);

// C[i*ldc + j] = sum_{t<K} (A(t,i) - muA[i]) B[t*ldb + j] with an FP64, uncentred B (FP64 MFMA).
int gram_tn_f64b(const float* A, int64_t lda, const int64_t* mapA, const double* muA, int64_t M,
                 const double* B, int64_t ldb, int64_t N, int64_t K, double* C, int64_t ldc,
                 double* scratch, hipStream_t stream);

}  // namespace vl
