// Column statistics and centred Gram matrices of sample-major data on gfx950 MFMA.
//
// Used for: the VAR normal equations (Sec. 2.1, Gram of the lag-embedded series), the
// refinement residual Z^T E, and the residual covariance whose normalisation gives the
// pairwise correlation of Eq. 1 (cov(x_i, x_j) / var(x_j) for standardised columns).
//
// Data are sample-major (row t = one time step).  A "column map" turns a virtual column c
// into the element offset of its first sample, which lets one launch read the lag-shifted
// views x(t - tau) of the same series without copies.
#include "gram.hpp"
#include "gram_dev.hpp"

namespace vl {

__global__ void reset_status_kernel(int32_t* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *st = VL_OK;
}

// ------------------------------------------------------------------------------------------
// Column sums over K samples, split over row blocks: part[rs * ncol + c] (FP64), plus a
// finiteness check.  Block = 256 threads = 64 columns x 4 row lanes.
// ------------------------------------------------------------------------------------------
// kRange: also each column's minimum and maximum over the split, at part[splits ncol + ...]
// and part[2 splits ncol + ...] (for the slice exponents).
template <bool kRange>
__global__ __launch_bounds__(256) void colsum_partial_kernel(const float* __restrict__ A,
                                                             int64_t lda,
                                                             const int64_t* __restrict__ colmap,
                                                             int64_t ncol, int64_t K,
                                                             int64_t rows_per_split,
                                                             double* __restrict__ part,
                                                             int32_t* st) {
  __shared__ double red[4][64];
  __shared__ float rmin[kRange ? 4 : 1][64], rmax[kRange ? 4 : 1][64];
  const int cc = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int64_t c = (int64_t)blockIdx.x * 64 + cc;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r1 = r0 + rows_per_split < K ? r0 + rows_per_split : K;
  double s = 0.0;
  float mn = INFINITY, mx = -INFINITY;
  bool bad = false;
  if (c < ncol) {
    const float* p = A + (colmap ? colmap[c] : c);
    int64_t t = r0 + rg;
    for (; t + 28 < r1; t += 32) {  // eight loads in flight, summed in row order
      float v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = p[(t + 4 * q) * lda];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        bad |= !isfinite(v[q]);
        s += (double)v[q];
        if constexpr (kRange) {
          mn = fminf(mn, v[q]);
          mx = fmaxf(mx, v[q]);
        }
      }
    }
    for (; t < r1; t += 4) {
      const float v = p[t * lda];
      bad |= !isfinite(v);
      s += (double)v;
      if constexpr (kRange) {
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
      }
    }
  }
  if (bad) raise_status(st, VL_ERR_NONFINITE);
  red[rg][cc] = s;
  if constexpr (kRange) {
    rmin[rg][cc] = mn;
    rmax[rg][cc] = mx;
  }
  __syncthreads();
  if (rg == 0 && c < ncol) {
    part[(int64_t)blockIdx.y * ncol + c] = ((red[0][cc] + red[1][cc]) + red[2][cc]) + red[3][cc];
    if constexpr (kRange) {
      const int64_t sn = (int64_t)gridDim.y * ncol;
      part[sn + (int64_t)blockIdx.y * ncol + c] =
          fminf(fminf(rmin[0][cc], rmin[1][cc]), fminf(rmin[2][cc], rmin[3][cc]));
      part[2 * sn + (int64_t)blockIdx.y * ncol + c] =
          fmaxf(fmaxf(rmax[0][cc], rmax[1][cc]), fmaxf(rmax[2][cc], rmax[3][cc]));
    }
  }
}

// sum_{z < splits} P[z * stride + e] in split order.  Eight loads are issued before they are
// added (the same sum): colmean_final has a few thousand threads at most, so their latency is
// hidden by loads in flight, not by other waves.
__device__ inline double sum_splits_at(const double* __restrict__ P, int splits, int64_t stride,
                                       int64_t e) {
  double s = 0.0;
  int z = 0;
  for (; z + 8 <= splits; z += 8) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = P[(int64_t)(z + q) * stride + e];
#pragma unroll
    for (int q = 0; q < 8; ++q) s += v[q];
  }
  for (; z < splits; ++z) s += P[(int64_t)z * stride + e];
  return s;
}

__global__ void colmean_final_kernel(const double* __restrict__ part, int64_t ncol, int splits,
                                     int64_t K, double* __restrict__ mean,
                                     double* __restrict__ rep, int64_t rep_m,
                                     int64_t rep_blocks, int32_t* __restrict__ range_exp,
                                     int64_t centre_m, int32_t* __restrict__ range_exp_own) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const double v = sum_splits_at(part, splits, ncol, c) / (double)K;
  mean[c] = v;
  if (rep && c < rep_m)
    for (int64_t h = 0; h < rep_blocks; ++h) rep[h * rep_m + c] = v;
  if (range_exp) {
    // |x - mu0| <= max(max - mu0, mu0 - min) over the column, mu0 the mean of column
    // c mod centre_m (the same sum, so the same value)
    const int64_t sn = (int64_t)splits * ncol, c0 = c % centre_m;
    const double mu0 = c0 == c ? v : sum_splits_at(part, splits, ncol, c0) / (double)K;
    double mn = INFINITY, mx = -INFINITY;
    int z = 0;
    for (; z + 8 <= splits; z += 8) {      // eight of each in flight
      double a[8], b[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        a[q] = part[sn + (int64_t)(z + q) * ncol + c];
        b[q] = part[2 * sn + (int64_t)(z + q) * ncol + c];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        mn = fmin(mn, a[q]);
        mx = fmax(mx, b[q]);
      }
    }
    for (; z < splits; ++z) {
      mn = fmin(mn, part[sn + (int64_t)z * ncol + c]);
      mx = fmax(mx, part[2 * sn + (int64_t)z * ncol + c]);
    }
    range_exp[c] = exponent_of(fmax(mx - mu0, mu0 - mn));
    if (range_exp_own) range_exp_own[c] = exponent_of(fmax(mx - v, v - mn));
  }
}

int colmeans(const float* A, int64_t lda, const int64_t* colmap, int64_t ncol, int64_t K,
             double* mean, double* scratch, int32_t* st, hipStream_t stream, double* rep,
             int64_t rep_m, int64_t rep_blocks, int32_t* range_exp, int64_t centre_m,
             int32_t* range_exp_own) {
  const int splits = colmean_splits(K);
  const int64_t rows = ceil_div(K, splits);
  dim3 grid((unsigned)ceil_div(ncol, 64), (unsigned)splits);
  if (range_exp)
    colsum_partial_kernel<true><<<grid, 256, 0, stream>>>(A, lda, colmap, ncol, K, rows,
                                                          scratch, st);
  else
    colsum_partial_kernel<false><<<grid, 256, 0, stream>>>(A, lda, colmap, ncol, K, rows,
                                                           scratch, st);
  VL_LAUNCH_CHECK();
  colmean_final_kernel<<<(unsigned)ceil_div(ncol, 256), 256, 0, stream>>>(
      scratch, ncol, splits, K, mean, rep, rep_m, rep_blocks, range_exp,
      centre_m > 0 ? centre_m : ncol, range_exp_own);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

// ------------------------------------------------------------------------------------------
// Centred TN Gram, split-K: blockIdx.z covers rows [z*kchunk, (z+1)*kchunk); each split writes
// its FP64 partial tile to P[z] (M x N, ld N).  With sym (A and B the same operand), blockIdx.x
// enumerates the tiles on and below the diagonal only.
// ------------------------------------------------------------------------------------------
__device__ inline void gram_tile_origin(int sym, int64_t& i0, int64_t& j0) {
  if (!sym) {
    i0 = (int64_t)blockIdx.y * kGT;
    j0 = (int64_t)blockIdx.x * kGT;
    return;
  }
  const int64_t e = blockIdx.x;
  int64_t ti = (int64_t)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
  while (ti * (ti + 1) / 2 > e) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= e) ++ti;
  i0 = ti * kGT;
  j0 = (e - ti * (ti + 1) / 2) * kGT;
}
template <int kFlush>
__global__ __launch_bounds__(256) void gram_tn_kernel(
    const float* __restrict__ A, int64_t lda, const int64_t* __restrict__ mapA,
    const double* __restrict__ muA, int64_t M, const float* __restrict__ B, int64_t ldb,
    const int64_t* __restrict__ mapB, const double* __restrict__ muB, int64_t N, int64_t K,
    int64_t kchunk, double* __restrict__ P, int sym) {
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = kb + kchunk < K ? kb + kchunk : K;
  int64_t i0, j0;
  gram_tile_origin(sym, i0, j0);
  gram_tile_f32<kFlush>(A, lda, mapA, muA, M, B, ldb, mapB, muB, N, i0, j0, kb, ke,
                        P + (int64_t)blockIdx.z * M * N, N, 1.0);
}

__global__ __launch_bounds__(256) void gram_tn_bf16_kernel(
    const float* __restrict__ A, int64_t lda, const int64_t* __restrict__ mapA,
    const double* __restrict__ muA, int64_t M, const float* __restrict__ B, int64_t ldb,
    const int64_t* __restrict__ mapB, const double* __restrict__ muB, int64_t N, int64_t K,
    int64_t kchunk, double* __restrict__ P, int sym) {
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = kb + kchunk < K ? kb + kchunk : K;
  int64_t i0, j0;
  gram_tile_origin(sym, i0, j0);
  gram_tile_bf16(A, lda, mapA, muA, M, B, ldb, mapB, muB, N, i0, j0, kb, ke,
                 P + (int64_t)blockIdx.z * M * N, N, 1.0);
}

__global__ __launch_bounds__(256) void gram_tn_f64_kernel(
    const float* __restrict__ A, int64_t lda, const int64_t* __restrict__ mapA,
    const double* __restrict__ muA, int64_t M, const float* __restrict__ B, int64_t ldb,
    const int64_t* __restrict__ mapB, const double* __restrict__ muB, int64_t N, int64_t K,
    int64_t kchunk, double* __restrict__ P, int sym) {
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = kb + kchunk < K ? kb + kchunk : K;
  int64_t i0, j0;
  gram_tile_origin(sym, i0, j0);
  gram_tile_f64(A, lda, mapA, muA, M, B, ldb, mapB, muB, N, i0, j0, kb, ke,
                P + (int64_t)blockIdx.z * M * N, N, 1.0);
}

// C[i][j] = sum_t (A(t,i) - muA[i]) B64[t][j] with an FP64 right operand (not centred): the
// refinement residual Zc^T E64.  Same tiling as gram_tn_f64_kernel.
__global__ __launch_bounds__(256) void gram_tn_f64b_kernel(
    const float* __restrict__ A, int64_t lda, const int64_t* __restrict__ mapA,
    const double* __restrict__ muA, int64_t M, const double* __restrict__ B, int64_t ldb,
    int64_t N, int64_t K, int64_t kchunk, double* __restrict__ P) {
  __shared__ float As[kGK64 * kGLd];
  __shared__ double Bs[kGK64 * kGLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.y * kGT, j0 = (int64_t)blockIdx.x * kGT;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = kb + kchunk < K ? kb + kchunk : K;
  const int cc = tid & 63, rg = tid >> 6;
  const int64_t ia = i0 + cc, jb = j0 + cc;
  const bool va = ia < M, vb = jb < N;
  const float* pa = A + (va ? (mapA ? mapA[ia] : ia) : 0);
  const double* pb = B + (vb ? jb : 0);
  const int wi = wave >> 1, wj = wave & 1;
  double mua[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int64_t ii = i0 + wi * 32 + q * 16 + (lane & 15);
    mua[q] = ii < M ? muA[ii] : 0.0;
  }
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  float ra[kGK64 / 4];
  double rb[kGK64 / 4];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < kGK64 / 4; ++r) {
      const int64_t t = k0 + rg + 4 * r;
      const bool in = t < ke;
      // a plain conditional load (no arithmetic on the value here, so no wait per load)
      ra[r] = (va && in) ? pa[t * lda] : 0.f;
      rb[r] = (vb && in) ? pb[t * ldb] : 0.0;
    }
  };
  load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kGK64) {
#pragma unroll
    for (int r = 0; r < kGK64 / 4; ++r) {
      As[(rg + 4 * r) * kGLd + cc] = ra[r];
      Bs[(rg + 4 * r) * kGLd + cc] = rb[r];
    }
    __syncthreads();
    if (k0 + kGK64 < ke) load(k0 + kGK64);
#pragma unroll
    for (int kk = 0; kk < kGK64; kk += 4) {
      const bool in = k0 + kk + (lane >> 4) < ke;
      double av[2], bv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double ra = (double)As[(kk + (lane >> 4)) * kGLd + wi * 32 + q * 16 + (lane & 15)];
        av[q] = in ? ra - mua[q] : 0.0;
        bv[q] = Bs[(kk + (lane >> 4)) * kGLd + wj * 32 + q * 16 + (lane & 15)];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  double* Pz = P + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wi * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int64_t j = j0 + wj * 32 + b * 16 + (lane & 15);
        if (i < M && j < N) Pz[i * N + j] = acc[a][b][r];
      }
}

// C[i * ldc + j] = scale * sum_z P[z][i][j], fixed order (deterministic).
__global__ void sum_splits_kernel(const double* __restrict__ P, int splits, int64_t M, int64_t N,
                                  double scale, double* __restrict__ C, int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  const double s = sum_splits_at(P, splits, M * N, e);
  C[(e / N) * ldc + (e % N)] = s * scale;
}

// Symmetric form: entries (i, j) with i >= j of the lower tiles are summed and written to both
// (i, j) and (j, i), so C is exactly symmetric.
__global__ void sum_splits_sym_kernel(const double* __restrict__ P, int splits, int64_t M,
                                      double scale, double* __restrict__ C, int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * M) return;
  const int64_t i = e / M, j = e % M;
  if (j > i) return;
  const double s = sum_splits_at(P, splits, M * M, e);
  C[i * ldc + j] = s * scale;
  C[j * ldc + i] = s * scale;
}

int sum_splits(const double* P, int splits, int64_t M, int64_t N, double scale, double* C,
               int64_t ldc, bool sym, hipStream_t stream) {
  const int64_t tot = M * N;
  if (sym)
    sum_splits_sym_kernel<<<(unsigned)ceil_div(tot, 256), 256, 0, stream>>>(P, splits, M, scale,
                                                                            C, ldc);
  else
    sum_splits_kernel<<<(unsigned)ceil_div(tot, 256), 256, 0, stream>>>(P, splits, M, N, scale,
                                                                       C, ldc);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

int gram_tn(const float* A, int64_t lda, const int64_t* mapA, const double* muA, int64_t M,
            const float* B, int64_t ldb, const int64_t* mapB, const double* muB, int64_t N,
            int64_t K, GramMode mode, double scale, double* C, int64_t ldc, double* scratch,
            hipStream_t stream, bool sym) {
  const int splits = gram_splits(M, N, K);
  const int64_t kchunk = round_up(ceil_div(K, splits), kGK);
  const int64_t tm = ceil_div(M, kGT), tn = ceil_div(N, kGT);
  dim3 grid(sym ? (unsigned)(tm * (tm + 1) / 2) : (unsigned)tn, sym ? 1u : (unsigned)tm,
            (unsigned)splits);
  const int sy = sym ? 1 : 0;
  if (mode == GramMode::kFp64)
    gram_tn_f64_kernel<<<grid, 256, 0, stream>>>(A, lda, mapA, muA, M, B, ldb, mapB, muB, N, K,
                                                 kchunk, scratch, sy);
  else if (mode == GramMode::kBf16)
    gram_tn_bf16_kernel<<<grid, 256, 0, stream>>>(A, lda, mapA, muA, M, B, ldb, mapB, muB, N, K,
                                                  kchunk, scratch, sy);
  else if (mode == GramMode::kFp32Flush64)
    gram_tn_kernel<4><<<grid, 256, 0, stream>>>(A, lda, mapA, muA, M, B, ldb, mapB, muB, N, K,
                                                kchunk, scratch, sy);
  else
    gram_tn_kernel<0><<<grid, 256, 0, stream>>>(A, lda, mapA, muA, M, B, ldb, mapB, muB, N, K,
                                                kchunk, scratch, sy);
  VL_LAUNCH_CHECK();
  const int64_t tot = M * N;
  if (sym)
    sum_splits_sym_kernel<<<(unsigned)ceil_div(tot, 256), 256, 0, stream>>>(scratch, splits, M,
                                                                            scale, C, ldc);
  else
    sum_splits_kernel<<<(unsigned)ceil_div(tot, 256), 256, 0, stream>>>(scratch, splits, M, N,
                                                                       scale, C, ldc);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

int gram_tn_f64b(const float* A, int64_t lda, const int64_t* mapA, const double* muA, int64_t M,
                 const double* B, int64_t ldb, int64_t N, int64_t K, double* C, int64_t ldc,
                 double* scratch, hipStream_t stream) {
  const int splits = gram_splits(M, N, K);
  const int64_t kchunk = round_up(ceil_div(K, splits), kGK);
  dim3 grid((unsigned)ceil_div(N, kGT), (unsigned)ceil_div(M, kGT), (unsigned)splits);
  gram_tn_f64b_kernel<<<grid, 256, 0, stream>>>(A, lda, mapA, muA, M, B, ldb, N, K, kchunk,
                                                scratch);
  VL_LAUNCH_CHECK();
  sum_splits_kernel<<<(unsigned)ceil_div(M * N, 256), 256, 0, stream>>>(scratch, splits, M, N,
                                                                       1.0, C, ldc);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

}  // namespace vl
