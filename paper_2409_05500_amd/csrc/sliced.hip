// FP64-grade products from int8 slices (declarations and the digit format in sliced.hpp).
//
// Slicing kernels write the K-blocked planes of sliced.hpp.  The product kernel stages each
// 32-step of K of a 64 x 64 tile in LDS (one contiguous kilobyte per wave and slice), runs
// v_mfma_i32_32x32x32_i8 on every kept digit pair with one int32 accumulator per digit-weight
// class, and combines the classes in FP64 at the end.  The result does not depend on the
// order of the K loop: int32 sums are exact.
#include <algorithm>

#include "gram.hpp"
#include "sliced.hpp"

namespace vl {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// The six digits of v (|v| < 1): d_0 = rint(64 v), then each remainder (exact in FP64, at most
// 1/2 in magnitude) times 128, rounded.
__device__ __forceinline__ void digits6(double v, int (&d)[kSlices]) {
  double r = v * 64.0;
#pragma unroll
  for (int k = 0; k < kSlices; ++k) {
    const double q = rint(r);
    d[k] = (int)q;
    r = (r - q) * 128.0;
  }
}

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v = fmax(v, __shfl_xor(v, s, kWave));
  return v;
}

// ------------------------------------------------------------------------------------------
// Lag-embedded column slices.  Block: 64 samples x 64 variables of lag h = blockIdx.z; the
// digits go through LDS as [slice][variable][sample] bytes so that the stores run along the
// samples, 16 bytes a thread.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void slc_cols_kernel(const float* __restrict__ X, int64_t ldx,
                                                       int64_t m, int64_t t0, int64_t K,
                                                       const double* __restrict__ mu,
                                                       const int32_t* __restrict__ e,
                                                       int8_t* __restrict__ D, int64_t R,
                                                       int64_t kpad, int64_t plane) {
  __shared__ __align__(16) int8_t sd[kSlices][64][80];    // 64 samples + 16 bytes of padding
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t tb = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  const int h = blockIdx.z;
  const int64_t j = j0 + tx;
  const bool vj = j < m;
  const double c = vj ? mu[j] : 0.0;
  const int ej = vj ? e[(int64_t)h * m + j] : 0;
  // thread (j, ty): samples 16 ty + [0, 16) in groups of four, each group's digits packed into
  // one 32-bit LDS store per slice
#pragma unroll
  for (int g4 = 0; g4 < 4; ++g4) {
    const int r0 = 16 * ty + 4 * g4;
    int d[4][kSlices];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t t = tb + r0 + q;
#pragma unroll
      for (int s = 0; s < kSlices; ++s) d[q][s] = 0;
      if (vj && t < K) digits6(ldexp((double)X[(t0 + t - h) * ldx + j] - c, -ej), d[q]);
    }
#pragma unroll
    for (int s = 0; s < kSlices; ++s)
      *reinterpret_cast<uint32_t*>(&sd[s][tx][r0]) =
          (uint32_t)(uint8_t)d[0][s] | ((uint32_t)(uint8_t)d[1][s] << 8) |
          ((uint32_t)(uint8_t)d[2][s] << 16) | ((uint32_t)(uint8_t)d[3][s] << 24);
  }
  __syncthreads();
  for (int it = threadIdx.x; it < kSlices * 64 * 4; it += 256) {
    const int g = it & 3, jj = (it >> 2) & 63, s = it >> 8;
    const int64_t jr = j0 + jj, t = tb + 16 * g;
    if (jr >= m || t >= kpad) continue;       // kpad a multiple of 32, t of 16
    *reinterpret_cast<v4i*>(D + s * plane + (t >> 5) * R * 32 + ((int64_t)h * m + jr) * 32 +
                            (t & 31)) = *reinterpret_cast<const v4i*>(&sd[s][jj][16 * g]);
  }
}

int slice_columns(const float* X, int64_t ldx, int64_t m, int L, int64_t t0, int64_t K,
                  const double* mu, const int32_t* e, int8_t* D, hipStream_t stream) {
  const int64_t kpad = slice_ldk(K), R = (int64_t)L * m;
  dim3 g((unsigned)ceil_div(kpad, 64), (unsigned)ceil_div(m, 64), (unsigned)L);
  slc_cols_kernel<<<g, 256, 0, stream>>>(X, ldx, m, t0, K, mu, e, D, R, kpad, R * kpad);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

// ------------------------------------------------------------------------------------------
// Design slices with a scale per design column: z_k(t) 2^-f[k], every value below 1 (f from the
// column's range about its mean), no exponent per row.  Block: one K block of 32 columns x 8
// samples; thread (k, t) writes its digit bytes at consecutive addresses along k.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void store_digits4(int8_t* __restrict__ D, int64_t plane,
                                              int64_t off, const int (&d)[4][kSlices]) {
#pragma unroll
  for (int s = 0; s < kSlices; ++s) {
    const uint32_t w = (uint32_t)(uint8_t)d[0][s] | ((uint32_t)(uint8_t)d[1][s] << 8) |
                       ((uint32_t)(uint8_t)d[2][s] << 16) | ((uint32_t)(uint8_t)d[3][s] << 24);
    *reinterpret_cast<uint32_t*>(D + s * plane + off) = w;
  }
}

__global__ __launch_bounds__(256) void slc_design_kernel(const float* __restrict__ X, int64_t ldx,
                                                         const int64_t* __restrict__ colmap,
                                                         const double* __restrict__ mu,
                                                         const int32_t* __restrict__ f,
                                                         int64_t m, int64_t dz, int64_t n_eff,
                                                         int8_t* __restrict__ D,
                                                         int64_t plane) {
  const int kk = threadIdx.x & 31;
  const int64_t k = (int64_t)blockIdx.x * 32 + kk;
  const int64_t t = (int64_t)blockIdx.y * 8 + (threadIdx.x >> 5);
  if (t >= n_eff) return;
  int d[kSlices] = {0, 0, 0, 0, 0, 0};
  if (k < dz) digits6(ldexp((double)X[colmap[m + k] + t * ldx] - mu[m + k], -f[k]), d);
  int8_t* dst = D + (int64_t)blockIdx.x * n_eff * 32 + t * 32 + kk;
#pragma unroll
  for (int s = 0; s < kSlices; ++s) dst[s * plane] = (int8_t)d[s];
}

int slice_design(const float* X, int64_t ldx, const int64_t* colmap, const double* mu,
                 const int32_t* f, int64_t m, int64_t dz, int64_t n_eff, int8_t* D,
                 hipStream_t stream) {
  const int64_t kpad = slice_ldk(dz);
  dim3 g((unsigned)(kpad / 32), (unsigned)ceil_div(n_eff, 8));
  slc_design_kernel<<<g, 256, 0, stream>>>(X, ldx, colmap, mu, f, m, dz, n_eff, D, n_eff * kpad);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

// Columns of a row-major FP64 K x N matrix, entry k scaled by 2^f[k] (f == nullptr: none): one
// wave per column.
__global__ __launch_bounds__(256) void slc_matcols_kernel(const double* __restrict__ C,
                                                          const int32_t* __restrict__ f,
                                                          int64_t K, int64_t N,
                                                          int8_t* __restrict__ D, int64_t kpad,
                                                          int64_t plane,
                                                          int32_t* __restrict__ e) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= N) return;
  auto val = [&](int64_t k) { return f ? ldexp(C[k * N + j], f[k]) : C[k * N + j]; };
  double mx = 0.0;
  for (int64_t k = lane; k < K; k += 64) mx = fmax(mx, fabs(val(k)));
  const int ex = exponent_of(wave_max_d(mx));
  if (lane == 0) e[j] = ex;
  for (int64_t k4 = 4 * (int64_t)lane; k4 < kpad; k4 += 256) {
    int d[4][kSlices];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t k = k4 + q;
#pragma unroll
      for (int s = 0; s < kSlices; ++s) d[q][s] = 0;
      if (k < K) digits6(ldexp(val(k), -ex), d[q]);
    }
    store_digits4(D, plane, (k4 >> 5) * N * 32 + j * 32 + (k4 & 31), d);
  }
}

int slice_matrix_columns(const double* C, const int32_t* f, int64_t K, int64_t N, int8_t* D,
                         int32_t* e, hipStream_t stream) {
  const int64_t kpad = slice_ldk(K);
  slc_matcols_kernel<<<(unsigned)ceil_div(N, 4), 256, 0, stream>>>(C, f, K, N, D, kpad,
                                                                  N * kpad, e);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

// ------------------------------------------------------------------------------------------
// The product.  Workgroup tile (32 WM) x (32 WN) of (row of A, row of B), WM x WN waves of
// 32 x 32.  Each 32-step of K is staged in LDS once for the workgroup (the K-blocked planes make
// a tile's records one contiguous run per slice), double-buffered with one barrier a step; lane
// l of a wave then reads the 16 bytes at K offset 16 (l / 32) of row (l mod 32) of its 32 rows
// for every slice (the int8 MFMA's operand layout: A and B take the same K offsets), one
// contiguous kilobyte per wave and slice, and issues the 21 digit-pair MFMAs.
// ------------------------------------------------------------------------------------------
template <int WM, int WN>
__device__ __forceinline__ void slice_mma(const SliceOp& A, int64_t i0, const SliceOp& B,
                                          int64_t j0, int64_t kbeg, int64_t kend,
                                          v16i (&acc)[kSlices]) {
  constexpr int TM = 32 * WM, TN = 32 * WN, NT = 64 * WM * WN;
  constexpr int CA = kSlices * TM * 2, CB = kSlices * TN * 2;    // 16-byte chunks a step
  static_assert(CA % NT == 0 && CB % NT == 0, "chunks divide among the threads");
  constexpr int PA = CA / NT, PB = CB / NT;
  __shared__ __align__(16) int8_t sA[2][kSlices * TM * 32];
  __shared__ __align__(16) int8_t sB[2][kSlices * TN * 32];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WN, wc = wave % WN, h = lane >> 5, l32 = lane & 31;
#pragma unroll
  for (int g = 0; g < kSlices; ++g) acc[g] = v16i{};
  if (kbeg >= kend) return;      // a split the rounding of the chunk left empty: zeros
  v4i ga[PA], gb[PB];
  // chunk c of a step: slice c / (2 T), row (c mod 2 T) / 2, half c mod 2 -- at byte 16 c of
  // the stage; rows past the operand's last are read from its last row (masked at the end)
  auto gload = [&](int64_t k) {
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      const int c = tid + q * NT, sl = c / (2 * TM), rem = c % (2 * TM);
      const int64_t r = std::min(i0 + (rem >> 1), A.rows - 1);
      ga[q] = *reinterpret_cast<const v4i*>(A.D + sl * A.plane + k * A.rows + r * 32 +
                                            16 * (rem & 1));
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int c = tid + q * NT, sl = c / (2 * TN), rem = c % (2 * TN);
      const int64_t r = std::min(j0 + (rem >> 1), B.rows - 1);
      gb[q] = *reinterpret_cast<const v4i*>(B.D + sl * B.plane + k * B.rows + r * 32 +
                                            16 * (rem & 1));
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < PA; ++q) *reinterpret_cast<v4i*>(&sA[buf][16 * (tid + q * NT)]) = ga[q];
#pragma unroll
    for (int q = 0; q < PB; ++q) *reinterpret_cast<v4i*>(&sB[buf][16 * (tid + q * NT)]) = gb[q];
  };
  gload(kbeg);
  lstore(0);
  __syncthreads();
  int buf = 0;
  for (int64_t k = kbeg; k < kend; k += kSliceK) {
    const bool more = k + kSliceK < kend;       // the same in every thread
    if (more) gload(k + kSliceK);
    v4i a[kSlices], b[kSlices];
#pragma unroll
    for (int sl = 0; sl < kSlices; ++sl) {
      a[sl] = *reinterpret_cast<const v4i*>(&sA[buf][sl * TM * 32 + (wr * 32 + l32) * 32 + 16 * h]);
      b[sl] = *reinterpret_cast<const v4i*>(&sB[buf][sl * TN * 32 + (wc * 32 + l32) * 32 + 16 * h]);
    }
#pragma unroll
    for (int i = 0; i < kSlices; ++i)
#pragma unroll
      for (int j = 0; i + j < kSlices; ++j)
        acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i + j], 0, 0, 0);
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
}

// The FP64 value of output element q of the lane: sum_g acc_g 2^(-12 - 7g) 2^(eA + eB).
__device__ __forceinline__ double slice_value(const v16i (&acc)[kSlices], int q, int esum) {
  double v = (double)acc[kSlices - 1][q];
#pragma unroll
  for (int g = kSlices - 2; g >= 0; --g) v = fma(v, 0x1p-7, (double)acc[g][q]);
  return ldexp(v, esum - 12);
}

__device__ __forceinline__ int row_exponent(const SliceOp& S, int64_t r) {
  return S.e ? S.e[S.e_period ? r % S.e_period : r] : 0;
}

// Workgroups are taken in an order that gives each XCD (block id mod 8) a contiguous range of
// the (split, row tile, column tile) sequence, column tiles fastest: the tiles that read the
// same rows of A and the same K range run on one XCD and share its L2.  total = tiles x splits;
// the grid is rounded up to a multiple of 8 and the extra blocks return.
__device__ __forceinline__ bool slice_block(int64_t total, int64_t& lb) {
  const int64_t nb = gridDim.x, b = blockIdx.x;
  lb = (b & 7) * (nb >> 3) + (b >> 3);
  return lb < total;
}

// Tile origin of tile index e: row-major over (tm x tn) tiles, or the lower triangle (sym).
__device__ __forceinline__ void slice_tile_origin(bool sym, int64_t e, int64_t tn, int64_t& i0,
                                                  int64_t& j0) {
  if (!sym) {
    i0 = (e / tn) * 64;
    j0 = (e % tn) * 64;
    return;
  }
  int64_t ti = (int64_t)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
  while (ti * (ti + 1) / 2 > e) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= e) ++ti;
  i0 = ti * 64;
  j0 = (e - ti * (ti + 1) / 2) * 64;
}

// Split z = blockIdx.z covers K in [z kchunk, (z + 1) kchunk); its FP64 partial tile goes to
// P[z] (M x N, ld N).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void slc_gram_kernel(
    SliceOp A, int64_t M, SliceOp B, int64_t N, int64_t Kpad, int64_t kchunk, int sym,
    int64_t tiles, int64_t tn, int64_t splits, double* __restrict__ P) {
  int64_t lb;
  if (!slice_block(tiles * splits, lb)) return;
  const int64_t z = lb / tiles;
  int64_t i0, j0;
  slice_tile_origin(sym != 0, lb - z * tiles, tn, i0, j0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1, h = lane >> 5, l32 = lane & 31;
  const int64_t kbeg = z * kchunk;
  const int64_t kend = std::min(Kpad, kbeg + kchunk);
  const int64_t col = j0 + wj * 32 + l32;
  const int ec = row_exponent(B, col < N ? col : 0);   // read before the products
  v16i acc[kSlices];
  slice_mma<2, 2>(A, i0, B, j0, kbeg, kend, acc);
  double* Pz = P + z * M * N;
  if (col >= N) return;
  // the row exponents, all read before the first store (clamped rows: a read under each
  // store's bounds test would wait for each in turn)
  int ea[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int64_t row = i0 + wi * 32 + 8 * (q >> 2) + 4 * h + (q & 3);
    ea[q] = row_exponent(A, row < M ? row : 0);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int64_t row = i0 + wi * 32 + 8 * (q >> 2) + 4 * h + (q & 3);
    if (row < M) Pz[row * N + col] = slice_value(acc, q, ea[q] + ec);
  }
}

// Split-K count.  Modelled time: rounds(s) ceil(K / s) a + s M N b, rounds(s) = ceil(tiles s /
// 768) (3 workgroups resident per CU of the 256: 48 KB of LDS each), a = 0.054 us per K entry
// of a round and b = 3.2e-6 us per partial element written and summed (16 bytes at ~5 TB/s),
// both measured on the m = 400, n = 10^4 lag products.  Without the rounds term the 1064
// workgroups of 8 splits ran 1.4 rounds, the last one mostly idle.  Constraints: at least
// 256 K entries a split, at most 64 splits, at most 65536 K entries a split (int32 range: a
// class sums at most 6 digit pairs of |d d'| <= 4096).
int slice_gram_splits(int64_t M, int64_t N, int64_t K, bool sym) {
  constexpr int64_t kSlots = 3 * 256;
  constexpr double kPerK = 0.054, kPerPartial = 3.2e-6;
  const int64_t tm = ceil_div(M, 64);
  const int64_t tiles = sym ? tm * (tm + 1) / 2 : tm * ceil_div(N, 64);
  const int64_t smin = std::max<int64_t>(1, ceil_div(K, 65536));
  const int64_t smax = std::max(smin, std::min<int64_t>(64, K / 256));
  int64_t best = smin;
  double best_t = 1e300;
  for (int64_t s = smin; s <= smax; ++s) {
    const double t = (double)ceil_div(tiles * s, kSlots) * (double)ceil_div(K, s) * kPerK +
                     (double)s * (double)M * (double)N * kPerPartial;
    if (t < best_t) {
      best_t = t;
      best = s;
    }
  }
  return (int)best;
}

int slice_gram(const SliceOp& A, int64_t M, const SliceOp& B, int64_t N, int64_t K, double scale,
               double* C, int64_t ldc, double* part, hipStream_t stream, bool sym) {
  const int splits = slice_gram_splits(M, N, K, sym);
  const int64_t Kpad = slice_ldk(K);
  const int64_t kchunk = round_up(ceil_div(Kpad, splits), kSliceK);
  const int64_t tm = ceil_div(M, 64), tn = ceil_div(N, 64);
  const int64_t tiles = sym ? tm * (tm + 1) / 2 : tm * tn;
  slc_gram_kernel<<<(unsigned)round_up(tiles * splits, 8), 256, 0, stream>>>(
      A, M, B, N, Kpad, kchunk, sym ? 1 : 0, tiles, tn, splits, part);
  VL_LAUNCH_CHECK();
  return sum_splits(part, splits, M, N, scale, C, ldc, sym, stream);
}

// The residual: rows of A are samples, rows of B variables; no split (K = dz).
template <class TOut>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void slc_residual_kernel(
    SliceOp A, int64_t n_eff, SliceOp B, int64_t m, int64_t Kpad,
    const float* __restrict__ X, int64_t ldx, const int64_t* __restrict__ colmap,
    const double* __restrict__ mu, TOut* __restrict__ E, int64_t lde, int64_t tiles,
    int64_t tn) {
  int64_t lb;
  if (!slice_block(tiles, lb)) return;
  int64_t i0, j0;
  slice_tile_origin(false, lb, tn, i0, j0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1, h = lane >> 5, l32 = lane & 31;
  v16i acc[kSlices];
  slice_mma<2, 2>(A, i0, B, j0, 0, Kpad, acc);
  const int64_t j = j0 + wj * 32 + l32;
  if (j >= m) return;
  const int ec = row_exponent(B, j);
  const double muj = mu[j];
  const int64_t cj = colmap[j];
  // Y and the row exponents (0 for the design's slices, whose rows carry none) at this lane's
  // outputs: every load issued before the first store (clamped rows)
  float yin[16];
  int ea[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int64_t t = i0 + wi * 32 + 8 * (q >> 2) + 4 * h + (q & 3);
    const int64_t tc = t < n_eff ? t : n_eff - 1;
    yin[q] = X[cj + tc * ldx];
    ea[q] = row_exponent(A, tc);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int64_t t = i0 + wi * 32 + 8 * (q >> 2) + 4 * h + (q & 3);
    if (t < n_eff)
      E[t * lde + j] = (TOut)(((double)yin[q] - muj) - slice_value(acc, q, ea[q] + ec));
  }
}

template <class TOut>
int slice_residual(const SliceOp& A, int64_t n_eff, const SliceOp& B, int64_t m, int64_t dz,
                   const float* X, int64_t ldx, const int64_t* colmap, const double* mu, TOut* E,
                   int64_t lde, hipStream_t stream) {
  const int64_t tn = ceil_div(m, 64), tiles = ceil_div(n_eff, 64) * tn;
  slc_residual_kernel<TOut><<<(unsigned)round_up(tiles, 8), 256, 0, stream>>>(
      A, n_eff, B, m, slice_ldk(dz), X, ldx, colmap, mu, E, lde, tiles, tn);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

template int slice_residual<float>(const SliceOp&, int64_t, const SliceOp&, int64_t, int64_t,
                                   const float*, int64_t, const int64_t*, const double*, float*,
                                   int64_t, hipStream_t);
template int slice_residual<double>(const SliceOp&, int64_t, const SliceOp&, int64_t, int64_t,
                                    const float*, int64_t, const int64_t*, const double*,
                                    double*, int64_t, hipStream_t);

}  // namespace vl
