// Fused blocked Cholesky + forward substitution, and the FP64 MFMA GEMM: the block-level bodies,
// shared by the single-problem kernels (one problem per launch) and the batched kernels (many
// problems per launch through block -> problem tables).
#pragma once
#include "common.hpp"
#include "linalg_dev.hpp"

namespace vl {

// ------------------------------------------------------------------------------------------
// FP64 GEMM on MFMA: C = beta C + alpha op(A) op(B).  A workgroup owns a 32 x 32 block of C (2 x 2
// v_mfma_f64_16x16x4f64 blocks); its four waves split the K range in four and add their partial
// products through LDS in a fixed order.  Operands are read straight from global memory (the
// callers' matrices are a few MB and stay in cache), four K steps in flight, through clamped
// in-bounds addresses with the padding masked.  tri = 1 / 2: op(A) lower / upper triangular (the
// zero part of the K range is skipped).  lower_only: entries above the diagonal are not written.
// ------------------------------------------------------------------------------------------
typedef double f64x4g __attribute__((ext_vector_type(4)));

// C0 (optional) supplies the beta term instead of C: C = beta C0 + alpha op(A) op(B).
__device__ __attribute__((always_inline)) inline void gemm_f64_block(
    int64_t M, int64_t N, int64_t K, double alpha, const double* __restrict__ A, int64_t lda,
    int transA, const double* __restrict__ Bm, int64_t ldb, int transB, double beta,
    double* __restrict__ C, int64_t ldc, int lower_only, int tri, int64_t i0, int64_t j0,
    const double* __restrict__ C0 = nullptr) {
  __shared__ double part[3][32 * 32];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
  if (lower_only && j0 > i0 + 31) return;
  // the beta term's inputs of wave 0's outputs, loaded before the products so that their
  // latency is hidden (clamped in-bounds addresses; only in-range elements use them)
  double cin[2][2][4];
  const bool use_c0 = beta != 0.0;
  if (use_c0 && w == 0) {
    const double* src = C0 ? C0 : C;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gi = i0 + x * 16 + lk + 4 * r, gj = j0 + y * 16 + li;
          const bool ok = gi < M && gj < N;
          cin[x][y][r] = src[(ok ? gi : 0) * ldc + (ok ? gj : 0)];
        }
  }
  int64_t kb = 0, ke = K;
  if (tri == 2) kb = i0 < K ? i0 : K;
  if (tri == 1) ke = i0 + 32 < K ? i0 + 32 : K;
  // this wave's quarter of [kb, ke), in steps of 4
  const int64_t span = round_up(ceil_div(ke - kb, (int64_t)4), (int64_t)4);
  const int64_t wb = kb + w * span, we = wb + span < ke ? wb + span : ke;
  int64_t ra[2], cb[2];
  bool vr[2], vc[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int64_t r = i0 + x * 16 + li, c = j0 + x * 16 + li;
    vr[x] = r < M;
    vc[x] = c < N;
    ra[x] = vr[x] ? r : M - 1;
    cb[x] = vc[x] ? c : N - 1;
  }
  f64x4g acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f64x4g{0.0, 0.0, 0.0, 0.0};
  // operands of the next 16-wide K slice are loaded while the current one is multiplied; the
  // padding is masked when a slice is used, not when it is loaded (masking a loaded value
  // waits for it, which would leave no load in flight across the products)
  double a[4][2], b[4][2], an[4][2], bn[4][2];
  auto load = [&](int64_t k0, double (&pa)[4][2], double (&pb)[4][2]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t k = k0 + 4 * s + lk;
      const int64_t kc = k < we ? k : (K > 0 ? K - 1 : 0);
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        pa[s][x] = transA ? A[kc * lda + ra[x]] : A[ra[x] * lda + kc];
        pb[s][x] = transB ? Bm[cb[x] * ldb + kc] : Bm[kc * ldb + cb[x]];
      }
    }
  };
  auto mask = [&](int64_t k0, double (&pa)[4][2], double (&pb)[4][2]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool vk = k0 + 4 * s + lk < we;
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        pa[s][x] = mask_f64(pa[s][x], vk && vr[x]);
        pb[s][x] = mask_f64(pb[s][x], vk && vc[x]);
      }
    }
  };
  auto mul = [&](const double (&pa)[4][2], const double (&pb)[4][2]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[s][x], pb[s][y], acc[x][y], 0, 0, 0);
  };
  // two slices per trip, the buffers alternating (a copy of a buffer still being loaded would
  // wait for it); the next slice is loaded unconditionally (clamped addresses, masked on use)
  // so that the wait before a slice's use leaves the following slice's loads in flight
  // (the scheduling barriers keep each slice's loads ahead of the previous slice's products)
  if (wb < we) {
    load(wb, a, b);
    for (int64_t k0 = wb;; k0 += 32) {
      load(k0 + 16, an, bn);
      __builtin_amdgcn_sched_barrier(0);
      mask(k0, a, b);
      mul(a, b);
      if (k0 + 16 >= we) break;
      load(k0 + 32, a, b);
      __builtin_amdgcn_sched_barrier(0);
      mask(k0 + 16, an, bn);
      mul(an, bn);
      if (k0 + 32 >= we) break;
    }
  }
  // result element (x, y, r) of this lane: row x*16 + lk + 4r, column y*16 + li of the block
  if (w > 0) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          part[w - 1][(x * 16 + lk + 4 * r) * 32 + y * 16 + li] = acc[x][y][r];
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rr = x * 16 + lk + 4 * r, cc = y * 16 + li;
          const double v = ((acc[x][y][r] + part[0][rr * 32 + cc]) + part[1][rr * 32 + cc]) +
                           part[2][rr * 32 + cc];
          const int64_t gi = i0 + rr, gj = j0 + cc;
          if (gi < M && gj < N && (!lower_only || gj <= gi))
            C[gi * ldc + gj] = beta * (use_c0 ? cin[x][y][r] : 0.0) + alpha * v;
        }
  }
}


// ------------------------------------------------------------------------------------------
// Fused blocked Cholesky + forward substitution.  Panel width 64; nb = ceil(n / 64) block rows.
// Per block k the workspace keeps Y_k = L_kk^{-1} (the inverse factor of the diagonal block after
// the updates of panels < k; exact zeros above its diagonal).  Right-looking step k applies panel
// k everywhere at once, each workgroup forming the panel rows it needs, L_ik = A_ik Y_k^T:
//   trailing tile (i, j), k < j <= i:   A_ij -= L_ik L_jk^T
//   right-hand tile (i, c), i > k:      R_ic -= L_ik (Y_k R_kc)        (= L_ik (L^{-1} R)_kc)
// and the workgroup of tile (k+1, k+1) goes on to factor and invert it (Y_{k+1}), so one launch
// per panel covers the factorisation and the substitution.  The critical chain through the
// launches is, per step, L = A Y^T, A -= L L^T and the 64 x 64 factor; nothing else (no
// Y^T Y product, no store beyond Y) sits on it.  Block row k of the right-hand sides is final
// after step k - 1; step k + 1 (or the last step) scales it in place: (L^{-1} R)_kc = Y_k R_kc.
// L^{-1} itself is the substitution applied to R = I, whose column tile c stays zero above
// block row c (those tiles are skipped).
// ------------------------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kTL = kLd;  // LDS tile leading dimension (65: rows land on different banks)

// Tiles move global -> registers -> LDS: v[u] = src[r * ld + c] (0 outside rows x cols) for the
// element e = threadIdx.x + 256 u, r = e / 64, c = e % 64, so all 16 loads of a thread are in
// flight at once and can be issued before a product that still reads the LDS tile.
__device__ inline void tile_fetch(double (&v)[16], const double* __restrict__ src, int64_t ld,
                                  int rows, int cols) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = threadIdx.x + 256 * u, r = e >> 6, c = e & 63;
    const bool ok = r < rows && c < cols;
    v[u] = mask_f64(src[(int64_t)(ok ? r : 0) * ld + (ok ? c : 0)], ok);
  }
}

__device__ inline void tile_put(double (*D)[kTL], const double (&v)[16]) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = threadIdx.x + 256 * u;
    D[e >> 6][e & 63] = v[u];
  }
}

// acc += op(P) op(Q) over 64 terms, P and Q 64 x 64 tiles in LDS (op = transpose when kTP /
// kTQ).  Wave w owns rows 32 (w >> 1) .. +31 and columns 32 (w & 1) .. +31 as 2 x 2 blocks of
// v_mfma_f64_16x16x4f64: A operand lane l -> (row l % 16, k l / 16), B operand -> (k l / 16,
// column l % 16), result register r -> (row l / 16 + 4 r, column l % 16).
template <bool kTP, bool kTQ>
__device__ inline void mm64(const double (*P)[kTL], const double (*Q)[kTL], f64x4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w >> 1, wj = w & 1, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < kNb; kk += 4) {
    double a[2], b[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const int row = wi * 32 + x * 16 + lr, col = wj * 32 + x * 16 + lr;
      a[x] = kTP ? P[kk + lk][row] : P[row][kk + lk];
      b[x] = kTQ ? Q[col][kk + lk] : Q[kk + lk][col];
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
  }
}

__device__ inline void acc_zero(f64x4 (&acc)[2][2]) {
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
}

// f(row, col, value) for every result element this thread holds
template <class F>
__device__ inline void acc_each(const f64x4 (&acc)[2][2], F f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w >> 1, wj = w & 1;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        f(wi * 32 + x * 16 + (lane >> 4) + 4 * r, wj * 32 + y * 16 + (lane & 15), acc[x][y][r]);
}

// L = P Y^T with Y lower-triangular (Y_qp = 0 for p > q), so output column block c needs only
// k < 16 (c + 1): wave w owns row block w (rows 16 w .. +15) and all four column blocks, 40 MFMAs
// per wave instead of 64.  Result register r of block c: row 16 w + l / 16 + 4 r, column
// 16 c + l % 16.  The skipped terms are exact zeros.
__device__ inline void mm64_tri(const double (*P)[kTL], const double (*Yl)[kTL],
                                f64x4 (&acc)[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < kNb; kk += 4) {
    const double a = P[16 * w + lr][kk + lk];
#pragma unroll
    for (int c = kk / 16; c < 4; ++c)
      acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Yl[16 * c + lr][kk + lk], acc[c], 0, 0, 0);
  }
}

__device__ inline void tri_zero(f64x4 (&acc)[4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};
}

template <class F>
__device__ inline void tri_each(const f64x4 (&acc)[4], F f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) f(16 * w + (lane >> 4) + 4 * r, 16 * c + (lane & 15), acc[c][r]);
}

// The lower block triangle (row block >= column block) of P P^T: ten 16 x 16 blocks over the
// four waves as 3, 3, 2, 2 (48 MFMAs per wave at most instead of 64).  Blocks above the
// diagonal are neither formed nor written: no consumer reads them.
__device__ inline int lower_blocks(int w, int b, int& bi, int& bj) {
  // wave 0: (0,0) (1,0) (1,1); wave 1: (2,0) (2,1) (2,2); wave 2: (3,0) (3,1); wave 3: (3,2) (3,3)
  if (w == 0) {
    bi = b == 0 ? 0 : 1;
    bj = b == 2 ? 1 : 0;
  } else if (w == 1) {
    bi = 2;
    bj = b;
  } else {
    bi = 3;
    bj = 2 * (w - 2) + b;
  }
  return w < 2 ? 3 : 2;
}

__device__ inline void mm64_lower(const double (*P)[kTL], f64x4 (&acc)[3]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lk = lane >> 4;
  int bi[3], bj[3];
  int n = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) n = lower_blocks(w, b, bi[b], bj[b]);
#pragma unroll
  for (int kk = 0; kk < kNb; kk += 4) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (b < n) {
        const double x = P[16 * bi[b] + lr][kk + lk];
        const double y = P[16 * bj[b] + lr][kk + lk];
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[b], 0, 0, 0);
      }
    }
  }
}

// f(slot, row, column) for the (up to 12) result positions a lane holds in mm64_lower
template <class F>
__device__ inline void lower_each(F f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    int bi, bj;
    const int n = lower_blocks(w, b, bi, bj);
    if (b < n) {
#pragma unroll
      for (int r = 0; r < 4; ++r) f(4 * b + r, 16 * bi + (lane >> 4) + 4 * r, 16 * bj + (lane & 15));
    }
  }
}

// Scratch doubles of the factorisation: the original diagonal, then per 64-row block Y_k.
__host__ __device__ inline int64_t chol_ws_doubles_dev(int64_t n) {
  return n + ((n + kNb - 1) / kNb) * kNb * kNb;
}

struct CholArgs {
  double* A;
  int64_t n, lda;
  double* R;          // right-hand sides (n x nrhs) or null
  int64_t nrhs, ldr;
  double* Li;         // L^{-1} (n x n) or null
  int64_t ldli;
  double* diag0;      // n: diagonal before elimination (pivot test)
  double* Yb;         // nb x 64 x 64: Y_k
  int32_t* st;
};

__host__ __device__ inline int64_t blk_rows(int64_t n, int64_t b) {
  return n - b * kNb < kNb ? n - b * kNb : kNb;
}

// Work items of step k, in launch order: trailing tiles (the critical tile (k+1, k+1) first),
// right-hand updates, L^{-1} updates, then the in-place scalings of block rows k - 1 and (last
// step) k for the right-hand sides and for L^{-1}.
struct StepItems {
  int64_t trail, upd_r, upd_i, fin_r, fin_i;
  __host__ __device__ int64_t total() const { return trail + upd_r + upd_i + fin_r + fin_i; }
};

__host__ __device__ inline StepItems step_items(int64_t nb, int64_t k, int64_t cr, bool li) {
  StepItems s;
  const int64_t t = nb - 1 - k;
  s.trail = t * (t + 1) / 2;
  s.upd_r = t * cr;
  s.upd_i = li ? t * (k + 1) : 0;
  const int64_t nfin = (k >= 1 ? 1 : 0) + (k == nb - 1 ? 1 : 0);
  s.fin_r = nfin * cr;
  s.fin_i = li ? (k >= 1 ? k : 0) + (k == nb - 1 ? k + 1 : 0) : 0;
  return s;
}

// Y_b (zeros above the diagonal; the LDS tile's upper part is not read) to the workspace
__device__ inline void store_y(const double (*Y)[kTL], const CholArgs& a, int64_t b) {
  double* Yo = a.Yb + b * kNb * kNb;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = threadIdx.x + 256 * u, r = e >> 6, q = e & 63;
    Yo[e] = q <= r ? Y[r][q] : 0.0;
  }
}

// Entry threadIdx.x of block row b's original diagonal (1 past the matrix), the pivot floor's
// reference; loaded by the critical tile's workgroup together with its operand tiles.
__device__ inline double diag0_entry(const CholArgs& a, int64_t b) {
  const int64_t i = b * kNb + threadIdx.x;
  const bool ok = threadIdx.x < kNb && i < a.n;
  return mask_f64(a.diag0[ok ? i : 0], ok) + (ok ? 0.0 : 1.0);
}

// The critical tile's lower 16 x 16 blocks of L L^T, in row order (0,0) (1,0) (1,1) (2,0) ...
// (3,3): wave 0 takes block 0 alone (leaf 0 of the factorisation follows at once), waves 1..3
// take three each.  Returns the number of blocks of wave w; block b of the wave is (bi, bj).
__device__ inline int crit_blocks(int w, int b, int& bi, int& bj) {
  const int f = w == 0 ? 0 : 3 * (w - 1) + b + 1;
  bi = f >= 6 ? 3 : (f >= 3 ? 2 : (f >= 1 ? 1 : 0));
  bj = f - bi * (bi + 1) / 2;
  return w == 0 ? 1 : 3;
}

// f(slot, row, column) for the (up to 12) positions a lane holds in the critical tile's blocks:
// block b, register r of the 16 x 16 product -> slot 4 b + r
template <class F>
__device__ inline void crit_each(F f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    int bi, bj;
    const int n = crit_blocks(w, b, bi, bj);
    if (b < n) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        f(4 * b + r, 16 * bi + (lane >> 4) + 4 * r, 16 * bj + (lane & 15));
    }
  }
}

// Step 0's diagonal block: the original diagonal is saved for the pivot test, block 0 is
// factored and inverted (one workgroup).  All global loads are issued before the first store.
__device__ __attribute__((always_inline)) inline void chol_prologue_block(const CholArgs& a) {
  __shared__ double S[kNb][kTL];
  __shared__ double Y[kNb][kTL];
  __shared__ double buf[kFactorBuf];
  __shared__ double D0[kNb];
  const int kb = (int)blk_rows(a.n, 0);
  double v[16];
  tile_fetch(v, a.A, a.lda, kb, kb);
  const bool dk = (int)threadIdx.x < kb;
  const double d0v = mask_f64(a.A[(dk ? threadIdx.x : 0) * (a.lda + 1)], dk) + (dk ? 0.0 : 1.0);
  for (int64_t i0 = 0; i0 < a.n; i0 += 4 * 256) {
    double dg[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0 + threadIdx.x + 256 * u;
      dg[u] = a.A[(i < a.n ? i : 0) * (a.lda + 1)];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0 + threadIdx.x + 256 * u;
      if (i < a.n) a.diag0[i] = dg[u];
    }
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = threadIdx.x + 256 * u, r = e >> 6, q = e & 63;
    S[r][q] = (r < kb && q < kb) ? v[u] : (r == q ? 1.0 : 0.0);
  }
  if (threadIdx.x < kNb) D0[threadIdx.x] = d0v;
  block_factor_inv(S, Y, buf, D0, a.st);
  store_y(Y, a, 0);
}

// L^{-1} starts as the identity (the substitution works on it in place): element e of n x n.
__device__ inline void chol_linv_init(const CholArgs& a, int64_t e) {
  if (a.Li && e < a.n * a.n) {
    const int64_t r = e / a.n, c = e % a.n;
    a.Li[r * a.ldli + c] = r == c ? 1.0 : 0.0;
  }
}

// Work item e of step k (see step_items for the order of the items).
__device__ __attribute__((always_inline)) inline void chol_step_item(const CholArgs& a, int64_t k,
                                                                     int64_t e) {
  __shared__ double X[kNb][kTL];
  __shared__ double Z[kNb][kTL];
  __shared__ double buf[kFactorBuf];
  __shared__ double D0[kNb];
  const int64_t nb = ceil_div(a.n, (int64_t)kNb);
  const int64_t cr = a.R ? ceil_div(a.nrhs, (int64_t)kNb) : 0;
  const StepItems s = step_items(nb, k, cr, a.Li != nullptr);
  const double* Ak = a.A + k * kNb;                 // column block k of A
  const double* Yk = a.Yb + k * kNb * kNb;
  f64x4 acc[2][2];
  if (e < s.trail + s.upd_r + s.upd_i) {
    // L_ik = A_ik Y_k^T for the row block i of this item
    int64_t i, j = -1, c = -1;
    bool inv_side = false;
    if (e < s.trail) {
      int64_t ii = (int64_t)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
      while (ii * (ii + 1) / 2 > e) --ii;
      while ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
      i = k + 1 + ii;
      j = k + 1 + (e - ii * (ii + 1) / 2);
    } else if (e < s.trail + s.upd_r) {
      e -= s.trail;
      i = k + 1 + e / cr;
      c = e % cr;
    } else {
      e -= s.trail + s.upd_r;
      i = k + 1 + e / (k + 1);
      c = e % (k + 1);
      inv_side = true;
    }
    const int64_t ri = blk_rows(a.n, i);
    // the tile this item updates, and the second operand: A_jk (off-diagonal trailing tile) or
    // the right-hand tile of block row k
    double* out;
    const double* src2 = nullptr;
    int64_t ldo, ld2 = 0, rows2 = kNb, cols;
    if (j >= 0) {
      out = a.A + i * kNb * a.lda + j * kNb;
      ldo = a.lda;
      cols = blk_rows(a.n, j);
      if (j != i) {
        src2 = Ak + j * kNb * a.lda;
        ld2 = a.lda;
        rows2 = cols;
      }
    } else if (!inv_side) {
      cols = a.nrhs - c * kNb < kNb ? a.nrhs - c * kNb : kNb;
      out = a.R + i * kNb * a.ldr + c * kNb;
      ldo = a.ldr;
      src2 = a.R + k * kNb * a.ldr + c * kNb;
      ld2 = a.ldr;
    } else {
      cols = blk_rows(a.n, c);
      out = a.Li + i * kNb * a.ldli + c * kNb;
      ldo = a.ldli;
      src2 = a.Li + k * kNb * a.ldli + c * kNb;
      ld2 = a.ldli;
    }
    const int64_t cols2 = j >= 0 ? kNb : cols;
    const bool diag = j == i;
    // all global loads of the item are issued before the first product; cur follows the layout
    // of the item's last product (lower blocks for a diagonal tile)
    double cur[16], nxt[16];
    const bool crit = diag && i == k + 1;
    const double d0v = crit ? diag0_entry(a, k + 1) : 1.0;
    {
      double pa[16], py[16];
      if (crit) {
        crit_each([&](int u, int r, int q) {
          const bool ok = r < ri && q < cols;
          cur[u] = out[(int64_t)(ok ? r : 0) * ldo + (ok ? q : 0)];
        });
      } else if (diag) {
        lower_each([&](int u, int r, int q) {
          const bool ok = r < ri && q < cols;
          cur[u] = out[(int64_t)(ok ? r : 0) * ldo + (ok ? q : 0)];
        });
      } else {
        int u = 0;
        acc_each(acc, [&](int r, int q, double) {
          const bool ok = r < ri && q < cols;
          cur[u++] = out[(int64_t)(ok ? r : 0) * ldo + (ok ? q : 0)];
        });
      }
      tile_fetch(pa, Ak + i * kNb * a.lda, a.lda, (int)ri, kNb);
      tile_fetch(py, Yk, kNb, kNb, kNb);
      if (src2) tile_fetch(nxt, src2, ld2, (int)rows2, (int)cols2);
      tile_put(X, pa);
      tile_put(Z, py);
      if (crit && threadIdx.x < kNb) D0[threadIdx.x] = d0v;
    }
    __syncthreads();
    f64x4 l1[4];
    tri_zero(l1);
    mm64_tri(X, Z, l1);                              // L_ik
    __syncthreads();
    if (crit) {
      // The critical tile: S = A_ii - L_ik L_ik^T (identity-padded) goes to Z block by block,
      // (0,0) first: wave 0 factors leaf 0 of S while waves 1..3 form the other nine blocks.
      // L_ik stays in X until every block is formed; Y (the factor's inverse) then takes X.
      tri_each(l1, [&](int r, int q, double v) { X[r][q] = v; });
      __syncthreads();
      const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
      // register rr of a block product: row 16 bi + lane / 16 + 4 rr, column 16 bj + lane % 16
      auto put_s = [&](int b, int bi, int bj, const f64x4_t& p) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int r = 16 * bi + (lane >> 4) + 4 * rr, q = 16 * bj + (lane & 15);
          Z[r][q] = (r < ri && q < ri) ? cur[4 * b + rr] - p[rr] : (r == q ? 1.0 : 0.0);
        }
      };
      if (w == 0) {
        // block (0,0): four partial sums over the K quarters (independent MFMA chains)
        f64x4_t p[4];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
          p[kc] = f64x4_t{0.0, 0.0, 0.0, 0.0};
          mfma_blk16<true>(&X[0][16 * kc], kTL, &X[0][16 * kc], kTL, p[kc]);
        }
        put_s(0, 0, 0, (p[0] + p[1]) + (p[2] + p[3]));
      } else {
        // three blocks, their MFMA chains interleaved
        int bi[3], bj[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) crit_blocks(w, b, bi[b], bj[b]);
        f64x4_t p[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) p[b] = f64x4_t{0.0, 0.0, 0.0, 0.0};
        const int li = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < kNb; kk += 4) {
#pragma unroll
          for (int b = 0; b < 3; ++b)
            p[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(X[16 * bi[b] + li][kk + lk],
                                                         X[16 * bj[b] + li][kk + lk], p[b], 0,
                                                         0, 0);
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) put_s(b, bi[b], bj[b], p[b]);
      }
      double y0[kLeaf];
      bool bad_any = false;
      if (w == 0) leaf_factor_regs(Z, D0, 0, bad_any, y0);   // reads only its own block
      __syncthreads();
      if (w == 0) leaf_store_y(X, 0, y0);
      __syncthreads();
      block_factor_rest(Z, X, buf, D0, a.st, bad_any);
      store_y(X, a, k + 1);
      return;
    }
    if (diag) {
      // L_ik L_ik^T, lower blocks only
      tri_each(l1, [&](int r, int q, double v) { X[r][q] = v; });
      __syncthreads();
      f64x4 lo[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) lo[u] = f64x4{0.0, 0.0, 0.0, 0.0};
      mm64_lower(X, lo);
      lower_each([&](int u, int r, int q) {
        if (r < ri && q < cols) out[(int64_t)r * ldo + q] = cur[u] - lo[u >> 2][u & 3];
      });
      return;
    }
    tile_put(X, nxt);
    __syncthreads();
    if (j >= 0) {
      f64x4 l2[4];
      tri_zero(l2);
      mm64_tri(X, Z, l2);                            // L_jk
      __syncthreads();
      tri_each(l1, [&](int r, int q, double v) { X[r][q] = v; });
      tri_each(l2, [&](int r, int q, double v) { Z[r][q] = v; });
    } else {
      f64x4 l2[2][2];
      acc_zero(l2);
      mm64<false, false>(Z, X, l2);                  // Y_k R_kc
      __syncthreads();
      tri_each(l1, [&](int r, int q, double v) { X[r][q] = v; });
      acc_each(l2, [&](int r, int q, double v) { Z[r][q] = v; });
    }
    __syncthreads();
    acc_zero(acc);
    if (j >= 0) mm64<false, true>(X, Z, acc);
    else mm64<false, false>(X, Z, acc);
    int u = 0;
    acc_each(acc, [&](int r, int q, double v) {
      const double o = cur[u++];
      if (r < ri && q < cols) out[(int64_t)r * ldo + q] = o - v;
    });
    return;
  }
  // in-place scaling of a finished block row f: tile <- Y_f tile
  e -= s.trail + s.upd_r + s.upd_i;
  int64_t f, c;
  bool inv_side;
  if (e < s.fin_r) {
    const int64_t first = k >= 1 ? cr : 0;         // items of block row k - 1 come first
    f = e < first ? k - 1 : k;
    c = e < first ? e : e - first;
    inv_side = false;
  } else {
    e -= s.fin_r;
    if (k >= 1 && e < k) {
      f = k - 1;
      c = e;
    } else {
      f = k;
      c = e - (k >= 1 ? k : 0);
    }
    inv_side = true;
  }
  double* tile;
  int64_t ld, cols;
  if (!inv_side) {
    tile = a.R + f * kNb * a.ldr + c * kNb;
    ld = a.ldr;
    cols = a.nrhs - c * kNb < kNb ? a.nrhs - c * kNb : kNb;
  } else {
    tile = a.Li + f * kNb * a.ldli + c * kNb;
    ld = a.ldli;
    cols = blk_rows(a.n, c);
  }
  const int64_t rf = blk_rows(a.n, f);
  {
    double py[16], pt[16];
    tile_fetch(py, a.Yb + f * kNb * kNb, kNb, kNb, kNb);
    tile_fetch(pt, tile, ld, (int)rf, (int)cols);
    tile_put(X, py);
    tile_put(Z, pt);
  }
  __syncthreads();
  acc_zero(acc);
  mm64<false, false>(X, Z, acc);
  acc_each(acc, [&](int r, int q, double v) {
    if (r < rf && q < cols) tile[(int64_t)r * ld + q] = v;
  });
}

}  // namespace vl
