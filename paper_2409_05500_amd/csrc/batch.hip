// Batched fit of many small VarLiNGAM problems of uneven size: the whole path (VAR fit of
// Sec. 2.1, pairwise precompute of Sec. 4.2 with Eq. 1-2, ordering of Alg. 1 with Eq. 3, and
// B0 / B_tau) with one kernel launch per stage for all problems.
//
// Throughput stages (column means, Gram matrices, residual GEMM, standardisation, Hx, pair
// coefficients, pairwise moments, combine) launch the sum of the problems' blocks; a
// block -> problem table and each problem's first block turn a block index into (problem,
// local block), and the block runs the same body as the single-problem kernel.  The two
// Cholesky factorisations (VAR normal equations; permuted residual covariance for B0) run the
// fused panel steps of the single-problem path, one launch per panel step for all problems
// (at most four steps: d <= 256), followed by batched FP64 GEMM tiles (back substitution, lag
// matrices B_tau).  The ordering runs one workgroup per problem.
//
// The Gram tiles here run over all samples in one block (no split-K; the batch supplies the
// parallelism), so results differ from the single-problem path by summation order only.
#include <stdio.h>
#include <stdlib.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "chol_dev.hpp"
#include "gram_dev.hpp"
#include "order_dev.hpp"
#include "pairwise_dev.hpp"
#include "profile.hpp"
#include "var_dev.hpp"

namespace vl {

constexpr int kBatchMaxM = 256;      // order body with 4 variables per lane
constexpr int kBatchMaxDz = 256;
constexpr int kMaxCholSteps = kBatchMaxDz / kNb;   // panel steps of either factorisation
static_assert(kBatchMaxM <= kBatchMaxDz, "the B0 factorisation uses the same step maps");

// Per-problem descriptor as the kernels see it (device copy in the workspace).
struct BInst {
  const float* X;
  int64_t n, m, ldx, n_eff, dz, nc;   // nc: columns of the lag map, m (p + 1)
  int p, fp32;
  double* M;
  double* intercept;
  float* E;
  int64_t lde;
  double* S;
  int32_t* order;
  double* margin;
  double* B0;
  double* Blag;
  // pairwise plan
  int nt, nchunk, chunk_len, pad;
  int64_t m_pad, tiles, n_pad, items;
  // workspace
  int64_t* colmap;
  double *mu, *G, *Coef, *L, *Tmp, *chol;
  float* CoefF;
  double *emu, *cov, *momx, *Hx, *Hr;
  float* Xs;
  float2* coef;
  float *partU, *partB;
  int32_t* clist;   // near-collinear tile flags, count, list (2 tiles + 1)
  double *P, *Linv, *bchol;
};

enum BMap { kMapColVar, kMapColE, kMapGramVar, kMapGramCov, kMapResid, kMapStd, kMapPrep,
            kMapMom, kMapComb, kMapVarChol0, kMapBChol0 = kMapVarChol0 + kMaxCholSteps,
            kMapVarBack = kMapBChol0 + kMaxCholSteps, kMapBlag, kNumMaps };

struct BTables {
  const BInst* inst;
  const int32_t* bmap[kNumMaps];   // block -> problem
  const int64_t* first[kNumMaps];  // problem -> its first block
};

// Wave-uniform copies in scalar registers (the descriptor fields are the same for a block).
__device__ inline int64_t uni(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)(uint64_t)v);
  const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}
template <class T>
__device__ inline T* uni(T* p) {
  return reinterpret_cast<T*>(uni(reinterpret_cast<int64_t>(p)));
}

__device__ inline int bat_locate(const BTables& T, int map, int64_t blk, int64_t& local) {
  const int b = T.bmap[map][blk];
  local = blk - T.first[map][b];
  return b;
}

// ------------------------------------------------------------------------------------------
__global__ void bat_reset_kernel(int32_t* st, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) st[i] = VL_OK;
}

// Column means over all n_eff rows, 64 columns per block; which = 0: the lag map of X (VAR),
// 1: the residuals E.  Raises VL_ERR_NONFINITE.
__global__ __launch_bounds__(256) void bat_colmeans_kernel(BTables T, int which, int32_t* st0) {
  int64_t lb;
  const int b = bat_locate(T, which ? kMapColE : kMapColVar, blockIdx.x, lb);
  const BInst& d = T.inst[b];
  __shared__ double red[4][64];
  const int cc = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const float* A = which ? d.E : d.X;
  const int64_t lda = which ? d.lde : d.ldx;
  const int64_t ncol = which ? d.m : d.nc;
  const int64_t c = lb * 64 + cc;
  double s = 0.0;
  bool bad = false;
  if (c < ncol) {
    const float* p = A + (which ? c : d.colmap[c]);
    const int64_t n_eff = d.n_eff;
    int64_t t = rg;
    for (; t + 28 < n_eff; t += 32) {                 // eight loads in flight per thread
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = p[(t + 4 * u) * lda];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        bad |= !isfinite(v[u]);
        s += (double)v[u];
      }
    }
    for (; t < n_eff; t += 4) {
      const float v = p[t * lda];
      bad |= !isfinite(v);
      s += (double)v;
    }
  }
  if (bad) raise_status(st0 + b, VL_ERR_NONFINITE);
  red[rg][cc] = s;
  __syncthreads();
  if (rg == 0 && c < ncol)
    (which ? d.emu : d.mu)[c] =
        (((red[0][cc] + red[1][cc]) + red[2][cc]) + red[3][cc]) / (double)d.n_eff;
}

// Centred Gram tiles over all samples.  which = 0: the lower-triangle tiles of G = Zc^T Zc
// (dz x dz; the Cholesky reads nothing above the diagonal blocks) then R = Zc^T Yc (dz x m,
// into Tmp, where the forward substitution works on it); which = 1: the lower-triangle tiles of Cov = Ec^T Ec / n_eff, each off-diagonal
// tile also written transposed (Cov exactly symmetric).  kFp64: FP64 MFMA on the widened data;
// otherwise FP32 MFMA.
// k-th tile (row-major) of the lower triangle of a t x t tile grid: (ti, tj), tj <= ti
__device__ inline void lower_tile(int64_t k, int64_t& ti, int64_t& tj) {
  ti = (int64_t)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
  while (ti * (ti + 1) / 2 > k) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= k) ++ti;
  tj = k - ti * (ti + 1) / 2;
}

template <bool kFp64>
__device__ inline void bat_gram_tile(const float* A, int64_t lda, const int64_t* mapA,
                                     const double* muA, int64_t M, const float* B, int64_t ldb,
                                     const int64_t* mapB, const double* muB, int64_t N,
                                     int64_t i0, int64_t j0, int64_t K, double* C, int64_t ldc,
                                     double scale, bool mirror) {
  if (kFp64)
    gram_tile_f64(A, lda, mapA, muA, M, B, ldb, mapB, muB, N, i0, j0, 0, K, C, ldc, scale,
                  mirror);
  else  // FP32 partial sums over 128-sample blocks added in FP64 (the single-problem path gets
        // the same from its FP64 combination of split-K partials)
    gram_tile_f32<4>(A, lda, mapA, muA, M, B, ldb, mapB, muB, N, i0, j0, 0, K, C, ldc, scale,
                     mirror);
}

template <bool kFp64>
__global__ __launch_bounds__(256) void bat_gram_kernel(BTables T, int which) {
  int64_t lb;
  const int b = bat_locate(T, which ? kMapGramCov : kMapGramVar, blockIdx.x, lb);
  const BInst& d = T.inst[b];
  if (which == 0) {
    const int64_t tz = ceil_div(d.dz, kGT), tm = ceil_div(d.m, kGT);
    const int64_t* mapZ = d.colmap + d.m;
    const double* muZ = d.mu + d.m;
    const int64_t tri = tz * (tz + 1) / 2;
    if (lb < tri) {
      int64_t ti, tj;
      lower_tile(lb, ti, tj);
      bat_gram_tile<kFp64>(d.X, d.ldx, mapZ, muZ, d.dz, d.X, d.ldx, mapZ, muZ, d.dz, ti * kGT,
                           tj * kGT, d.n_eff, d.G, d.dz, 1.0, false);
    } else {
      const int64_t l2 = lb - tri;
      bat_gram_tile<kFp64>(d.X, d.ldx, mapZ, muZ, d.dz, d.X, d.ldx, d.colmap, d.mu, d.m,
                           (l2 / tm) * kGT, (l2 % tm) * kGT, d.n_eff, d.Tmp, d.m, 1.0, false);
    }
  } else {
    int64_t ti, tj;
    lower_tile(lb, ti, tj);
    bat_gram_tile<kFp64>(d.E, d.lde, nullptr, d.emu, d.m, d.E, d.lde, nullptr, d.emu, d.m,
                         ti * kGT, tj * kGT, d.n_eff, d.cov, d.m, 1.0 / (double)d.n_eff,
                         ti != tj);
  }
}

// The factorisation arguments of a problem: which = 0, the VAR normal equations (G, with the
// right-hand sides R in Tmp and L^{-1} into L); which = 1, the order-permuted covariance P for
// B0 (L^{-1} into Linv only).
__device__ inline CholArgs bat_chol_args(const BInst& d, int which, int32_t* st) {
  CholArgs a;
  const int64_t n = which ? d.m : d.dz;
  const int64_t nb = ceil_div(n, (int64_t)kNb);
  double* ws = which ? d.bchol : d.chol;
  a.A = which ? d.P : d.G;
  a.n = n;
  a.lda = n;
  a.R = which ? nullptr : d.Tmp;
  a.nrhs = which ? 0 : d.m;
  a.ldr = d.m;
  a.Li = which ? d.Linv : d.L;
  a.ldli = n;
  a.diag0 = ws;
  a.Yb = ws + n;
  a.st = st;
  return a;
}

// One workgroup per problem: L^{-1} set to the identity and the first diagonal block factored.
__global__ __launch_bounds__(256) void bat_chol_prologue_kernel(const BInst* __restrict__ I,
                                                                int which, int32_t* st0) {
  const CholArgs a = bat_chol_args(I[blockIdx.x], which, st0 + blockIdx.x);
  for (int64_t e = threadIdx.x; e < a.n * a.n; e += 256) chol_linv_init(a, e);
  chol_prologue_block(a);
}

// Panel step k of every problem that has one (its items through the step-k map).
__global__ __launch_bounds__(256) void bat_chol_step_kernel(BTables T, int which, int k,
                                                            int32_t* st0) {
  int64_t lb;
  const int b = bat_locate(T, (which ? kMapBChol0 : kMapVarChol0) + k, blockIdx.x, lb);
  const CholArgs a = bat_chol_args(T.inst[b], which, st0 + b);
  chol_step_item(a, k, lb);
}

// Back substitution Coef = L^{-T} (L^{-1} R), 32 x 32 tiles of Coef (dz x m).
__global__ __launch_bounds__(256) void bat_back_kernel(BTables T) {
  int64_t lb;
  const int b = bat_locate(T, kMapVarBack, blockIdx.x, lb);
  const BInst& d = T.inst[b];
  const int64_t tn = ceil_div(d.m, (int64_t)32);
  gemm_f64_block(d.dz, d.m, d.dz, 1.0, d.L, d.dz, 1, d.Tmp, d.m, 0, 0.0, d.Coef, d.m, 0, 2,
                 (lb / tn) * 32, (lb % tn) * 32);
}

// One workgroup per problem: lag matrices, intercept and (FP32 mode) the FP32 coefficients.
__global__ __launch_bounds__(256) void bat_var_post_kernel(const BInst* __restrict__ I) {
  const BInst& d = I[blockIdx.x];
  const int64_t m = d.m, dz = d.dz;
  const int tid = threadIdx.x;
  for (int64_t e = tid; e < (int64_t)d.p * m * m; e += 256) {
    const int64_t tau1 = e / (m * m), rem = e % (m * m), i = rem / m, k = rem % m;
    d.M[e] = d.Coef[(tau1 * m + k) * m + i];
  }
  for (int64_t i = tid; i < m; i += 256) {
    double s = 0.0;
    for (int64_t k = 0; k < dz; ++k) s += d.Coef[k * m + i] * d.mu[m + k];
    d.intercept[i] = d.mu[i] - s;
  }
  if (d.fp32)
    for (int64_t e = tid; e < dz * m; e += 256) d.CoefF[e] = (float)d.Coef[e];
}

template <bool kFp64>
__global__ __launch_bounds__(256) void bat_var_residual_kernel(BTables T) {
  int64_t lb;
  const int b = bat_locate(T, kMapResid, blockIdx.x, lb);
  const BInst& d = T.inst[b];
  const int64_t tm = ceil_div(d.m, 64);
  const int64_t t0 = (lb / tm) * 64, j0 = (lb % tm) * 64;
  if (kFp64)
    var_residual_tile_f64<float>(d.X, d.ldx, d.colmap, d.mu, d.m, d.p, d.n_eff, d.Coef, d.E,
                                 d.lde, t0, j0);
  else
    var_residual_tile_f32(d.X, d.ldx, d.colmap, d.mu, d.m, d.p, d.n_eff, d.CoefF, d.E, d.lde, t0,
                          j0);
}

__global__ __launch_bounds__(256) void bat_standardize_kernel(BTables T, int32_t* st0) {
  int64_t lb;
  const int b = bat_locate(T, kMapStd, blockIdx.x, lb);
  const BInst& d = T.inst[b];
  const int64_t gx = ceil_div(d.n_pad, 64);
  standardize_tile(d.E, d.lde, d.n_eff, d.m, d.emu, d.cov, d.Xs, d.n_pad, d.m_pad, st0 + b,
                   (lb % gx) * 64, (lb / gx) * 64, d.clist, d.tiles + 1, lb,
                   gx * ceil_div(d.m_pad, 64));
}

// Blocks [0, m): Hx of variable lb; then the pair coefficients, 256 entries per block.
__global__ __launch_bounds__(256) void bat_prep_kernel(BTables T, int32_t* st0) {
  int64_t lb;
  const int b = bat_locate(T, kMapPrep, blockIdx.x, lb);
  const BInst& d = T.inst[b];
  if (lb < d.m)
    hx_block<256>(d.Xs, d.n_pad, d.n_eff, d.Hx, d.momx, lb);
  else
    pair_coef_elem(d.cov, d.m, d.m_pad, d.coef, d.nt, d.tiles, d.clist, st0 + b,
                   (lb - d.m) * 256 + threadIdx.x);
}

// The pairwise-moment items of all problems, in the table's longest-first order (no XCD
// remap: that would hand one XCD all the long items).
__global__ __launch_bounds__(256) void bat_moments_kernel(BTables T, int64_t total) {
  const int64_t g = blockIdx.x;
  if (g >= total) return;
  int64_t lb;
  const int b = bat_locate(T, kMapMom, g, lb);
  const BInst& d = T.inst[b];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t item = uni(lb) * 4 + wave;
  if (item >= uni(d.items)) return;
  pairwise_moments_item(uni(d.Xs), uni(d.n_pad), uni(d.coef), uni(d.m_pad), uni(d.m),
                        (int)uni(d.nt), uni(d.tiles), (int)uni(d.chunk_len), item,
                        uni(d.partU), uni(d.partB));
}

// The listed near-collinear tiles of problem blockIdx.x, recomputed after the moment kernel
// (one workgroup per problem, grid-stride over its list).
__global__ __launch_bounds__(256) void bat_collinear_kernel(const BInst* __restrict__ I) {
  const BInst& d = I[blockIdx.x];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t total = (int64_t)d.clist[d.tiles] * d.nchunk;
  for (int64_t w = wave; w < total; w += 4) {
    const int64_t tile = d.clist[d.tiles + 1 + w / d.nchunk], chunk = w % d.nchunk;
    pairwise_collinear_item(d.E, d.lde, d.n_eff, d.emu, d.cov, d.m, d.nt, d.chunk_len, tile,
                            chunk, d.partU, d.partB);
  }
}

// Per unordered pair (one thread at i <= j): Hr of both orders, then S[i][j] and S[j][i] with
// the single-problem formula.
__global__ __launch_bounds__(256) void bat_combine_kernel(BTables T) {
  int64_t lb;
  const int b = bat_locate(T, kMapComb, blockIdx.x, lb);
  const BInst& d = T.inst[b];
  const int64_t m = d.m, e = lb * 256 + threadIdx.x;
  if (e >= m * m) return;
  const int64_t i = e / m, j = e % m;
  if (i > j) return;
  combine_hr_elem(d.partU, d.partB, d.nchunk, m, d.n_eff, d.Hr, nullptr, e);
  if (i == j) {
    d.S[e] = 0.0;
    return;
  }
  const int64_t e2 = j * m + i;
  combine_hr_elem(d.partU, d.partB, d.nchunk, m, d.n_eff, d.Hr, nullptr, e2);
  d.S[e] = (d.Hx[j] + d.Hr[e]) - (d.Hx[i] + d.Hr[e2]);
  d.S[e2] = (d.Hx[i] + d.Hr[e2]) - (d.Hx[j] + d.Hr[e]);
}

// One workgroup per problem: the ordering, then B0 from the LDL^T of the order-permuted
// covariance (B0_KK = I - L^{-1}) and B_tau = (I - B0) M_tau.
// One workgroup per problem: the ordering, then the covariance permuted into that order
// (with the permutation check).
__global__ __launch_bounds__(256) void bat_order_kernel(const BInst* __restrict__ I,
                                                        int32_t* st0) {
  const BInst& d = I[blockIdx.x];
  int32_t* st = st0 + blockIdx.x;
  const int64_t m = d.m;
  const int tid = threadIdx.x;
  order_wave_block<kBatchMaxM / 64, 256>(d.S, m, d.order, d.margin, st);
  __shared__ int seen[kBatchMaxM];
  for (int64_t a = tid; a < m; a += 256) seen[a] = 0;
  __syncthreads();
  const int32_t* K = d.order;
  for (int64_t e = tid; e < m * m; e += 256) {
    const int64_t a = e / m, c = e % m;
    const int32_t ka = K[a], kc = K[c];
    if (ka < 0 || ka >= m || kc < 0 || kc >= m) {
      raise_status(st, VL_ERR_INVALID_ARG);
      d.P[e] = a == c ? 1.0 : 0.0;
      continue;
    }
    d.P[e] = d.cov[(int64_t)ka * m + kc];
    if (c == 0) atomicAdd(&seen[ka], 1);
  }
  __syncthreads();
  for (int64_t a = tid; a < m; a += 256)
    if (seen[a] != 1) raise_status(st, VL_ERR_INVALID_ARG);
}

// One workgroup per problem: B0[K_a][K_b] = -Linv[a][b] / Linv[a][a] for b < a, else 0.
__global__ __launch_bounds__(256) void bat_b0_kernel(const BInst* __restrict__ I) {
  const BInst& d = I[blockIdx.x];
  const int64_t m = d.m;
  const int32_t* K = d.order;
  for (int64_t e = threadIdx.x; e < m * m; e += 256) {
    const int64_t a = e / m, c = e % m;
    const int32_t ka = K[a], kc = K[c];
    if (ka < 0 || ka >= m || kc < 0 || kc >= m) continue;
    d.B0[(int64_t)ka * m + kc] = c < a ? -d.Linv[a * m + c] / d.Linv[a * m + a] : 0.0;
  }
}

// B_tau = M_tau - B0 M_tau, 32 x 32 tiles of each B_tau.
__global__ __launch_bounds__(256) void bat_blag_kernel(BTables T) {
  int64_t lb;
  const int b = bat_locate(T, kMapBlag, blockIdx.x, lb);
  const BInst& d = T.inst[b];
  const int64_t m = d.m, tm = ceil_div(m, (int64_t)32);
  const int64_t tau = lb / (tm * tm), rem = lb % (tm * tm);
  const double* Mt = d.M + tau * m * m;
  gemm_f64_block(m, m, m, -1.0, d.B0, m, 0, Mt, m, 0, 1.0, d.Blag + tau * m * m, m, 0, 0,
                 (rem / tm) * 32, (rem % tm) * 32, Mt);
}

}  // namespace vl

// ==========================================================================================
// Host side: plan, workspace layout, tables, launches, autotuner.
// ==========================================================================================
using namespace vl;

namespace {

constexpr int kChunkCandidates[] = {512, 1024, 2048, 4096, 8192};
constexpr int kNumCand = sizeof(kChunkCandidates) / sizeof(int);

// Autotune buckets: 4 classes of m times 4 classes of n - p; every problem of a bucket takes
// the bucket's sample-chunk length for the pairwise stage.
constexpr int kNumBuckets = 16;
int bucket_of(const vl_instance& in) {
  const int64_t m = in.m, ne = in.n - in.p;
  const int mb = m <= 32 ? 0 : m <= 64 ? 1 : m <= 128 ? 2 : 3;
  const int nb = ne <= 1024 ? 0 : ne <= 2048 ? 1 : ne <= 4096 ? 2 : 3;
  return mb * 4 + nb;
}

struct InstLayout {
  size_t off = 0;                 // byte offset of this problem's slice in the workspace
  size_t cmap_off = 0;            // byte offset of its lag column map (in the table region)
  int nt = 0, nchunk = 0, chunk_len = 0;
  int64_t m_pad = 0, tiles = 0, n_pad = 0, items = 0;
};

// Carve one problem's slice; base == nullptr measures it.
size_t carve_inst(const vl_instance& in, const InstLayout& L, char* base, BInst* d) {
  Carver c(base);
  const int64_t m = in.m, dz = in.m * in.p, nc = in.m * (in.p + 1);
  const int64_t n_eff = in.n - in.p;
  BInst t = {};
  t.mu = c.take<double>(nc);
  t.G = c.take<double>(dz * dz);
  t.Coef = c.take<double>(dz * m);
  t.L = c.take<double>(dz * dz);
  t.Tmp = c.take<double>(dz * m);
  t.chol = c.take<double>(chol_ws_doubles_dev(dz));
  t.CoefF = c.take<float>(dz * m);
  t.emu = c.take<double>(m);
  t.cov = c.take<double>(m * m);
  t.momx = c.take<double>(2 * m);
  t.Hx = c.take<double>(m);
  t.Hr = c.take<double>(m * m);
  t.S = c.take<double>(m * m);               // used when the caller passes no S
  t.margin = c.take<double>(m);              // used when the caller passes no margin
  t.Xs = c.take<float>(L.m_pad * L.n_pad);
  t.coef = c.take<float2>(L.m_pad * L.m_pad);
  t.partU = c.take<float>((size_t)L.nchunk * m * m);
  t.partB = c.take<float>((size_t)L.nchunk * m * m);
  t.clist = c.take<int32_t>(2 * L.tiles + 1);
  t.P = c.take<double>(m * m);
  t.Linv = c.take<double>(m * m);
  t.bchol = c.take<double>(chol_ws_doubles_dev(m));
  (void)n_eff;
  if (d) *d = t;
  return c.used;
}

InstLayout layout_for(const vl_instance& in, int chunk) {
  InstLayout L;
  const int64_t m = in.m, n_eff = in.n - in.p;
  L.nt = (int)ceil_div(m, 4);
  L.m_pad = (int64_t)L.nt * 4;
  L.tiles = (int64_t)L.nt * (L.nt + 1) / 2;
  const int64_t cl = std::min<int64_t>(chunk, round_up(n_eff, 128));
  L.chunk_len = (int)cl;
  L.nchunk = (int)ceil_div(n_eff, cl);
  L.n_pad = (int64_t)L.nchunk * cl;
  L.items = L.tiles * L.nchunk;
  return L;
}

int64_t blocks_for(int map, const vl_instance& in, const InstLayout& L) {
  const int64_t m = in.m, dz = in.m * in.p, nc = in.m * (in.p + 1), n_eff = in.n - in.p;
  switch (map) {
    case kMapColVar: return ceil_div(nc, 64);
    case kMapColE: return ceil_div(m, 64);
    case kMapGramVar: return ceil_div(dz, 64) * (ceil_div(dz, 64) + 1) / 2 +
                             ceil_div(dz, 64) * ceil_div(m, 64);
    case kMapGramCov: return ceil_div(m, 64) * (ceil_div(m, 64) + 1) / 2;
    case kMapResid: return ceil_div(m, 64) * ceil_div(n_eff, 64);
    case kMapStd: return ceil_div(L.n_pad, 64) * ceil_div(L.m_pad, 64);
    case kMapPrep: return m + ceil_div(L.m_pad * L.m_pad, 256);
    case kMapMom: return ceil_div(L.items, 4);
    case kMapComb: return ceil_div(m * m, 256);
    case kMapVarBack: return ceil_div(dz, 32) * ceil_div(m, 32);
    case kMapBlag: return (int64_t)in.p * ceil_div(m, 32) * ceil_div(m, 32);
  }
  if (map >= kMapVarChol0 && map < kMapBChol0) {
    const int64_t k = map - kMapVarChol0, nb = ceil_div(dz, (int64_t)kNb);
    return k < nb ? step_items(nb, k, ceil_div(m, (int64_t)kNb), true).total() : 0;
  }
  if (map >= kMapBChol0 && map < kMapVarBack) {
    const int64_t k = map - kMapBChol0, nb = ceil_div(m, (int64_t)kNb);
    return k < nb ? step_items(nb, k, 0, true).total() : 0;
  }
  return 0;
}

}  // namespace

struct vl_batch {
  std::vector<vl_instance> inst;
  int count = 0;
  int prec = VL_PREC_MIXED;
  int chunk[kNumBuckets];    // sample-chunk length per autotune bucket
  size_t ws_bytes = 0;       // enough for any mix of chunk candidates
  // current layout
  std::vector<InstLayout> lay;
  int64_t total[kNumMaps] = {};
  size_t tab_off[kNumMaps * 2] = {};  // byte offsets of the bmap / first arrays
  size_t slices_off = 0;                // end of the tables and column maps
  void* bound = nullptr;
};

namespace {

// Layout for the batch's current chunk length; returns the workspace bytes it needs.
size_t build_layout(vl_batch* B) {
  const int n = B->count;
  B->lay.resize(n);
  size_t used = round_up((int64_t)(n * sizeof(BInst)), 256);
  for (int k = 0; k < kNumMaps; ++k) {
    int64_t tot = 0;
    for (int b = 0; b < n; ++b) {
      if (k == 0) B->lay[b] = layout_for(B->inst[b], B->chunk[bucket_of(B->inst[b])]);
      tot += blocks_for(k, B->inst[b], B->lay[b]);
    }
    B->total[k] = tot;
    B->tab_off[2 * k] = used;
    used += round_up((int64_t)((tot + 8) * sizeof(int32_t)), 256);
    B->tab_off[2 * k + 1] = used;
    used += round_up((int64_t)(n * sizeof(int64_t)), 256);
  }
  for (int b = 0; b < n; ++b) {
    B->lay[b].cmap_off = used;
    used += round_up(B->inst[b].m * (B->inst[b].p + 1) * (int64_t)sizeof(int64_t), 256);
  }
  B->slices_off = used;
  for (int b = 0; b < n; ++b) {
    B->lay[b].off = used;
    used += carve_inst(B->inst[b], B->lay[b], nullptr, nullptr);
  }
  return used;
}

// Workspace bound over every mix of per-bucket chunk lengths: each problem's table blocks and
// slice at its largest candidate.
size_t layout_bound(const vl_batch* B) {
  const int n = B->count;
  size_t used = round_up((int64_t)(n * sizeof(BInst)), 256);
  for (int k = 0; k < kNumMaps; ++k) {
    int64_t tot = 0;
    for (int b = 0; b < n; ++b) {
      int64_t mx = 0;
      for (int c : kChunkCandidates)
        mx = std::max(mx, blocks_for(k, B->inst[b], layout_for(B->inst[b], c)));
      tot += mx;
    }
    used += round_up((int64_t)((tot + 8) * sizeof(int32_t)), 256);
    used += round_up((int64_t)(n * sizeof(int64_t)), 256);
  }
  for (int b = 0; b < n; ++b)
    used += round_up(B->inst[b].m * (B->inst[b].p + 1) * (int64_t)sizeof(int64_t), 256);
  for (int b = 0; b < n; ++b) {
    size_t mx = 0;
    for (int c : kChunkCandidates)
      mx = std::max(mx, carve_inst(B->inst[b], layout_for(B->inst[b], c), nullptr, nullptr));
    used += mx;
  }
  return used;
}

int upload(vl_batch* B, void* ws, hipStream_t stream) {
  const int n = B->count;
  char* base = static_cast<char*>(ws);
  std::vector<char> host(B->slices_off, 0);
  BInst* I = reinterpret_cast<BInst*>(host.data());
  for (int b = 0; b < n; ++b) {
    const vl_instance& in = B->inst[b];
    const InstLayout& L = B->lay[b];
    BInst d;
    carve_inst(in, L, base + L.off, &d);
    d.colmap = reinterpret_cast<int64_t*>(base + L.cmap_off);
    // colmap[tau m + i] = offset of x_i(t - tau) at t = 0 in the lag-embedded view (tau = 0: Y)
    int64_t* cm = reinterpret_cast<int64_t*>(host.data() + L.cmap_off);
    for (int64_t c = 0; c < in.m * (in.p + 1); ++c) cm[c] = (in.p - c / in.m) * in.ldx + c % in.m;
    d.X = in.X;
    d.n = in.n;
    d.m = in.m;
    d.ldx = in.ldx;
    d.p = in.p;
    d.n_eff = in.n - in.p;
    d.dz = in.m * in.p;
    d.nc = in.m * (in.p + 1);
    d.fp32 = B->prec == VL_PREC_FP32 ? 1 : 0;
    d.M = in.M;
    d.intercept = in.intercept;
    d.E = in.E;
    d.lde = in.lde;
    if (in.S) d.S = in.S;
    d.order = in.order;
    if (in.margin) d.margin = in.margin;
    d.B0 = in.B0;
    d.Blag = in.Blag;
    d.nt = L.nt;
    d.nchunk = L.nchunk;
    d.chunk_len = L.chunk_len;
    d.m_pad = L.m_pad;
    d.tiles = L.tiles;
    d.n_pad = L.n_pad;
    d.items = L.items;
    I[b] = d;
  }
  // Longest blocks first: a block's duration grows with its problem's sample count (Gram,
  // residual, column means, moment items) or its variable count, so the problems are laid out
  // in the launch by decreasing n_eff, then m; the short blocks of small problems fill the tail.
  std::vector<int> lpt(n);
  for (int b = 0; b < n; ++b) lpt[b] = b;
  std::stable_sort(lpt.begin(), lpt.end(), [&](int a, int c) {
    const int64_t na = B->inst[a].n - B->inst[a].p, nc_ = B->inst[c].n - B->inst[c].p;
    return na != nc_ ? na > nc_ : B->inst[a].m > B->inst[c].m;
  });
  for (int k = 0; k < kNumMaps; ++k) {
    int32_t* bm = reinterpret_cast<int32_t*>(host.data() + B->tab_off[2 * k]);
    int64_t* first = reinterpret_cast<int64_t*>(host.data() + B->tab_off[2 * k + 1]);
    int64_t pos = 0;
    for (int b : lpt) {
      first[b] = pos;
      const int64_t nb = blocks_for(k, B->inst[b], B->lay[b]);
      for (int64_t q = 0; q < nb; ++q) bm[pos + q] = b;
      pos += nb;
    }
    for (int64_t q = pos; q < B->total[k] + 8; ++q) bm[q] = lpt[n - 1];   // padding blocks
  }
  if (hipMemcpyAsync(ws, host.data(), host.size(), hipMemcpyHostToDevice, stream) != hipSuccess)
    return VL_ERR_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return VL_ERR_HIP;
  B->bound = ws;
  return VL_OK;
}

BTables tables(const vl_batch* B, void* ws) {
  char* base = static_cast<char*>(ws);
  BTables T;
  T.inst = reinterpret_cast<const BInst*>(base);
  for (int k = 0; k < kNumMaps; ++k) {
    T.bmap[k] = reinterpret_cast<const int32_t*>(base + B->tab_off[2 * k]);
    T.first[k] = reinterpret_cast<const int64_t*>(base + B->tab_off[2 * k + 1]);
  }
  return T;
}

int launch_fit(const vl_batch* B, void* ws, int32_t* st, hipStream_t s) {
  const BTables T = tables(B, ws);
  const BInst* I = T.inst;
  const int n = B->count;
  const bool f64 = B->prec != VL_PREC_FP32;
  bat_reset_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(st, n);
  VL_LAUNCH_CHECK();
  {
    ProfileScope ps("batch_var", s);
    bat_colmeans_kernel<<<(unsigned)B->total[kMapColVar], 256, 0, s>>>(T, 0, st);
    VL_LAUNCH_CHECK();
    if (f64) bat_gram_kernel<true><<<(unsigned)B->total[kMapGramVar], 256, 0, s>>>(T, 0);
    else bat_gram_kernel<false><<<(unsigned)B->total[kMapGramVar], 256, 0, s>>>(T, 0);
    VL_LAUNCH_CHECK();
    bat_chol_prologue_kernel<<<(unsigned)n, 256, 0, s>>>(I, 0, st);
    VL_LAUNCH_CHECK();
    for (int k = 0; k < kMaxCholSteps; ++k) {
      if (B->total[kMapVarChol0 + k] == 0) continue;
      bat_chol_step_kernel<<<(unsigned)B->total[kMapVarChol0 + k], 256, 0, s>>>(T, 0, k, st);
      VL_LAUNCH_CHECK();
    }
    bat_back_kernel<<<(unsigned)B->total[kMapVarBack], 256, 0, s>>>(T);
    VL_LAUNCH_CHECK();
    bat_var_post_kernel<<<(unsigned)n, 256, 0, s>>>(I);
    VL_LAUNCH_CHECK();
    if (f64) bat_var_residual_kernel<true><<<(unsigned)B->total[kMapResid], 256, 0, s>>>(T);
    else bat_var_residual_kernel<false><<<(unsigned)B->total[kMapResid], 256, 0, s>>>(T);
    VL_LAUNCH_CHECK();
  }
  {
    ProfileScope ps("batch_pairwise", s);
    bat_colmeans_kernel<<<(unsigned)B->total[kMapColE], 256, 0, s>>>(T, 1, st);
    VL_LAUNCH_CHECK();
    if (f64) bat_gram_kernel<true><<<(unsigned)B->total[kMapGramCov], 256, 0, s>>>(T, 1);
    else bat_gram_kernel<false><<<(unsigned)B->total[kMapGramCov], 256, 0, s>>>(T, 1);
    VL_LAUNCH_CHECK();
    bat_standardize_kernel<<<(unsigned)B->total[kMapStd], 256, 0, s>>>(T, st);
    VL_LAUNCH_CHECK();
    bat_prep_kernel<<<(unsigned)B->total[kMapPrep], 256, 0, s>>>(T, st);
    VL_LAUNCH_CHECK();
  }
  {
    ProfileScope ps("batch_moments", s);
    const int64_t tot = B->total[kMapMom];
    bat_moments_kernel<<<(unsigned)round_up(tot, 8), 256, 0, s>>>(T, tot);
    VL_LAUNCH_CHECK();
    bat_collinear_kernel<<<(unsigned)n, 256, 0, s>>>(I);
    VL_LAUNCH_CHECK();
  }
  {
    ProfileScope ps("batch_order_b", s);
    bat_combine_kernel<<<(unsigned)B->total[kMapComb], 256, 0, s>>>(T);
    VL_LAUNCH_CHECK();
    bat_order_kernel<<<(unsigned)n, 256, 0, s>>>(I, st);
    VL_LAUNCH_CHECK();
    bat_chol_prologue_kernel<<<(unsigned)n, 256, 0, s>>>(I, 1, st);
    VL_LAUNCH_CHECK();
    for (int k = 0; k < kMaxCholSteps; ++k) {
      if (B->total[kMapBChol0 + k] == 0) continue;
      bat_chol_step_kernel<<<(unsigned)B->total[kMapBChol0 + k], 256, 0, s>>>(T, 1, k, st);
      VL_LAUNCH_CHECK();
    }
    bat_b0_kernel<<<(unsigned)n, 256, 0, s>>>(I);
    VL_LAUNCH_CHECK();
    bat_blag_kernel<<<(unsigned)B->total[kMapBlag], 256, 0, s>>>(T);
    VL_LAUNCH_CHECK();
  }
  return VL_OK;
}

// Autotune cache: per device and precision, the chunk length chosen for each bucket.  Kept in
// the process and in a text file (one "key chunk" line per bucket), read before tuning and
// rewritten after it through a temporary file and a rename.  The file is
// $VL_TUNE_CACHE if that is set (an empty value turns the file off), else
// $XDG_CACHE_HOME/varlingam/batch_tune.txt, else $HOME/.cache/varlingam/batch_tune.txt,
// taken at each call: the process's copy is that of the file named by the last call, and is
// read afresh when a call names another file.  File errors only cost a re-tune.
std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;
std::string g_tune_path;
bool g_tune_loaded = false;

std::string tune_file() {
  if (const char* e = getenv("VL_TUNE_CACHE")) return std::string(e);
  std::string dir;
  if (const char* x = getenv("XDG_CACHE_HOME"); x && *x) dir = x;
  else if (const char* h = getenv("HOME"); h && *h) dir = std::string(h) + "/.cache";
  else return std::string();
  return dir + "/varlingam/batch_tune.txt";
}

void tune_read(const std::string& path, std::map<std::string, int>& into) {
  if (path.empty()) return;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return;
  char key[256];
  int v = 0;
  while (fscanf(f, "%255s %d", key, &v) == 2)
    for (int c : kChunkCandidates)
      if (v == c) into[key] = v;
  fclose(f);
}

void tune_write(const std::string& path, const std::map<std::string, int>& entries) {
  if (path.empty()) return;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) {
    // create the directory chain (the cache's own folder and its parent at most)
    const std::string dir = path.substr(0, slash);
    const size_t up = dir.rfind('/');
    if (up != std::string::npos && up > 0) mkdir(dir.substr(0, up).c_str(), 0755);
    mkdir(dir.c_str(), 0755);
  }
  std::map<std::string, int> all;
  tune_read(path, all);
  for (const auto& kv : entries) all[kv.first] = kv.second;
  const std::string tmp = path + ".tmp." + std::to_string((long)getpid());
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  bool ok = true;
  for (const auto& kv : all) ok = ok && fprintf(f, "%s %d\n", kv.first.c_str(), kv.second) > 0;
  ok = (fclose(f) == 0) && ok;
  if (!ok || rename(tmp.c_str(), path.c_str()) != 0) remove(tmp.c_str());
}

std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string arch = prop.gcnArchName;
  for (char& ch : arch)
    if (ch == ' ' || ch == ':') ch = '_';
  return arch + "-cu" + std::to_string(prop.multiProcessorCount);
}

std::string bucket_key(const std::string& dev, int prec, int bucket) {
  return dev + ":p" + std::to_string(prec) + ":b" + std::to_string(bucket);
}

// The whole batch fit, warm-up and 3 timed repetitions, at the current chunk lengths.
int time_fit(vl_batch* B, void* ws, int32_t* dev_status, hipStream_t s, hipEvent_t e0,
             hipEvent_t e1, float* ms) {
  build_layout(B);
  int rc = upload(B, ws, s);
  if (rc) return rc;
  rc = launch_fit(B, ws, dev_status, s);
  if (rc) return rc;
  hipEventRecord(e0, s);
  for (int r = 0; r < 3 && !rc; ++r) rc = launch_fit(B, ws, dev_status, s);
  hipEventRecord(e1, s);
  if (rc) return rc;
  if (hipEventSynchronize(e1) != hipSuccess) return VL_ERR_HIP;
  return hipEventElapsedTime(ms, e0, e1) == hipSuccess ? VL_OK : VL_ERR_HIP;
}

}  // namespace

extern "C" {

int varlingam_batch_create(const vl_instance* inst, int count, int prec, vl_batch** out) {
  if (!out) return VL_ERR_INVALID_ARG;
  *out = nullptr;
  if (!inst || count < 1 || count > (1 << 20)) return VL_ERR_INVALID_ARG;
  if (prec != VL_PREC_FP32 && prec != VL_PREC_MIXED) return VL_ERR_INVALID_ARG;
  for (int b = 0; b < count; ++b) {
    const vl_instance& in = inst[b];
    if (!in.X || !in.M || !in.intercept || !in.E || !in.order || !in.B0 || !in.Blag)
      return VL_ERR_INVALID_ARG;
    if (in.m < 2 || in.m > kBatchMaxM || in.p < 1 || in.m * in.p > kBatchMaxDz ||
        in.n - in.p <= in.m * in.p + 1)
      return VL_ERR_SHAPE;
    if (in.ldx < in.m || in.lde < in.m) return VL_ERR_INVALID_ARG;
  }
  vl_batch* B = new vl_batch;
  B->inst.assign(inst, inst + count);
  B->count = count;
  B->prec = prec;
  for (int k = 0; k < kNumBuckets; ++k) B->chunk[k] = 2048;
  B->ws_bytes = std::max(layout_bound(B), build_layout(B));
  *out = B;
  return VL_OK;
}

size_t varlingam_batch_workspace_bytes(const vl_batch* B) { return B ? B->ws_bytes : 0; }

// the chunk length of the bucket that holds the most problems (ties: the lower bucket)
int varlingam_batch_chunk_len(const vl_batch* B) {
  if (!B) return 0;
  int cnt[kNumBuckets] = {};
  for (const auto& in : B->inst) ++cnt[bucket_of(in)];
  int best = 0;
  for (int k = 1; k < kNumBuckets; ++k)
    if (cnt[k] > cnt[best]) best = k;
  return B->chunk[best];
}

int varlingam_batch_chunk_len_of(const vl_batch* B, int problem) {
  if (!B || problem < 0 || problem >= B->count) return 0;
  return B->chunk[bucket_of(B->inst[problem])];
}

int varlingam_batch_bind(vl_batch* B, void* ws, size_t ws_bytes, void* stream) {
  if (!B || !ws) return VL_ERR_INVALID_ARG;
  if (ws_bytes < B->ws_bytes || (reinterpret_cast<uintptr_t>(ws) & 255u)) return VL_ERR_WORKSPACE;
  return upload(B, ws, reinterpret_cast<hipStream_t>(stream));
}

int varlingam_fit_batched(const vl_batch* B, void* ws, int32_t* dev_status, void* stream) {
  if (!B || !ws || !dev_status) return VL_ERR_INVALID_ARG;
  if (ws != B->bound) return VL_ERR_INVALID_ARG;
  return launch_fit(B, ws, dev_status, reinterpret_cast<hipStream_t>(stream));
}

// Search: every occupied bucket starts at the fastest uniform chunk length (all buckets
// equal), then coordinate descent visits the buckets by decreasing pairwise work (sum of
// m^2 (n - p)) and keeps a candidate only if the whole fit gets at least 1% faster.  Buckets
// found in the cache are not searched; with all of them cached nothing is timed.
int varlingam_batch_autotune(vl_batch* B, void* ws, size_t ws_bytes, int32_t* dev_status,
                             void* stream) {
  if (!B || !ws || !dev_status) return VL_ERR_INVALID_ARG;
  if (ws_bytes < B->ws_bytes || (reinterpret_cast<uintptr_t>(ws) & 255u)) return VL_ERR_WORKSPACE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const std::string dev = device_tag(), path = tune_file();
  double work[kNumBuckets] = {};
  for (const auto& in : B->inst)
    work[bucket_of(in)] += (double)in.m * (double)in.m * (double)(in.n - in.p);
  std::vector<int> occupied;
  for (int k = 0; k < kNumBuckets; ++k)
    if (work[k] > 0) occupied.push_back(k);
  std::stable_sort(occupied.begin(), occupied.end(),
                   [&](int a, int c) { return work[a] > work[c]; });
  std::vector<int> todo;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (!g_tune_loaded || path != g_tune_path) {
      g_tune_cache.clear();
      tune_read(path, g_tune_cache);
      g_tune_path = path;
      g_tune_loaded = true;
    }
    for (int k : occupied) {
      auto it = g_tune_cache.find(bucket_key(dev, B->prec, k));
      if (it != g_tune_cache.end()) B->chunk[k] = it->second;
      else todo.push_back(k);
    }
  }
  if (!todo.empty()) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return VL_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
      hipEventDestroy(e0);
      return VL_ERR_HIP;
    }
    int rc = VL_OK;
    float best_ms = 0.f;
    // uniform start for the buckets to search
    int best_c = B->chunk[todo[0]];
    for (int ci = 0; ci < kNumCand && !rc; ++ci) {
      for (int k : todo) B->chunk[k] = kChunkCandidates[ci];
      float ms = 0.f;
      rc = time_fit(B, ws, dev_status, s, e0, e1, &ms);
      if (!rc && (ci == 0 || ms < best_ms)) {
        best_ms = ms;
        best_c = kChunkCandidates[ci];
      }
    }
    for (int k : todo) B->chunk[k] = best_c;
    // coordinate descent, one pass
    for (size_t t = 0; t < todo.size() && !rc && todo.size() > 1; ++t) {
      const int k = todo[t], keep = B->chunk[k];
      int bestk = keep;
      for (int c : kChunkCandidates) {
        if (c == keep || rc) continue;
        B->chunk[k] = c;
        float ms = 0.f;
        rc = time_fit(B, ws, dev_status, s, e0, e1, &ms);
        if (!rc && ms < 0.99f * best_ms) {
          best_ms = ms;
          bestk = c;
        }
      }
      B->chunk[k] = bestk;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    std::map<std::string, int> found;
    for (int k : todo) found[bucket_key(dev, B->prec, k)] = B->chunk[k];
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (const auto& kv : found) g_tune_cache[kv.first] = kv.second;
    tune_write(path, found);
  }
  build_layout(B);
  return upload(B, ws, s);
}

void varlingam_batch_destroy(vl_batch* B) { delete B; }

}  // extern "C"
