// One-time precompute of every pairwise entropy statistic (Sec. 4.2 steps 1-2; the first two
// lines of Alg. 1) on gfx950.
//
// Stages (all on the caller's stream):
//   1. column means and the centred covariance of E (FP64 MFMA Gram of the FP32 data);
//   2. standardise (Sec. 3 step 1) and transpose to variable-major Xs (m_pad x n_pad, FP32,
//      zero padded), plus the per-variable moments that give Hx = H(x_i);
//   3. per unordered pair {i,j}: rho = cov/(sd_i sd_j); the Eq. 1 residual of a standardised
//      pair is x_i - rho x_j with variance 1 - rho^2, so the re-standardised residual is
//      u_{i<-j} = (x_i - rho x_j) / sqrt(1 - rho^2); the kernel receives the two scaled
//      coefficients a = c / sqrt(1-rho^2), b = c rho / sqrt(1-rho^2) and forms w = c u;
//   4. the hot kernel: for every pair and sample, both directions w_{i<-j}, w_{j<-i} and their
//      entropy moments (Eq. 2): sum log cosh u and sum u exp(-u^2/2); the micro-tiles holding
//      a near-collinear pair (sqrt(1 - rho^2) < 0.25) are then recomputed by a second kernel
//      that forms their residuals in FP64 from E;
//   5. FP64 combine: Hr = H(nu) - k1 (A - gamma)^2 - k2 B^2 and
//      S[i,j] = (Hx[j] + Hr[i,j]) - (Hx[i] + Hr[j,i]).
#include <algorithm>

#include "gram.hpp"
#include "pairwise.hpp"
#include "pairwise_dev.hpp"
#include "profile.hpp"
#include "sliced.hpp"

namespace vl {

// ------------------------------------------------------------------------------------------
// Kernels (single problem): one body call per block / thread.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void standardize_transpose_kernel(
    const float* __restrict__ E, int64_t lde, int64_t n_eff, int64_t m,
    const double* __restrict__ mu, const double* __restrict__ cov, float* __restrict__ Xs,
    int64_t n_pad, int64_t m_pad, int32_t* st, int32_t* __restrict__ zero, int64_t nzero) {
  standardize_tile(E, lde, n_eff, m, mu, cov, Xs, n_pad, m_pad, st, (int64_t)blockIdx.x * 64,
                   (int64_t)blockIdx.y * 64, zero, nzero,
                   (int64_t)blockIdx.y * gridDim.x + blockIdx.x, (int64_t)gridDim.x * gridDim.y);
}

// Hx takes 1024 threads per variable: one workgroup per variable is all the parallelism there
// is (a few hundred workgroups in a fit, a handful late in the iterative search), so each works
// its samples with 16 waves.  Measured effect is small: the iterative search at m = 400 went
// 118.7 -> 117.4 ms, the fit's preparation stage 40.3 -> 39.8 us.
constexpr int kHxThreads = 1024;

// One launch for the two independent preparation steps: blocks [0, m) are hx_kernel's, the
// blocks after them form the pair coefficients, one element per thread.
__global__ __launch_bounds__(kHxThreads) void prep_kernel(
    const float* __restrict__ Xs, int64_t n_pad, int64_t n_eff, double* __restrict__ Hx,
    double* __restrict__ momx, const double* __restrict__ cov, int64_t m, int64_t m_pad,
    float2* __restrict__ coef, int nt, int64_t tiles, int32_t* __restrict__ clist, int32_t* st) {
  if ((int64_t)blockIdx.x < m) {
    hx_block<kHxThreads>(Xs, n_pad, n_eff, Hx, momx, blockIdx.x);
    return;
  }
  pair_coef_elem(cov, m, m_pad, coef, nt, tiles, clist, st,
                 ((int64_t)blockIdx.x - m) * kHxThreads + threadIdx.x);
}

// Blocks are remapped so that XCD x (block id mod 8) processes a contiguous range of items in
// chunk-major order, i.e. mostly one sample chunk per XCD and its L2.
// TP = float: plain FP32 moment sums; TP = double: compensated sums, FP64 partials.
template <class TP>
__global__ __launch_bounds__(256) void pairwise_moments_kernel(
    const float* __restrict__ Xs, int64_t n_pad, const float2* __restrict__ coef, int64_t m_pad,
    int64_t m, int nt, int64_t tiles, int chunk_len, int64_t items,
    TP* __restrict__ partU, TP* __restrict__ partB) {
  const int64_t nb = gridDim.x;                     // a multiple of 8
  const int64_t b = blockIdx.x;
  const int64_t lb = (b & 7) * (nb >> 3) + (b >> 3);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t item = lb * 4 + wave;
  if (item >= items) return;
  if constexpr (std::is_same<TP, double>::value)
    pairwise_moments_item_comp(Xs, n_pad, coef, m_pad, m, nt, tiles, chunk_len, item, partU,
                               partB);
  else
    pairwise_moments_item(Xs, n_pad, coef, m_pad, m, nt, tiles, chunk_len, item, partU, partB);
}

// The (listed tile, chunk) items of the near-collinear micro-tiles, grid-stride over the list
// the coefficient stage built (count = clist[tiles]); with no listed tile every wave returns
// at once.
template <class TP>
__global__ __launch_bounds__(256) void pairwise_collinear_kernel(
    const float* __restrict__ E, int64_t lde, int64_t n_eff, const double* __restrict__ mu,
    const double* __restrict__ cov, int64_t m, int nt, int64_t tiles, int nc, int chunk_len,
    const int32_t* __restrict__ clist, TP* __restrict__ partU, TP* __restrict__ partB) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t total = (int64_t)clist[tiles] * nc;
  for (int64_t w = (int64_t)blockIdx.x * 4 + wave; w < total; w += (int64_t)gridDim.x * 4) {
    const int64_t tile = clist[tiles + 1 + w / nc], chunk = w % nc;
    pairwise_collinear_item(E, lde, n_eff, mu, cov, m, nt, chunk_len, tile, chunk, partU,
                            partB);
  }
}

template <class TP>
__global__ void combine_hr_kernel(const TP* __restrict__ partU, const TP* __restrict__ partB,
                                  int nc, int64_t m, int64_t n_eff, double* __restrict__ Hr,
                                  double* __restrict__ mom) {
  combine_hr_elem(partU, partB, nc, m, n_eff, Hr, mom,
                  (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void score_kernel(const double* __restrict__ Hx, const double* __restrict__ Hr,
                             int64_t m, double* __restrict__ S) {
  score_elem(Hx, Hr, m, S, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------
// Sample chunks: about 16K (tile, chunk) items -- at least 4 chunks, each of at least 512
// samples (4 steps of 2 samples per lane), chunks a multiple of 128.  Measured at one launch
// per fit: m = 400 (n = 10^4) within 1% of the best chunk count, m = 1000 (n = 5 10^4) within
// 0.5%, m = 100 (n = 5000) within 4% (a floor of 2048 samples per chunk was 49% slower there).
PairwisePlan plan_pairwise(int64_t n_eff, int64_t m, bool compensated, bool sliced) {
  PairwisePlan p;
  p.comp = compensated;
  p.sliced = sliced;
  p.m = m;
  p.n_eff = n_eff;
  p.nt = (int)ceil_div(m, kT);
  p.m_pad = (int64_t)p.nt * kT;
  p.tiles = (int64_t)p.nt * (p.nt + 1) / 2;
  const int64_t want = std::max<int64_t>(4, ceil_div(16384, p.tiles));
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(512, n_eff / 512));
  p.nc = (int)std::min(want, cap);
  p.chunk_len = (int)round_up(ceil_div(n_eff, p.nc), 128);
  p.n_pad = (int64_t)p.nc * p.chunk_len;
  p.items = p.tiles * p.nc;
  p.blocks = round_up(ceil_div(p.items, 4), 8);
  return p;
}

// The split partials of the column means and the covariance are dead once the covariance is
// formed, before anything of stages 2-5 is written: the two share one region.
size_t pairwise_ws_bytes(const PairwisePlan& p, void* base, PairwiseWs* out) {
  Carver c(base);
  PairwiseWs w;
  w.mu = c.take<double>(p.m);
  w.cov = c.take<double>(p.m * p.m);
  w.momx = c.take<double>(2 * p.m);
  char* region = base ? static_cast<char*>(base) + c.used : nullptr;
  Carver a(region);                              // stage 1
  w.scratch = a.take<double>(scratch_doubles(p));
  if (p.sliced) {
    w.slices = a.take<int8_t>(slice_bytes(p.m, p.n_eff));
    w.ex = a.take<int32_t>(p.m);
  }
  Carver b(region);                              // stages 2-5
  w.Xs = b.take<float>(p.m_pad * p.n_pad);
  w.coef = b.take<float2>(p.m_pad * p.m_pad);
  // FP32 partials, or FP64 ones for the compensated sums (the same region either way)
  const size_t np = (size_t)p.nc * p.m * p.m;
  if (p.comp) {
    w.partU64 = b.take<double>(np);
    w.partB64 = b.take<double>(np);
  } else {
    w.partU = b.take<float>(np);
    w.partB = b.take<float>(np);
  }
  w.clist = b.take<int32_t>(2 * p.tiles + 1);
  if (out) *out = w;
  return c.used + std::max(a.used, b.used);
}

size_t scratch_doubles(const PairwisePlan& p) {
  size_t a = (size_t)colmean_splits(p.n_eff) * p.m;
  size_t b = (size_t)gram_splits(p.m, p.m, p.n_eff) * p.m * p.m;
  if (p.sliced) {
    a *= 3;     // column ranges for the slice exponents
    b = std::max(b, (size_t)slice_gram_splits(p.m, p.m, p.n_eff, true) * p.m * p.m);
  }
  return a > b ? a : b;
}

int standardize_to(const float* E, int64_t lde, int64_t n_eff, int64_t m, const double* mu,
                   const double* cov, float* Xs, int64_t n_pad, int64_t m_pad, int32_t* st,
                   hipStream_t stream, int32_t* zero, int64_t nzero) {
  dim3 g((unsigned)ceil_div(n_pad, 64), (unsigned)ceil_div(m_pad, 64));
  standardize_transpose_kernel<<<g, 256, 0, stream>>>(E, lde, n_eff, m, mu, cov, Xs, n_pad,
                                                       m_pad, st, zero, nzero);
  VL_LAUNCH_CHECK();
  return VL_OK;
}

// Stages 4-5 with FP32 (plain sums) or FP64 (compensated sums) partials.
template <class TP>
static int launch_moments(const PairwisePlan& p, const PairwiseWs& w, const float* E,
                          int64_t lde, const double* cov, const double* Hx, double* Hr,
                          double* S, double* mom, TP* partU, TP* partB, hipStream_t stream) {
  const int64_t m = p.m, n_eff = p.n_eff;
  {
    ProfileScope ps("pairwise_moments", stream);
    pairwise_moments_kernel<TP><<<(unsigned)p.blocks, 256, 0, stream>>>(
        w.Xs, p.n_pad, w.coef, p.m_pad, m, p.nt, p.tiles, p.chunk_len, p.items, partU, partB);
    VL_LAUNCH_CHECK();
  }
  {
    ProfileScope ps("pairwise_collinear", stream);
    const int64_t blocks = std::min<int64_t>(ceil_div(p.items, 4), 256);
    pairwise_collinear_kernel<TP><<<(unsigned)blocks, 256, 0, stream>>>(
        E, lde, n_eff, w.mu, cov, m, p.nt, p.tiles, p.nc, p.chunk_len, w.clist, partU,
        partB);
    VL_LAUNCH_CHECK();
  }
  {
    ProfileScope ps("pairwise_combine", stream);
    combine_hr_kernel<TP><<<(unsigned)ceil_div(m * m, 256), 256, 0, stream>>>(
        partU, partB, p.nc, m, n_eff, Hr, mom);
    VL_LAUNCH_CHECK();
    score_kernel<<<(unsigned)ceil_div(m * m, 256), 256, 0, stream>>>(Hx, Hr, m, S);
    VL_LAUNCH_CHECK();
  }
  return VL_OK;
}

int run_pairwise(const PairwisePlan& p, const PairwiseWs& w, const float* E, int64_t lde,
                 int prec, double* Hx, double* Hr, double* S, double* Cov, double* mom,
                 int32_t* st, hipStream_t stream) {
  const int64_t m = p.m, n_eff = p.n_eff;
  double* cov = Cov ? Cov : w.cov;
  {
    ProfileScope ps("pairwise_cov", stream);
    int rc = colmeans(E, lde, nullptr, m, n_eff, w.mu, w.scratch, st, stream, nullptr, 0, 0,
                      p.sliced ? w.ex : nullptr);
    if (rc) return rc;
    if (p.sliced) {
      // the covariance from int8 slices of E's centred columns
      rc = slice_columns(E, lde, m, 1, 0, n_eff, w.mu, w.ex, w.slices, stream);
      if (rc) return rc;
      SliceOp D;
      D.D = w.slices;
      D.rows = m;
      D.plane = m * slice_ldk(n_eff);
      D.e = w.ex;
      rc = slice_gram(D, m, D, m, n_eff, 1.0 / (double)n_eff, cov, m, w.scratch, stream, true);
      if (rc) return rc;
    } else {
      // covariance: exact products and FP64 sums (plain FP32 mode: FP32 MFMA throughout)
      const bool fp32 = (prec & ~VL_PAIRWISE_COMPENSATED) == VL_PREC_FP32;
      rc = gram_tn(E, lde, nullptr, w.mu, m, E, lde, nullptr, w.mu, m, n_eff,
                   fp32 ? GramMode::kFp32 : GramMode::kFp64, 1.0 / (double)n_eff, cov, m,
                   w.scratch, stream, true);
      if (rc) return rc;
    }
  }
  {
    ProfileScope ps("pairwise_prep", stream);
    int rc = standardize_to(E, lde, n_eff, m, w.mu, cov, w.Xs, p.n_pad, p.m_pad, st, stream,
                            w.clist, p.tiles + 1);
    if (rc) return rc;
    prep_kernel<<<(unsigned)(m + ceil_div(p.m_pad * p.m_pad, (int64_t)kHxThreads)), kHxThreads,
                  0, stream>>>(w.Xs, p.n_pad, n_eff, Hx, w.momx, cov, m, p.m_pad, w.coef, p.nt,
                               p.tiles, w.clist, st);
    VL_LAUNCH_CHECK();
  }
  if (p.comp)
    return launch_moments(p, w, E, lde, cov, Hx, Hr, S, mom, w.partU64, w.partB64, stream);
  return launch_moments(p, w, E, lde, cov, Hx, Hr, S, mom, w.partU, w.partB, stream);
}

}  // namespace vl
