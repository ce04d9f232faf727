// Issue-rate probes that give the roofline denominators their measured values on the part the
// library runs on: FP32 exp2 (the transcendental unit the pairwise moments are bound by), FP32
// FMA (ordinary VALU), and FP64 MFMA 16x16x4 (the FP64 Gram / residual products).  Each kernel
// runs independent dependency chains per lane (enough to cover the pipeline latency), writes a
// value that depends on every chain so nothing is removed, and is timed with HIP events.
#include "common.hpp"

namespace vl {

constexpr int kProbeChains = 8;

__global__ __launch_bounds__(256) void probe_exp2_kernel(float* __restrict__ out, int iters) {
  float v[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) v[c] = 1e-3f * (float)(threadIdx.x + c);
  // v <- 2^-v: a pure chain of transcendentals (the negation is an input modifier), which
  // settles at the fixed point near 0.64
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) v[c] = __builtin_amdgcn_exp2f(-v[c]);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) s += v[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void probe_fma_kernel(float* __restrict__ out, int iters) {
  float v[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) v[c] = 1e-3f * (float)(threadIdx.x + c);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) v[c] = fmaf(v[c], 0.999f, 1e-4f);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) s += v[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

typedef double f64x4p __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void probe_mfma_f64_kernel(double* __restrict__ out,
                                                             int iters) {
  f64x4p acc[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) acc[c] = f64x4p{0.0, 0.0, 0.0, 0.0};
  const double a = 1e-3 * (double)(threadIdx.x & 63), b = 0.5;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c)
      acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace vl

using namespace vl;

namespace {
int probe_shape(int* blocks) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return VL_ERR_HIP;
  *blocks = 8 * cus;                    // 8 workgroups of 4 waves per CU: 8 waves per SIMD
  return VL_OK;
}
}  // namespace

extern "C" size_t varlingam_probe_workspace_bytes(void) {
  int blocks = 0;
  if (probe_shape(&blocks) != VL_OK) return 0;
  return (size_t)blocks * 256 * sizeof(double);
}

extern "C" int varlingam_probe_rates(double* rates, void* ws, size_t ws_bytes, void* stream) {
  if (!rates || !ws) return VL_ERR_INVALID_ARG;
  int blocks = 0;
  if (probe_shape(&blocks) != VL_OK) return VL_ERR_HIP;
  const int threads = 256;
  if (ws_bytes < (size_t)blocks * threads * sizeof(double)) return VL_ERR_WORKSPACE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double* buf = static_cast<double*>(ws);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return VL_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return VL_ERR_HIP;
  }
  int rc = VL_OK;
  auto timed = [&](auto launch, double work) -> double {
    launch();                                       // warm-up
    hipEventRecord(e0, s);
    launch();
    hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) {
      rc = VL_ERR_HIP;
      return 0.0;
    }
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    return ms > 0.f ? work / (ms * 1e-3) : 0.0;
  };
  const int it_t = 4096, it_f = 16384, it_m = 2048;
  const double lanes = (double)blocks * threads;
  // exp2 per second, FP32 FMA flop per second (2 per FMA), FP64 MFMA flop per second
  rates[0] = timed([&] { probe_exp2_kernel<<<blocks, threads, 0, s>>>((float*)buf, it_t); },
                   lanes * it_t * kProbeChains);
  rates[1] = timed([&] { probe_fma_kernel<<<blocks, threads, 0, s>>>((float*)buf, it_f); },
                   2.0 * lanes * it_f * kProbeChains);
  rates[2] = timed([&] { probe_mfma_f64_kernel<<<blocks, threads, 0, s>>>(buf, it_m); },
                   (double)blocks * (threads / 64) * it_m * kProbeChains * 16.0 * 16.0 * 4.0 *
                       2.0);
  if (hipGetLastError() != hipSuccess) rc = VL_ERR_HIP;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}
