// Microbenchmarks of the rates that bound the brick kernels: fp32 FMA issue,
// the transcendental unit (v_exp_f32), HBM streaming, and float atomics laid
// out as the fused kernel issues them (ten lanes into one 64-byte line).  The
// host times each launch with HIP events and divides the work by the time.
#include "common.h"

namespace gve {
namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;  // independent dependency chains per lane

// kChains FMA chains per lane, `iters` steps each: 2 * kChains * iters flops
// per lane.  The multiplier and addend keep every value finite.
__global__ __launch_bounds__(kThreads) void k_probe_fma(float* __restrict__ out, int iters) {
  float a[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) a[j] = 1e-3f * (float)(threadIdx.x + j);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = fmaf(a[j], 0.999999f, 1e-7f);
  }
  float t = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) t += a[j];
  out[(int64_t)blockIdx.x * kThreads + threadIdx.x] = t;
}

// kChains exponential chains per lane: a <- exp2(-a) keeps a in [1/2, 1].
__global__ __launch_bounds__(kThreads) void k_probe_exp(float* __restrict__ out, int iters) {
  float a[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) a[j] = 0.5f + 1e-3f * (float)j;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = __builtin_amdgcn_exp2f(-a[j]);
  }
  float t = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) t += a[j];
  out[(int64_t)blockIdx.x * kThreads + threadIdx.x] = t;
}

// Grid-stride copy of n4 float4 values.
__global__ __launch_bounds__(kThreads) void k_probe_copy(const float4* __restrict__ src,
                                                         float4* __restrict__ dst, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride)
    dst[i] = src[i];
}

// Each wave issues `iters` atomic instructions; in each, lanes 0..9 add to
// ten consecutive floats of one 64-byte line (line index cycling through
// `nlines`), the pattern of the fused kernel's gathered gradient sums.
__global__ __launch_bounds__(kThreads) void k_probe_atomic(float* __restrict__ acc, int64_t nlines,
                                                           int iters) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  for (int i = 0; i < iters; ++i) {
    const int64_t line = (wave * iters + i) % nlines;
    if (lane < 10) unsafeAtomicAdd(&acc[line * kAccStride + lane], 1.0f);
  }
}

}  // namespace

hipError_t launch_probe(int kind, float* buf, int64_t n, int iters, int blocks, hipStream_t s) {
  switch (kind) {
    case kProbeFma:
      hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(kThreads), 0, s, buf, iters);
      break;
    case kProbeExp:
      hipLaunchKernelGGL(k_probe_exp, dim3(blocks), dim3(kThreads), 0, s, buf, iters);
      break;
    case kProbeCopy:
      // n floats = n / 4 float4: the first half is the source, the second
      // the destination
      hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(kThreads), 0, s,
                         reinterpret_cast<const float4*>(buf),
                         reinterpret_cast<float4*>(buf) + n / 8, n / 8);
      break;
    case kProbeAtomic:
      hipLaunchKernelGGL(k_probe_atomic, dim3(blocks), dim3(kThreads), 0, s, buf,
                         n / kAccStride, iters);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int probe_threads() { return kThreads; }
int probe_chains() { return kChains; }

}  // namespace gve
