// Device-wide exclusive prefix scan of uint32 values (reduce-then-scan).
//
// Used to turn per-primitive brick-overlap counts into write offsets for the
// (brick, primitive) pair list.  A tile of 1024 values is scanned per 256-lane
// workgroup; tile totals are scanned recursively and added back.
#include "common.h"

namespace gve {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;
constexpr int kTile = kThreads * kPerThread;

__device__ inline uint32_t wave_inclusive_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Exclusive scan of one value per thread across the workgroup; *total gets the sum.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[kThreads / 64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    uint32_t s = wsum[w];
    before += (w < wave) ? s : 0u;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

__global__ __launch_bounds__(kThreads) void k_tile_reduce(const uint32_t* __restrict__ in,
                                                          int64_t n, uint32_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kTile;
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    int64_t i = base + (int64_t)j * kThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  uint32_t total;
  (void)block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Scans one tile per workgroup; adds the tile offset (if given) and writes
// out[i] for i < n, plus out[n] = grand total from the last tile.
__global__ __launch_bounds__(kThreads) void k_tile_scan(const uint32_t* __restrict__ in, int64_t n,
                                                        const uint32_t* __restrict__ tile_off,
                                                        uint32_t* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kPerThread;
  uint32_t x[kPerThread];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    int64_t i = base + j;
    x[j] = (i < n) ? in[i] : 0u;
    s += x[j];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(s, &total);
  const uint32_t off = tile_off ? tile_off[blockIdx.x] : 0u;
  run += off;
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    int64_t i = base + j;
    if (i < n) out[i] = run;
    run += x[j];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = off + total;
}

// One workgroup scans up to kSmallTiles tiles in order, carrying the running
// total: one launch instead of three for the short scans of small workloads.
constexpr int kSmallTiles = 8;

__global__ __launch_bounds__(kThreads) void k_small_scan(const uint32_t* __restrict__ in,
                                                         int64_t n, uint32_t* __restrict__ out) {
  uint32_t carry = 0;
  for (int64_t base0 = 0; base0 < n; base0 += kTile) {
    const int64_t base = base0 + (int64_t)threadIdx.x * kPerThread;
    uint32_t x[kPerThread];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) {
      const int64_t i = base + j;
      x[j] = (i < n) ? in[i] : 0u;
      s += x[j];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, &total) + carry;
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) {
      const int64_t i = base + j;
      if (i < n) out[i] = run;
      run += x[j];
    }
    carry += total;
  }
  if (threadIdx.x == 0) out[n] = carry;
}

__global__ void k_store_zero(uint32_t* p) { *p = 0u; }

int64_t ntiles(int64_t n) { return (n + kTile - 1) / kTile; }

}  // namespace

size_t scan_tmp_bytes(int64_t n) {
  size_t b = 0;
  while (n > kTile) {
    int64_t t = ntiles(n);
    b += 2 * (size_t)(t + 1) * sizeof(uint32_t);
    n = t;
  }
  return b + 256;
}

hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, void* tmp,
                              hipStream_t s) {
  if (n <= 0) {
    hipLaunchKernelGGL(k_store_zero, dim3(1), dim3(1), 0, s, out);
    return hipGetLastError();
  }
  if (n <= kTile) {
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kThreads), 0, s, in, n, nullptr, out);
    return hipGetLastError();
  }
  if (n <= (int64_t)kSmallTiles * kTile) {
    hipLaunchKernelGGL(k_small_scan, dim3(1), dim3(kThreads), 0, s, in, n, out);
    return hipGetLastError();
  }
  const int64_t t = ntiles(n);
  uint32_t* sums = static_cast<uint32_t*>(tmp);
  uint32_t* offs = sums + (t + 1);
  hipLaunchKernelGGL(k_tile_reduce, dim3((unsigned)t), dim3(kThreads), 0, s, in, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive_u32(sums, offs, t, offs + (t + 1), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)t), dim3(kThreads), 0, s, in, n, offs, out);
  return hipGetLastError();
}

}  // namespace gve
