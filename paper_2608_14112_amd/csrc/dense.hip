// Dense reference path: every (primitive, voxel) pair of the grid is
// evaluated, with no binning and no skipping.  The cost of considering every
// primitive-sample pair is what truncation-aware binning removes (Sec. III-G);
// these kernels compute the same truncated field, loss and gradient sums as
// the brick kernels (every pair still takes the m^2 < k^2 test), so the two
// paths can be timed against each other on the same inputs.
//
//   k_dense_forward  : one lane per voxel, all primitives in index order
//                      (wave-uniform scalar loads of the records).  Writes
//                      Vhat, or with a target the residual r = 2 (Vhat - V)
//                      and each block's share of L = sum (Vhat - V)^2.
//   k_dense_backward : one lane per primitive, a wave walks a chunk of voxels
//                      row by row (the residual read 64 voxels at a time and
//                      handed out with lane reads).  Along a row (fixed dy, dz)
//                      only sum e, sum e dx and sum e dx^2 change per voxel;
//                      the ten gradient sums are formed from them at the end
//                      of each row, then added to the accumulators with float
//                      atomics once per (primitive, chunk).
#include <algorithm>

#include "common.h"

namespace gve {
namespace {

constexpr int kDenseThreads = 256;

struct DenseGrid {
  int64_t nx, ny, nz, x0, y0, z0;
};

__global__ __launch_bounds__(kDenseThreads) void k_dense_forward(
    const Record* __restrict__ rec, int64_t n, DenseGrid g, float thr,
    const float* __restrict__ field, float* __restrict__ out, float* __restrict__ block_loss) {
  __shared__ float red[kDenseThreads / 64];
  const int64_t M = g.nx * g.ny * g.nz;
  const int64_t v = (int64_t)blockIdx.x * kDenseThreads + threadIdx.x;
  const bool live = v < M;
  const int64_t vc = live ? v : M - 1;
  const int64_t ix = vc % g.nx, row = vc / g.nx;
  // coordinates stay below 2^24 in magnitude: exact in int32 and float32
  const float px = (float)(int)(g.x0 + ix);
  const float py = (float)(int)(g.y0 + row % g.ny);
  const float pz = (float)(int)(g.z0 + row / g.ny);
  float acc = 0.0f;
#pragma unroll 4
  for (int64_t i = 0; i < n; ++i) {
    const Record r = rec[i];
    const float dx = px - r.mu[0];
    const float dy = py - r.mu[1];
    const float dz = pz - r.mu[2];
    const float qxy = fmaf(r.s[0], dx, r.s[1] * dy) * dx + r.s[2] * dy * dy;
    const float w = r.sz * (dz - fmaf(r.gx, dx, r.gy * dy));
    const float q = fmaf(-w, w, qxy);
    acc = fmaf(r.c, q > thr ? __builtin_amdgcn_exp2f(q) : 0.0f, acc);
  }
  if (!field) {
    if (live) out[v] = acc;
    return;
  }
  float d = 0.0f;
  if (live) {
    d = acc - field[v];
    out[v] = 2.0f * d;
  }
  float l = d * d;
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) l += __shfl_xor(l, s, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < kDenseThreads / 64; ++w) t += red[w];
    block_loss[blockIdx.x] = t;
  }
}

// Block (x, y): voxel chunk x of `chunk` voxels, primitives 64 y .. 64 y + 63.
__global__ __launch_bounds__(64) void k_dense_backward(const Record* __restrict__ rec, int64_t n,
                                                       DenseGrid g, float thr,
                                                       const float* __restrict__ resid,
                                                       int64_t chunk, float* __restrict__ acc) {
  const int lane = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.y * 64 + lane;
  const bool live = i < n;
  const Record r = rec[live ? i : n - 1];
  const int64_t M = g.nx * g.ny * g.nz;
  const int64_t v0 = (int64_t)blockIdx.x * chunk;
  const int64_t v1 = std::min(M, v0 + chunk);
  float se = 0.0f, sx = 0.0f, sy = 0.0f, sz = 0.0f, sxx = 0.0f, sxy = 0.0f, sxz = 0.0f,
        syy = 0.0f, syz = 0.0f, szz = 0.0f;
  for (int64_t v = v0; v < v1;) {
    // one row segment: voxels v .. v + len - 1 share (iy, iz)
    const int64_t row = v / g.nx;
    const int64_t ix0 = v - row * g.nx;
    const int64_t len = std::min(g.nx - ix0, v1 - v);
    const float dy = (float)(int)(g.y0 + row % g.ny) - r.mu[1];
    const float dz = (float)(int)(g.z0 + row / g.ny) - r.mu[2];
    // per-row parts of qxy and of the column coordinate t = dz - gx dx - gy dy
    const float qa = r.s[1] * dy;
    const float qb = r.s[2] * dy * dy;
    const float tc = dz - r.gy * dy;
    float re = 0.0f, rx = 0.0f, rxx = 0.0f;  // sum e, sum e dx, sum e dx^2 along the row
    for (int64_t xb = 0; xb < len; xb += 64) {
      const int64_t nb = std::min<int64_t>(64, len - xb);
      const float rv = lane < nb ? resid[v + xb + lane] : 0.0f;
      for (int u = 0; u < (int)nb; ++u) {
        const float res = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rv), u));
        const float dx = (float)(int)(g.x0 + ix0 + xb + u) - r.mu[0];
        const float qxy = fmaf(fmaf(r.s[0], dx, qa), dx, qb);
        const float w = r.sz * fmaf(-r.gx, dx, tc);
        const float q = fmaf(-w, w, qxy);
        const float e = res * (live && q > thr ? __builtin_amdgcn_exp2f(q) : 0.0f);
        re += e;
        const float ex = e * dx;
        rx += ex;
        rxx = fmaf(ex, dx, rxx);
      }
    }
    se += re;
    sx += rx;
    sy = fmaf(dy, re, sy);
    sz = fmaf(dz, re, sz);
    sxx += rxx;
    sxy = fmaf(dy, rx, sxy);
    sxz = fmaf(dz, rx, sxz);
    syy = fmaf(dy * dy, re, syy);
    syz = fmaf(dy * dz, re, syz);
    szz = fmaf(dz * dz, re, szz);
    v += len;
  }
  if (!live) return;
  // accumulator order of the brick kernels: e, e dx, e dy, e dz, e dx dx,
  // e dx dy, e dx dz, e dy dy, e dy dz, e dz dz
  float* a = acc + i * kAccStride;
  const float sums[10] = {se, sx, sy, sz, sxx, sxy, sxz, syy, syz, szz};
#pragma unroll
  for (int k = 0; k < 10; ++k)
    if (sums[k] != 0.0f) unsafeAtomicAdd(&a[k], sums[k]);
}

DenseGrid dense_grid(const gve_grid& g) {
  return DenseGrid{g.nx, g.ny, g.nz, g.x0, g.y0, g.z0};
}

}  // namespace

int64_t dense_blocks(const gve_grid& g) {
  return (g.nx * g.ny * g.nz + kDenseThreads - 1) / kDenseThreads;
}

hipError_t launch_dense_forward(const Record* rec, int64_t n, const gve_grid& g, float k,
                                const float* field, float* out, float* block_loss,
                                hipStream_t s) {
  const float thr = -kHalfLog2e * k * k;
  hipLaunchKernelGGL(k_dense_forward, dim3((unsigned)dense_blocks(g)), dim3(kDenseThreads), 0, s,
                     rec, n, dense_grid(g), thr, field, out, block_loss);
  return hipGetLastError();
}

hipError_t launch_dense_backward(const Record* rec, int64_t n, const gve_grid& g, float k,
                                 const float* resid, float* acc, hipStream_t s) {
  const float thr = -kHalfLog2e * k * k;
  const int64_t M = g.nx * g.ny * g.nz;
  const int64_t groups = (n + 63) / 64;
  // about 16K waves in all, chunks of at least 256 voxels
  int64_t chunks = std::max<int64_t>(1, (16384 + groups - 1) / groups);
  chunks = std::min<int64_t>(chunks, std::max<int64_t>(1, M / 256));
  const int64_t chunk = (M + chunks - 1) / chunks;
  chunks = (M + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_dense_backward, dim3((unsigned)chunks, (unsigned)groups), dim3(64), 0, s,
                     rec, n, dense_grid(g), thr, resid, chunk, acc);
  return hipGetLastError();
}

}  // namespace gve
