// Chain rule from the brick kernels' per-primitive sums to the 11 parameters,
// fused with the bias-corrected Adam step (Sec. III-F cites Kingma and Ba).
//
// Inputs per primitive (from the fused brick kernel, e = r G, d = p - mu):
// S_e = sum e,  S_ed = sum e d,  D_e = sum e d d^T, either accumulated by
// atomics or summed over the primitive's per-brick partials in a fixed order
// (deterministic) by k_reduce_parts first.  With g = c e the weighted sums are
// S_gd = c S_ed and D = c D_e (c is the same in every brick, so it is applied
// here once).
//   dL/dc    = S_e
//   dL/dmu   = P S_gd                      (P = R S^-2 R^T)
//   dL/dl_j  = s_j^-2 (R^T D R)_jj
//   dL/dR    = -D R S^-2, contracted with dR/dq_n (R is quadratic in q_n)
//   dL/dq    = (I - q_n q_n^T) dL/dq_n / |q|   (zero if |q| < 1e-12)
#include "common.h"
#include "devmath.h"

namespace gve {
namespace {

constexpr int kThreads = 256;

struct AdamCoef {
  float lr, b1, b2, eps, inv_bc1, inv_bc2, lmin, lmax;
};

__global__ __launch_bounds__(kThreads) void k_update(int mode, float* __restrict__ theta,
                                                     float* __restrict__ m, float* __restrict__ v,
                                                     float* __restrict__ acc,
                                                     const float* __restrict__ part,
                                                     const uint32_t* __restrict__ offset,
                                                     const float* __restrict__ grad_in,
                                                     float* __restrict__ grad_out, int64_t n,
                                                     AdamCoef ac,
                                                     unsigned long long* __restrict__ nclamp,
                                                     const uint32_t* __restrict__ fits) {
  // a binning that did not fit its buffers produced no gradient: no step
  if (fits && *fits == 0u) return;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  unsigned int clamped = 0, nonfinite = 0;
  if (i < n) {
    float th[11], gr[11];
#pragma unroll
    for (int a = 0; a < 11; ++a) th[a] = theta[a * n + i];
    if (mode == 2) {
#pragma unroll
      for (int a = 0; a < 11; ++a) gr[a] = grad_in[a * n + i];
    } else {
      float s[10];
      if (part) {
#pragma unroll
        for (int a = 0; a < 10; ++a) s[a] = 0.0f;
        const uint32_t pe = offset[i + 1];
        for (uint32_t p = offset[i]; p < pe; ++p) {
#pragma unroll
          for (int a = 0; a < 10; ++a) s[a] += part[(size_t)p * 10 + a];
        }
      } else {
#pragma unroll
        for (int a = 0; a < 10; ++a) {
          s[a] = acc[i * kAccStride + a];
          acc[i * kAccStride + a] = 0.0f;
        }
      }
      const float c = th[10];
      const float sgd[3] = {c * s[1], c * s[2], c * s[3]};
      const float Dv[6] = {c * s[4], c * s[5], c * s[6], c * s[7], c * s[8], c * s[9]};
      geometry_grad(&th[3], &th[7], sgd, Dv, gr);
      gr[10] = s[0];
    }
    if (mode == 0) {
#pragma unroll
      for (int a = 0; a < 11; ++a) grad_out[a * n + i] = gr[a];
    } else {
#pragma unroll
      for (int a = 0; a < 11; ++a) {
        float mm = m[a * n + i], vv = v[a * n + i];
        mm = ac.b1 * mm + (1.0f - ac.b1) * gr[a];
        vv = ac.b2 * vv + (1.0f - ac.b2) * gr[a] * gr[a];
        m[a * n + i] = mm;
        v[a * n + i] = vv;
        float p = th[a] - ac.lr * (mm * ac.inv_bc1) / (sqrtf(vv * ac.inv_bc2) + ac.eps);
        if (a >= 7 && a <= 9) {
          if (p < ac.lmin) { p = ac.lmin; ++clamped; }
          if (p > ac.lmax) { p = ac.lmax; ++clamped; }
        }
        nonfinite += isfinite(p) ? 0u : 1u;
        theta[a * n + i] = p;
      }
    }
  }
  if (mode != 0 && nclamp) {
    unsigned long long c = clamped, b = nonfinite;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      c += __shfl_xor(c, d, 64);
      b += __shfl_xor(b, d, 64);
    }
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&nclamp[0], c);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(&nclamp[1], b);
  }
}

// Per-primitive sums of the per-pair partials in a fixed order, one wave per
// primitive: the primitive's c slots are 10 c contiguous floats; lane l < 60
// reads elements l, l + 60, l + 120, ... (always component l % 10, coalesced
// 240-byte rows) into four interleaved partial sums, then lanes c, c + 10,
// ..., c + 50 are combined in that order.  Writes acc[i * kAccStride + slot]
// (the update then reads and clears acc).
__global__ __launch_bounds__(kThreads) void k_reduce_parts(const float* __restrict__ part,
                                                           const uint32_t* __restrict__ offset,
                                                           int64_t n, float* __restrict__ acc) {
  const int64_t i = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const size_t a = (size_t)offset[i] * 10, e = (size_t)offset[i + 1] * 10;
  // four independent loads in flight per lane; the sum order stays fixed
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
  if (lane < 60) {
    size_t k = a + (size_t)lane;
    for (; k + 180 < e; k += 240) {
      s0 += part[k];
      s1 += part[k + 60];
      s2 += part[k + 120];
      s3 += part[k + 180];
    }
    for (; k < e; k += 60) s0 += part[k];
  }
  const float s = (s0 + s1) + (s2 + s3);
  float t = s;
#pragma unroll
  for (int r = 1; r < 6; ++r) t += __shfl(s, lane + 10 * r, 64);
  if (lane < 10) acc[i * kAccStride + lane] = t;
}

}  // namespace

hipError_t launch_update(int mode, float* theta, float* m, float* v, float* acc,
                         const float* part, const uint32_t* offset, const float* grad_in,
                         float* grad_out, int64_t n, int64_t t, const gve_options& opt,
                         unsigned long long* clamp_count, hipStream_t s, const uint32_t* fits) {
  AdamCoef ac;
  ac.lr = opt.lr;
  ac.b1 = opt.beta1;
  ac.b2 = opt.beta2;
  ac.eps = opt.eps;
  const double tt = (double)(t > 0 ? t : 1);
  ac.inv_bc1 = (float)(1.0 / (1.0 - pow((double)opt.beta1, tt)));
  ac.inv_bc2 = (float)(1.0 / (1.0 - pow((double)opt.beta2, tt)));
  ac.lmin = opt.ell_min;
  ac.lmax = opt.ell_max;
  if (part && mode != 2) {
    const unsigned wblocks = (unsigned)((n * 64 + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_reduce_parts, dim3(wblocks), dim3(kThreads), 0, s, part, offset, n, acc);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    part = nullptr;
  }
  const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_update, dim3(blocks), dim3(kThreads), 0, s, mode, theta, m, v, acc, part,
                     offset, grad_in, grad_out, n, ac, clamp_count, fits);
  return hipGetLastError();
}

}  // namespace gve
