// Chain rule from the brick kernels' per-primitive sums to the 11 parameters,
// fused with the bias-corrected Adam step (Sec. III-F cites Kingma and Ba).
//
// Inputs per primitive (from the fused brick kernel, e = r G, g = c e,
// d = p - mu):  S_e = sum e,  S_gd = sum g d,  D = sum g d d^T, either
// accumulated by atomics or summed here over the primitive's per-brick
// partials in emission order (deterministic).
//   dL/dc    = S_e
//   dL/dmu   = P S_gd                      (P = R S^-2 R^T)
//   dL/dl_j  = s_j^-2 (R^T D R)_jj
//   dL/dR    = -D R S^-2, contracted with dR/dq_n (R is quadratic in q_n)
//   dL/dq    = (I - q_n q_n^T) dL/dq_n / |q|   (zero if |q| < 1e-12)
#include "common.h"

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
                                                     unsigned long long* __restrict__ nclamp) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  unsigned int clamped = 0;
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
          s[a] = acc[a * n + i];
          acc[a * n + i] = 0.0f;
        }
      }
      float qw = th[3], qx = th[4], qy = th[5], qz = th[6];
      const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
      const bool qok = qn >= 1e-12f;
      const float qinv = qok ? 1.0f / qn : 0.0f;
      if (qok) {
        qw *= qinv; qx *= qinv; qy *= qinv; qz *= qinv;
      } else {
        qw = 1.f; qx = qy = qz = 0.f;
      }
      float R[3][3];
      R[0][0] = 1.f - 2.f * (qy * qy + qz * qz);
      R[0][1] = 2.f * (qx * qy - qw * qz);
      R[0][2] = 2.f * (qx * qz + qw * qy);
      R[1][0] = 2.f * (qx * qy + qw * qz);
      R[1][1] = 1.f - 2.f * (qx * qx + qz * qz);
      R[1][2] = 2.f * (qy * qz - qw * qx);
      R[2][0] = 2.f * (qx * qz - qw * qy);
      R[2][1] = 2.f * (qy * qz + qw * qx);
      R[2][2] = 1.f - 2.f * (qx * qx + qy * qy);
      const float is2[3] = {expf(-2.f * th[7]), expf(-2.f * th[8]), expf(-2.f * th[9])};
      float P[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          P[a][b] = R[a][0] * R[b][0] * is2[0] + R[a][1] * R[b][1] * is2[1] +
                    R[a][2] * R[b][2] * is2[2];
      const float sgd[3] = {s[1], s[2], s[3]};
      const float D[3][3] = {{s[4], s[5], s[6]}, {s[5], s[7], s[8]}, {s[6], s[8], s[9]}};
#pragma unroll
      for (int a = 0; a < 3; ++a) gr[a] = P[a][0] * sgd[0] + P[a][1] * sgd[1] + P[a][2] * sgd[2];
      float M[3][3];  // D R
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) M[a][b] = D[a][0] * R[0][b] + D[a][1] * R[1][b] + D[a][2] * R[2][b];
#pragma unroll
      for (int j = 0; j < 3; ++j)
        gr[7 + j] = is2[j] * (R[0][j] * M[0][j] + R[1][j] * M[1][j] + R[2][j] * M[2][j]);
      float G[3][3];  // dL/dR = -D R S^-2
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) G[a][b] = -M[a][b] * is2[b];
      const float w = qw, x = qx, y = qy, z = qz;
      float dw = 2.f * (-z * G[0][1] + y * G[0][2] + z * G[1][0] - x * G[1][2] - y * G[2][0] +
                        x * G[2][1]);
      float dxq = 2.f * (y * G[0][1] + z * G[0][2] + y * G[1][0] - 2.f * x * G[1][1] -
                         w * G[1][2] + z * G[2][0] + w * G[2][1] - 2.f * x * G[2][2]);
      float dyq = 2.f * (-2.f * y * G[0][0] + x * G[0][1] + w * G[0][2] + x * G[1][0] +
                         z * G[1][2] - w * G[2][0] + z * G[2][1] - 2.f * y * G[2][2]);
      float dzq = 2.f * (-2.f * z * G[0][0] - w * G[0][1] + x * G[0][2] + w * G[1][0] -
                         2.f * z * G[1][1] + y * G[1][2] + x * G[2][0] + y * G[2][1]);
      const float dot = w * dw + x * dxq + y * dyq + z * dzq;
      gr[3] = (dw - w * dot) * qinv;
      gr[4] = (dxq - x * dot) * qinv;
      gr[5] = (dyq - y * dot) * qinv;
      gr[6] = (dzq - z * dot) * qinv;
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
        theta[a * n + i] = p;
      }
    }
  }
  if (mode != 0 && nclamp) {
    unsigned long long c = clamped;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(nclamp, c);
  }
}

}  // namespace

hipError_t launch_update(int mode, float* theta, float* m, float* v, float* acc,
                         const float* part, const uint32_t* offset, const float* grad_in,
                         float* grad_out, int64_t n, int64_t t, const gve_options& opt,
                         unsigned long long* clamp_count, hipStream_t s) {
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
  const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_update, dim3(blocks), dim3(kThreads), 0, s, mode, theta, m, v, acc, part,
                     offset, grad_in, grad_out, n, ac, clamp_count);
  return hipGetLastError();
}

}  // namespace gve
