// Device helpers shared by the allocation and warm-start feature kernels:
// float32 field gradients (central differences, one-sided at the faces) and
// a cyclic Jacobi eigensolver for symmetric 3x3 matrices.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gve {

struct Dims {
  int64_t nx, ny, nz;
};

static __device__ inline float half_diff(const float* __restrict__ f, int64_t v, int64_t i, int64_t n,
                                  int64_t stride) {
  if (n == 1) return 0.0f;
  if (i == 0) return f[v + stride] - f[v];
  if (i == n - 1) return f[v] - f[v - stride];
  return 0.5f * (f[v + stride] - f[v - stride]);
}

static __device__ inline void grad_parts(const float* __restrict__ f, Dims d, int64_t i, int64_t j,
                                  int64_t k, float* gx, float* gy, float* gz) {
  const int64_t v = i + d.nx * (j + d.ny * k);
  *gx = half_diff(f, v, i, d.nx, 1);
  *gy = half_diff(f, v, j, d.ny, d.nx);
  *gz = half_diff(f, v, k, d.nz, d.nx * d.ny);
}

static __device__ inline float grad_mag32(const float* __restrict__ f, Dims d, int64_t v) {
  const int64_t i = v % d.nx, j = (v / d.nx) % d.ny, k = v / (d.nx * d.ny);
  float gx, gy, gz;
  grad_parts(f, d, i, j, k, &gx, &gy, &gz);
  const double x = gx, y = gy, z = gz;
  return (float)sqrt((x * x + y * y) + z * z);
}

// Cyclic Jacobi on a symmetric 3x3 matrix (double); eigenvectors in V's columns.
static __device__ inline void jacobi3(double A[3][3], double V[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) V[a][b] = (a == b) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-32 * dia || off == 0.0) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = (pq == 2) ? 1 : 0;
      const int q = (pq == 0) ? 1 : 2;
      const double apq = A[p][q];
      if (apq == 0.0) continue;
      const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
      const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      A[p][p] -= t * apq;
      A[q][q] += t * apq;
      A[p][q] = A[q][p] = 0.0;
      const int r = 3 - p - q;
      const double arp = A[r][p], arq = A[r][q];
      A[r][p] = A[p][r] = c * arp - s * arq;
      A[r][q] = A[q][r] = s * arp + c * arq;
      for (int k = 0; k < 3; ++k) {
        const double vp = V[k][p], vq = V[k][q];
        V[k][p] = c * vp - s * vq;
        V[k][q] = s * vp + c * vq;
      }
    }
  }
}


}  // namespace gve
