// Device helpers shared by several kernel files: float32 field gradients
// (central differences, one-sided at the faces), a cyclic Jacobi eigensolver
// for symmetric 3x3 matrices, the counter-based random generator, and the
// chain rule from per-primitive kernel moments to the geometric parameters.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gve {

// SplitMix64 finaliser (Steele, Lea and Flood, 2014) applied to a counter:
// 64 random bits for (seed, stream, idx), and a double uniform in (0, 1].
// The one definition of the library's counter generator (host and device).
static __host__ __device__ inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static __host__ __device__ inline uint64_t hash_bits(uint64_t seed, uint64_t stream,
                                                     uint64_t idx) {
  return splitmix64(splitmix64(seed ^ (stream * 0xD1B54A32D192ED03ull)) ^ idx);
}

// (top 53 bits + 1) * 2^-53: uniform in (0, 1], exact in double.
static __device__ inline double uniform01(uint64_t seed, uint64_t stream, uint64_t idx) {
  return (double)((hash_bits(seed, stream, idx) >> 11) + 1ull) * 0x1.0p-53;
}

// Chain rule for one primitive with raw quaternion q (4), log-scales ell (3):
// from S_gd = sum g d (3) and D = sum g d d^T (xx, xy, xz, yy, yz, zz) of
// d(sum g G)/dtheta written through G's moments, out[0..2] = dmu = P S_gd,
// out[3..6] = dq = (I - q_n q_n^T) dq_n / |q| with dq_n = <-D R S^-2, dR/dq_n>
// (zero if |q| < 1e-12), out[7..9] = dell_j = s_j^-2 (R^T D R)_jj.
static __device__ inline void geometry_grad(const float q[4], const float ell[3],
                                            const float sgd[3], const float Dv[6],
                                            float out[10]) {
  float qw = q[0], qx = q[1], qy = q[2], qz = q[3];
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
  const float is2[3] = {expf(-2.f * ell[0]), expf(-2.f * ell[1]), expf(-2.f * ell[2])};
  float P[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      P[a][b] = R[a][0] * R[b][0] * is2[0] + R[a][1] * R[b][1] * is2[1] + R[a][2] * R[b][2] * is2[2];
  const float D[3][3] = {{Dv[0], Dv[1], Dv[2]}, {Dv[1], Dv[3], Dv[4]}, {Dv[2], Dv[4], Dv[5]}};
#pragma unroll
  for (int a = 0; a < 3; ++a) out[a] = P[a][0] * sgd[0] + P[a][1] * sgd[1] + P[a][2] * sgd[2];
  float M[3][3];  // D R
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) M[a][b] = D[a][0] * R[0][b] + D[a][1] * R[1][b] + D[a][2] * R[2][b];
#pragma unroll
  for (int j = 0; j < 3; ++j)
    out[7 + j] = is2[j] * (R[0][j] * M[0][j] + R[1][j] * M[1][j] + R[2][j] * M[2][j]);
  float G[3][3];  // -D R S^-2
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) G[a][b] = -M[a][b] * is2[b];
  const float w = qw, x = qx, y = qy, z = qz;
  const float dw = 2.f * (-z * G[0][1] + y * G[0][2] + z * G[1][0] - x * G[1][2] - y * G[2][0] +
                          x * G[2][1]);
  const float dxq = 2.f * (y * G[0][1] + z * G[0][2] + y * G[1][0] - 2.f * x * G[1][1] -
                           w * G[1][2] + z * G[2][0] + w * G[2][1] - 2.f * x * G[2][2]);
  const float dyq = 2.f * (-2.f * y * G[0][0] + x * G[0][1] + w * G[0][2] + x * G[1][0] +
                           z * G[1][2] - w * G[2][0] + z * G[2][1] - 2.f * y * G[2][2]);
  const float dzq = 2.f * (-2.f * z * G[0][0] - w * G[0][1] + x * G[0][2] + w * G[1][0] -
                           2.f * z * G[1][1] + y * G[1][2] + x * G[2][0] + y * G[2][1]);
  const float dot = w * dw + x * dxq + y * dyq + z * dzq;
  out[3] = (dw - w * dot) * qinv;
  out[4] = (dxq - x * dot) * qinv;
  out[5] = (dyq - y * dot) * qinv;
  out[6] = (dzq - z * dot) * qinv;
}

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

// Structure tensor at voxel (ci, cj, ck): the sum of g g^T over the 7^3 box
// around it, clipped to the grid, with g the central-difference gradient
// (grad_parts).  Called by all 64 lanes of a wave: the box's voxels are dealt
// to the lanes (voxel t, x fastest, to lane t mod 64), so that a wave's loads
// fall on neighbouring voxels; each lane sums its own in float64, the six
// unique entries (xx, xy, xz, yy, yz, zz) are added across the wave, and
// lanes 0 .. 5 store entry `lane` to J6.
static __device__ inline void wave_structure_tensor(const float* __restrict__ f, Dims d,
                                                    int64_t ci, int64_t cj, int64_t ck,
                                                    double* __restrict__ J6) {
  const int lane = threadIdx.x & 63;
  const int64_t ia = ci - 3 < 0 ? 0 : ci - 3, ib = ci + 3 > d.nx - 1 ? d.nx - 1 : ci + 3;
  const int64_t ja = cj - 3 < 0 ? 0 : cj - 3, jb = cj + 3 > d.ny - 1 ? d.ny - 1 : cj + 3;
  const int64_t ka = ck - 3 < 0 ? 0 : ck - 3, kb = ck + 3 > d.nz - 1 ? d.nz - 1 : ck + 3;
  const int wx = (int)(ib - ia + 1), wy = (int)(jb - ja + 1), wz = (int)(kb - ka + 1);
  const int cnt = wx * wy * wz;
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int t = lane; t < cnt; t += 64) {
    const int x = t % wx, r = t / wx;
    float gx, gy, gz;
    grad_parts(f, d, ia + x, ja + r % wy, ka + r / wy, &gx, &gy, &gz);
    const double X = gx, Y = gy, Z = gz;
    s[0] += X * X; s[1] += X * Y; s[2] += X * Z;
    s[3] += Y * Y; s[4] += Y * Z; s[5] += Z * Z;
  }
  double out = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double v = s[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == k) out = v;
  }
  if (lane < 6) J6[lane] = out;
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
