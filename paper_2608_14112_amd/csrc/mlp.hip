// Learned warm start: per-primitive features, a 16-128-128-11 GELU network
// run on bfloat16 matrix cores with float32 accumulation, its training
// (backward GEMMs, bias and GELU gradients, Adam on float32 master weights),
// and the warm-start application with its fallback to the plain allocation.
//
// GEMMs use v_mfma_f32_16x16x16_bf16: a 256-lane workgroup computes a 64x64
// output tile (each wave 32x32 = 2x2 MFMA tiles), staging 64x16 / 16x64
// operand tiles in LDS after rounding float32 to bfloat16 (nearest even).
// Operand fragments: lane l holds A[l % 16][4 (l / 16) + j] and
// B[4 (l / 16) + j][l % 16]; results D[4 (l / 16) + j][l % 16], j = 0..3.
// Large-K products (weight gradients over the batch) are split over K into
// per-split partial tiles that a second kernel sums in a fixed order.
#include "common.h"
#include "devmath.h"

namespace gve {
namespace {

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;
constexpr int kK = 16;

__device__ inline unsigned short f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ inline float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// C (+ split offset) = op(A) op(B) (+ bias); EPI 1 also writes gelu(C) to C2.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A,
                                              int lda, const float* __restrict__ B, int ldb,
                                              float* __restrict__ C, int ldc,
                                              const float* __restrict__ bias,
                                              float* __restrict__ C2, int kchunk,
                                              size_t split_stride) {
  __shared__ unsigned short As[kTile][kK + 4];
  __shared__ unsigned short Bs[kK][kTile + 4];
  const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  float4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) acc[i][jj] = float4v{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += kK) {
    {
      const int r = t >> 2, kk = (t & 3) * 4;
      const int m = m0 + r;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + kk + j;
        float v = 0.0f;
        if (m < M && k < kend) v = TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
        As[r][kk + j] = f2bf(v);
      }
    }
    {
      const int kk = t >> 4, c = (t & 15) * 4;
      const int k = k0 + kk;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = n0 + c + j;
        float v = 0.0f;
        if (n < N && k < kend) v = TB ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n];
        Bs[kk][c + j] = f2bf(v);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      short4v a;
#pragma unroll
      for (int j = 0; j < 4; ++j) a[j] = (short)As[wm + 16 * i + (lane & 15)][4 * (lane >> 4) + j];
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        short4v b;
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = (short)Bs[4 * (lane >> 4) + j][wn + 16 * jj + (lane & 15)];
        acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[i][jj], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  float* Cz = C + (size_t)blockIdx.z * split_stride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + j;
        const int n = n0 + wn + 16 * jj + (lane & 15);
        if (m < M && n < N) {
          float v = acc[i][jj][j];
          if (bias) v += bias[n];
          Cz[(size_t)m * ldc + n] = v;
          if (EPI == 1) C2[(size_t)m * ldc + n] = gelu_f(v);
        }
      }
}

__global__ void k_sum_splits(const float* __restrict__ parts, int splits, int M, int N,
                             size_t stride, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  float s = 0.0f;
  for (int z = 0; z < splits; ++z) s += parts[(size_t)z * stride + i];
  out[i] = s;
}

// dZ = dH * gelu'(Z), in place on dH.
__global__ void k_gelu_back(float* __restrict__ dH, const float* __restrict__ Z, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dH[i] *= gelu_grad_f(Z[i]);
}

// Column sums of a [rows][cols] matrix (bias gradients), fixed order.
__global__ void k_colsum(const float* __restrict__ X, int rows, int cols, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.0f;
  for (int r = 0; r < rows; ++r) s += X[(size_t)r * cols + c];
  out[c] = s;
}

// dY = 2 (Y - T) / (rows * cols); per-block double partial of sum (Y - T)^2.
__global__ __launch_bounds__(256) void k_mse_grad(const float* __restrict__ Y,
                                                  const float* __restrict__ T, int64_t n,
                                                  float scale, float* __restrict__ dY,
                                                  double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float r = Y[i] - T[i];
    s += (double)r * r;
    if (dY) dY[i] = 2.0f * r * scale;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_double(const double* __restrict__ part, int np, double scale,
                             double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < np; ++i) s += part[i];
  *out += s * scale;
}

// Bias-corrected Adam on a flat float32 array.
__global__ void k_adam_flat(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                            float eps, float ibc1, float ibc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mm = b1 * m[i] + (1.0f - b1) * gi;
  const float vv = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mm;
  v[i] = vv;
  w[i] -= lr * (mm * ibc1) / (sqrtf(vv * ibc2) + eps);
}

// Per-column mean and standard deviation (double) of a [rows][cols] matrix.
__global__ void k_colstats(const float* __restrict__ X, int64_t rows, int cols,
                           float* __restrict__ mean, float* __restrict__ stdv) {
  __shared__ double s1[256], s2[256];
  const int c = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t r = threadIdx.x; r < rows; r += 256) {
    const double x = X[(size_t)r * cols + c];
    a += x;
    b += x * x;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mu = s1[0] / (double)rows;
    double var = s2[0] / (double)rows - mu * mu;
    if (var < 0.0) var = 0.0;
    const double sd = sqrt(var);
    mean[c] = (float)mu;
    stdv[c] = (float)(sd > 1e-6 ? sd : 1.0);
  }
}

// out[r][c] = (X[perm[r]][c] - mean[c]) / std[c]   (perm may be null)
__global__ void k_standardize(const float* __restrict__ X, const uint32_t* __restrict__ perm,
                              int64_t rows, int cols, const float* __restrict__ mean,
                              const float* __restrict__ stdv, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int64_t r = i / cols;
  const int c = (int)(i % cols);
  const int64_t src = perm ? (int64_t)perm[r] : r;
  out[i] = (X[(size_t)src * cols + c] - mean[c]) / stdv[c];
}

// Random 32-bit keys and identity values for an epoch's permutation.
__global__ void k_perm_keys(uint32_t* __restrict__ keys, uint32_t* __restrict__ vals, int64_t n,
                            uint64_t seed, uint64_t epoch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  keys[i] = (uint32_t)(hash_bits(seed, epoch, (uint64_t)i) >> 32);
  vals[i] = (uint32_t)i;
}

// ---- features --------------------------------------------------------------

// Inclusive prefix sums of V and V^2 along x (one workgroup per (y, z) line).
__global__ __launch_bounds__(256) void k_sat_x(const float* __restrict__ f, int64_t nx,
                                               double* __restrict__ s1, double* __restrict__ s2) {
  __shared__ double c1[256], c2[256];
  const size_t base = (size_t)blockIdx.x * nx;
  double carry1 = 0.0, carry2 = 0.0;
  for (int64_t x0 = 0; x0 < nx; x0 += 256) {
    const int64_t x = x0 + threadIdx.x;
    const double v = x < nx ? (double)f[base + x] : 0.0;
    c1[threadIdx.x] = v;
    c2[threadIdx.x] = v * v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
      const double a = threadIdx.x >= (unsigned)d ? c1[threadIdx.x - d] : 0.0;
      const double b = threadIdx.x >= (unsigned)d ? c2[threadIdx.x - d] : 0.0;
      __syncthreads();
      c1[threadIdx.x] += a;
      c2[threadIdx.x] += b;
      __syncthreads();
    }
    if (x < nx) {
      s1[base + x] = carry1 + c1[threadIdx.x];
      s2[base + x] = carry2 + c2[threadIdx.x];
    }
    carry1 += c1[255];
    carry2 += c2[255];
    __syncthreads();
  }
}

// Running sums along an axis with element stride `stride` (line = thread).
__global__ void k_sat_axis(double* __restrict__ s1, double* __restrict__ s2, int64_t nlines,
                           int64_t inner, int64_t len, int64_t stride) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nlines) return;
  const size_t base = (size_t)(l / inner) * (size_t)(inner * len) + (size_t)(l % inner);
  double a = 0.0, b = 0.0;
  for (int64_t k = 0; k < len; ++k) {
    const size_t o = base + (size_t)k * stride;
    a += s1[o];
    b += s2[o];
    s1[o] = a;
    s2[o] = b;
  }
}

__device__ inline double sat_at(const double* __restrict__ S, int64_t nx, int64_t ny, int64_t x,
                                int64_t y, int64_t z) {
  if (x < 0 || y < 0 || z < 0) return 0.0;
  return S[(size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * (size_t)z)];
}

__device__ inline double box_sum(const double* __restrict__ S, int64_t nx, int64_t ny, int64_t xa,
                                 int64_t xb, int64_t ya, int64_t yb, int64_t za, int64_t zb) {
  return sat_at(S, nx, ny, xb, yb, zb) - sat_at(S, nx, ny, xa - 1, yb, zb) -
         sat_at(S, nx, ny, xb, ya - 1, zb) - sat_at(S, nx, ny, xb, yb, za - 1) +
         sat_at(S, nx, ny, xa - 1, ya - 1, zb) + sat_at(S, nx, ny, xa - 1, yb, za - 1) +
         sat_at(S, nx, ny, xb, ya - 1, za - 1) - sat_at(S, nx, ny, xa - 1, ya - 1, za - 1);
}

struct FeatArgs {
  const float* f;
  const float* theta;
  int64_t n, n_detail;
  gve_grid g;
  double g99;
  float k;
  const double* s1;
  const double* s2;
  const double* J6;  // [n][6] structure tensors at the centres (k_feat_tensor)
  float* X;  // [n][16]
};

// The voxel nearest primitive i's centre, clamped to the grid.
__device__ inline void centre_voxel(const float* __restrict__ theta, int64_t n, int64_t i,
                                    const gve_grid& g, int64_t c[3]) {
  const double mu[3] = {theta[0 * n + i], theta[1 * n + i], theta[2 * n + i]};
  const int64_t org[3] = {g.x0, g.y0, g.z0};
  const int64_t dim[3] = {g.nx, g.ny, g.nz};
  for (int ax = 0; ax < 3; ++ax) {
    int64_t v = (int64_t)floor(mu[ax] - (double)org[ax] + 0.5);
    c[ax] = v < 0 ? 0 : (v > dim[ax] - 1 ? dim[ax] - 1 : v);
  }
}

// One wave per primitive: the structure tensor at its centre voxel.
__global__ __launch_bounds__(256) void k_feat_tensor(const float* __restrict__ f,
                                                     const float* __restrict__ theta, int64_t n,
                                                     gve_grid g, double* __restrict__ J6) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;  // wave-uniform
  int64_t c[3];
  centre_voxel(theta, n, i, g, c);
  wave_structure_tensor(f, Dims{g.nx, g.ny, g.nz}, c[0], c[1], c[2], J6 + 6 * i);
}

__global__ __launch_bounds__(128) void k_features(FeatArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 128 + threadIdx.x;
  if (i >= a.n) return;
  const int64_t n = a.n;
  const Dims d{a.g.nx, a.g.ny, a.g.nz};
  const double mu[3] = {a.theta[0 * n + i], a.theta[1 * n + i], a.theta[2 * n + i]};
  const int64_t org[3] = {a.g.x0, a.g.y0, a.g.z0};
  const int64_t dim[3] = {a.g.nx, a.g.ny, a.g.nz};
  int64_t c[3];
  centre_voxel(a.theta, n, i, a.g, c);
  // structure tensor at the seed voxel, from k_feat_tensor
  const double* t = a.J6 + 6 * i;
  double J[3][3] = {{t[0], t[1], t[2]}, {t[1], t[3], t[4]}, {t[2], t[4], t[5]}};
  double lam[3] = {0, 0, 0};
  double E[3][3] = {{0, 0, 1}, {0, 1, 0}, {1, 0, 0}};  // rows: e1, e2, e3
  if (J[0][0] + J[1][1] + J[2][2] >= 1e-12) {
    double Am[3][3], V[3][3];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) Am[r][q] = J[r][q];
    jacobi3(Am, V);
    double w[3] = {Am[0][0], Am[1][1], Am[2][2]};
    int idx[3] = {0, 1, 2};  // descending
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 3; ++q)
        if (w[idx[q]] > w[idx[p]]) { int t = idx[p]; idx[p] = idx[q]; idx[q] = t; }
    for (int r = 0; r < 3; ++r) {
      const int e = idx[r];
      lam[r] = w[e];
      int am = 0;
      double best = fabs(V[0][e]);
      for (int q = 1; q < 3; ++q)
        if (fabs(V[q][e]) > best) { best = fabs(V[q][e]); am = q; }
      const double sg = V[am][e] < 0.0 ? -1.0 : 1.0;
      for (int q = 0; q < 3; ++q) E[r][q] = sg * V[q][e];
    }
  }
  float* out = a.X + (size_t)i * 16;
  const double gg = a.g99 > 0.0 ? a.g99 * a.g99 : 1.0;
  for (int r = 0; r < 3; ++r) out[r] = (float)log1p(fmax(lam[r], 0.0) / gg);
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) out[3 + 3 * r + q] = (float)E[r][q];
  const int64_t vox = c[0] + d.nx * (c[1] + d.ny * c[2]);
  out[12] = a.g99 > 0.0 ? (float)((double)grad_mag32(a.f, d, vox) / a.g99) : 0.0f;
  // mean and variance of V over the k-sigma box (summed-area tables)
  double qw = a.theta[3 * n + i], qx = a.theta[4 * n + i], qy = a.theta[5 * n + i],
         qz = a.theta[6 * n + i];
  const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  if (qn >= 1e-12) { qw /= qn; qx /= qn; qy /= qn; qz /= qn; } else { qw = 1; qx = qy = qz = 0; }
  const double R[3][3] = {{1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
                          {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
                          {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
  const double s2v[3] = {exp(2.0 * (double)a.theta[7 * n + i]), exp(2.0 * (double)a.theta[8 * n + i]),
                         exp(2.0 * (double)a.theta[9 * n + i])};
  int64_t lo[3], hi[3];
  bool empty = false;
  for (int ax = 0; ax < 3; ++ax) {
    const double sd = R[ax][0] * R[ax][0] * s2v[0] + R[ax][1] * R[ax][1] * s2v[1] +
                      R[ax][2] * R[ax][2] * s2v[2];
    const double h = (double)a.k * sqrt(sd);
    double lf = ceil(mu[ax] - h - (double)org[ax]), hf = floor(mu[ax] + h - (double)org[ax]);
    lf = fmax(lf, 0.0);
    hf = fmin(hf, (double)(dim[ax] - 1));
    if (lf > hf) empty = true;
    lo[ax] = (int64_t)lf;
    hi[ax] = (int64_t)hf;
  }
  if (!empty) {
    const double cnt = (double)((hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1));
    const double m1 = box_sum(a.s1, d.nx, d.ny, lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]) / cnt;
    const double m2 = box_sum(a.s2, d.nx, d.ny, lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]) / cnt;
    out[13] = (float)m1;
    out[14] = (float)fmax(m2 - m1 * m1, 0.0);
  } else {
    out[13] = 0.0f;
    out[14] = 0.0f;
  }
  out[15] = i < a.n_detail ? 1.0f : 0.0f;
}

// Targets: theta_ref - theta_alloc per primitive, refined q normalised and
// sign-aligned to the allocated q; [n][11].
__global__ void k_targets(const float* __restrict__ ta, const float* __restrict__ tr, int64_t n,
                          float* __restrict__ T) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double q[4], qa[4];
  double nn = 0.0, dot = 0.0;
  for (int c = 0; c < 4; ++c) {
    q[c] = tr[(3 + c) * n + i];
    qa[c] = ta[(3 + c) * n + i];
    nn += q[c] * q[c];
  }
  nn = sqrt(nn);
  if (nn < 1e-30) nn = 1e-30;
  for (int c = 0; c < 4; ++c) {
    q[c] /= nn;
    dot += q[c] * qa[c];
  }
  const double sg = dot < 0.0 ? -1.0 : 1.0;
  float* out = T + (size_t)i * 11;
  for (int c = 0; c < 11; ++c) {
    const double r = (c >= 3 && c <= 6) ? sg * q[c - 3] : (double)tr[c * n + i];
    out[c] = (float)(r - (double)ta[c * n + i]);
  }
}

// theta += alpha * (Y * tstd + tmean)   (Y: standardised network output [n][11])
__global__ void k_apply_delta(float* __restrict__ theta, const float* __restrict__ base,
                              const float* __restrict__ Y, int64_t n, const float* __restrict__ tmean,
                              const float* __restrict__ tstd, float alpha) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < 11; ++c) {
    const float dlt = Y[(size_t)i * 11 + c] * tstd[c] + tmean[c];
    theta[c * n + i] = base[c * n + i] + alpha * dlt;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host-side helpers.

hipError_t mlp_gemm(bool ta, bool tb, int epi, int M, int N, int K, const float* A, int lda,
                    const float* B, int ldb, float* C, int ldc, const float* bias, float* C2,
                    float* split_tmp, size_t split_tmp_floats, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int gx = (N + kTile - 1) / kTile, gy = (M + kTile - 1) / kTile;
  // split long reductions (weight gradients over the batch) into K chunks
  int kchunk = ((K + kK - 1) / kK) * kK;
  int splits = 1;
  if (epi == 0 && !bias && K > 1024 && split_tmp && ldc == N) {
    kchunk = 512;
    splits = (K + kchunk - 1) / kchunk;
    while (splits > 1 && (size_t)splits * M * ldc > split_tmp_floats) {
      kchunk *= 2;
      splits = (K + kchunk - 1) / kchunk;
    }
  }
  if (kchunk <= 0) kchunk = kK;
  float* out = splits > 1 ? split_tmp : C;
  const size_t stride = (size_t)M * ldc;
  const dim3 grid(gx, gy, splits);
#define GVE_GEMM(TA, TB, EPI)                                                                 \
  hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb,   \
                     out, ldc, bias, C2, kchunk, stride)
  if (epi == 1) {
    if (!ta && !tb) GVE_GEMM(false, false, 1);
    else if (!ta && tb) GVE_GEMM(false, true, 1);
    else return hipErrorInvalidValue;
  } else {
    if (!ta && !tb) GVE_GEMM(false, false, 0);
    else if (!ta && tb) GVE_GEMM(false, true, 0);
    else if (ta && !tb) GVE_GEMM(true, false, 0);
    else GVE_GEMM(true, true, 0);
  }
#undef GVE_GEMM
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  const int64_t tot = (int64_t)M * N;
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, split_tmp,
                     splits, M, N, stride, C);
  return hipGetLastError();
}

hipError_t mlp_gelu_back(float* dH, const float* Z, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_gelu_back, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dH, Z, n);
  return hipGetLastError();
}

hipError_t mlp_colsum(const float* X, int rows, int cols, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)((cols + 127) / 128)), dim3(128), 0, s, X, rows, cols,
                     out);
  return hipGetLastError();
}

hipError_t mlp_mse_grad(const float* Y, const float* T, int64_t n, float scale, float* dY,
                        double* part, double* acc_out, double acc_scale, hipStream_t s) {
  hipLaunchKernelGGL(k_mse_grad, dim3(64), dim3(256), 0, s, Y, T, n, scale, dY, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_double, dim3(1), dim3(64), 0, s, part, 64, acc_scale, acc_out);
  return hipGetLastError();
}

hipError_t mlp_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1,
                    float b2, float eps, int64_t t, hipStream_t s) {
  const float ibc1 = (float)(1.0 / (1.0 - pow((double)b1, (double)t)));
  const float ibc2 = (float)(1.0 / (1.0 - pow((double)b2, (double)t)));
  hipLaunchKernelGGL(k_adam_flat, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, m, v, g, n,
                     lr, b1, b2, eps, ibc1, ibc2);
  return hipGetLastError();
}

hipError_t mlp_colstats(const float* X, int64_t rows, int cols, float* mean, float* stdv,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_colstats, dim3(cols), dim3(256), 0, s, X, rows, cols, mean, stdv);
  return hipGetLastError();
}

hipError_t mlp_standardize(const float* X, const uint32_t* perm, int64_t rows, int cols,
                           const float* mean, const float* stdv, float* out, hipStream_t s) {
  const int64_t tot = rows * cols;
  hipLaunchKernelGGL(k_standardize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, perm,
                     rows, cols, mean, stdv, out);
  return hipGetLastError();
}

hipError_t mlp_perm_keys(uint32_t* keys, uint32_t* vals, int64_t n, uint64_t seed, uint64_t epoch,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_perm_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys, vals, n,
                     seed, epoch);
  return hipGetLastError();
}

hipError_t mlp_sat(const float* f, const gve_grid& g, double* s1, double* s2, hipStream_t s) {
  const int64_t lines = g.ny * g.nz;
  hipLaunchKernelGGL(k_sat_x, dim3((unsigned)lines), dim3(256), 0, s, f, g.nx, s1, s2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // along y: lines (x, z), inner = nx, len = ny, stride nx
  const int64_t ly = g.nx * g.nz;
  hipLaunchKernelGGL(k_sat_axis, dim3((unsigned)((ly + 255) / 256)), dim3(256), 0, s, s1, s2, ly,
                     g.nx, g.ny, g.nx);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // along z: lines (x, y), inner = nx * ny, len = nz, stride nx * ny
  const int64_t lz = g.nx * g.ny;
  hipLaunchKernelGGL(k_sat_axis, dim3((unsigned)((lz + 255) / 256)), dim3(256), 0, s, s1, s2, lz,
                     g.nx * g.ny, g.nz, g.nx * g.ny);
  return hipGetLastError();
}

hipError_t mlp_features(const float* f, const float* theta, int64_t n, int64_t n_detail,
                        const gve_grid& g, double g99, float k, const double* s1, const double* s2,
                        double* J6, float* X, hipStream_t s) {
  FeatArgs a{f, theta, n, n_detail, g, g99, k, s1, s2, J6, X};
  hipLaunchKernelGGL(k_feat_tensor, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, f, theta, n, g,
                     J6);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, a);
  return hipGetLastError();
}

hipError_t mlp_targets(const float* ta, const float* tr, int64_t n, float* T, hipStream_t s) {
  hipLaunchKernelGGL(k_targets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ta, tr, n, T);
  return hipGetLastError();
}

hipError_t mlp_apply_delta(float* theta, const float* base, const float* Y, int64_t n,
                           const float* tmean, const float* tstd, float alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_delta, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, base,
                     Y, n, tmean, tstd, alpha);
  return hipGetLastError();
}

}  // namespace gve
