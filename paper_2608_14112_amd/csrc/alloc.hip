// Structure-aware fixed-budget allocation on the device (paper Sec. III-E;
// stages S1a-S1e of the stage table):
//
//   S1a  k_grad         : |grad V| per voxel (float32 central differences,
//                         one-sided at the faces; magnitude formed in double
//                         and rounded to float), occupied / eligible counts.
//   S1b  select + write : the N_det detail seeds (probability ~ |grad V| over
//                         V > 0.02, without replacement: exponential-clock keys
//                         -ln(u)/g, the N_det smallest) and the N_cov coverage
//                         seeds (uniform keys), by MSB-first radix select over
//                         64-bit keys and an order-preserving compaction, ties
//                         to the lower voxel index; u from the SplitMix64
//                         finaliser of the counter (seed, stream, voxel).
//   S1b  k_jitter       : off-grid centre c + u - 1/2 per axis.
//   S1c  k_nn / k_median: per group, the lower median over a strided subsample
//                         (<= 4096 seeds) of nearest-neighbour distances.
//   S1d/e k_assemble    : 7^3 structure tensor, Jacobi eigen
//                         frame R = [e3, e2, e1] (tangent = smallest
//                         eigenvalue), scales from the group spacing elongated
//                         along the tangent with the gradient, value V(c).
//   weights             : one truncated evaluation U = sum a_i G_i, then
//                         kappa = <U, V> / <U, U> scales every weight.
#include "common.h"
#include "devmath.h"

namespace gve {
namespace {

constexpr int kThreads = 256;
constexpr int kVoxPerThread = 16;
constexpr int kBlockVox = kThreads * kVoxPerThread;
constexpr float kOcc = 0.02f;

template <typename T>
__device__ inline T wave_reduce_add(T v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
  return v;
}

// S1a: g32 per voxel and counts of occupied (V > 0.02) and eligible (and g > 0).
__global__ __launch_bounds__(kThreads) void k_grad(const float* __restrict__ f, Dims d, int64_t M,
                                                   float* __restrict__ g32,
                                                   unsigned long long* __restrict__ counts) {
  unsigned long long occ = 0, el = 0;
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < M;
       v += (int64_t)gridDim.x * kThreads) {
    const float g = grad_mag32(f, d, v);
    g32[v] = g;
    const bool o = f[v] > kOcc;
    occ += o;
    el += (o && g > 0.0f);
  }
  occ = wave_reduce_add(occ);
  el = wave_reduce_add(el);
  if ((threadIdx.x & 63) == 0) {
    if (occ) atomicAdd(&counts[0], occ);
    if (el) atomicAdd(&counts[1], el);
  }
}

// Key functions.  Mode 0: detail (candidate V > 0.02 and g > 0; key = bits of
// -ln(u)/g as a positive double, monotone as uint64).  Mode 1: coverage
// (candidate V > 0.02; key = top 53 hash bits).  Mode 2: order statistic of
// g32 over V > 0.02 (key = float bits of g32, monotone for g >= 0).
struct KeyCtx {
  const float* f;
  const float* g32;
  uint64_t seed;
};

template <int MODE>
__device__ inline bool key_of(const KeyCtx& kc, int64_t v, uint64_t* key) {
  const float fv = kc.f[v];
  if (!(fv > kOcc)) return false;
  if (MODE == 0) {
    const float g = kc.g32[v];
    if (!(g > 0.0f)) return false;
    const double u = uniform01(kc.seed, 1, (uint64_t)v);
    const double kd = -log(u) / (double)g;
    *key = (uint64_t)__double_as_longlong(kd);
    return true;
  } else if (MODE == 1) {
    *key = hash_bits(kc.seed, 2, (uint64_t)v) >> 11;
    return true;
  } else {
    *key = (uint64_t)__float_as_uint(kc.g32[v]);
    return true;
  }
}

// Select state in device memory: [0] prefix, [1] remaining rank (1-based
// count of smallest keys still to take at or below the prefix).
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_sel_hist(KeyCtx kc, int64_t M,
                                                       const unsigned long long* __restrict__ st,
                                                       int shift,
                                                       unsigned long long* __restrict__ hist) {
  __shared__ unsigned int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t prefix = st[0];
  const uint64_t hi_mask = (shift + 8 >= 64) ? 0ull : (~0ull << (shift + 8));
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < M;
       v += (int64_t)gridDim.x * kThreads) {
    uint64_t key;
    if (key_of<MODE>(kc, v, &key) && ((key & hi_mask) == (prefix & hi_mask)))
      atomicAdd(&h[(key >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

__global__ void k_sel_step(unsigned long long* __restrict__ st, int shift,
                           unsigned long long* __restrict__ hist) {
  if (threadIdx.x != 0) return;
  unsigned long long k = st[1], cum = 0;
  int d = 0;
  for (; d < 256; ++d) {
    if (cum + hist[d] >= k) break;
    cum += hist[d];
  }
  if (d > 255) d = 255;
  st[0] |= ((unsigned long long)d) << shift;
  st[1] = k - cum;
  for (int e = 0; e < 256; ++e) hist[e] = 0;
}

// Per-block counts of candidates with key < K and key == K.
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_sel_count(KeyCtx kc, int64_t M,
                                                        const unsigned long long* __restrict__ st,
                                                        uint32_t* __restrict__ less_cnt,
                                                        uint32_t* __restrict__ tie_cnt) {
  __shared__ uint32_t sl[kThreads / 64], stt[kThreads / 64];
  const uint64_t K = st[0];
  const int64_t base = (int64_t)blockIdx.x * kBlockVox + (int64_t)threadIdx.x * kVoxPerThread;
  uint32_t nl = 0, nt = 0;
  for (int j = 0; j < kVoxPerThread; ++j) {
    const int64_t v = base + j;
    uint64_t key;
    if (v < M && key_of<MODE>(kc, v, &key)) {
      nl += key < K;
      nt += key == K;
    }
  }
  nl = wave_reduce_add(nl);
  nt = wave_reduce_add(nt);
  if ((threadIdx.x & 63) == 0) {
    sl[threadIdx.x >> 6] = nl;
    stt[threadIdx.x >> 6] = nt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0, b = 0;
    for (int w = 0; w < kThreads / 64; ++w) { a += sl[w]; b += stt[w]; }
    less_cnt[blockIdx.x] = a;
    tie_cnt[blockIdx.x] = b;
  }
}

__global__ void k_take_count(const uint32_t* __restrict__ less_cnt,
                             const uint32_t* __restrict__ tie_cnt,
                             const uint32_t* __restrict__ tie_off,
                             const unsigned long long* __restrict__ st, int64_t nb,
                             uint32_t* __restrict__ take) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int64_t krem = (int64_t)st[1];
  int64_t t = krem - (int64_t)tie_off[b];
  if (t < 0) t = 0;
  if (t > tie_cnt[b]) t = tie_cnt[b];
  take[b] = less_cnt[b] + (uint32_t)t;
}

__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t u = __shfl_up(inc, d, 64);
    if (lane >= d) inc += u;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wave; ++w) before += wsum[w];
  __syncthreads();
  return before + inc - v;
}

// Writes the selected voxel indices in increasing voxel order.
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_sel_write(KeyCtx kc, int64_t M,
                                                        const unsigned long long* __restrict__ st,
                                                        const uint32_t* __restrict__ tie_off,
                                                        const uint32_t* __restrict__ out_off,
                                                        int64_t* __restrict__ out) {
  __shared__ uint32_t wsum[kThreads / 64];
  const uint64_t K = st[0];
  const int64_t krem = (int64_t)st[1];
  const int64_t base = (int64_t)blockIdx.x * kBlockVox + (int64_t)threadIdx.x * kVoxPerThread;
  uint32_t lessm = 0, tiem = 0;
  for (int j = 0; j < kVoxPerThread; ++j) {
    const int64_t v = base + j;
    uint64_t key;
    if (v < M && key_of<MODE>(kc, v, &key)) {
      if (key < K) lessm |= 1u << j;
      else if (key == K) tiem |= 1u << j;
    }
  }
  uint32_t tie_rank = block_excl_scan((uint32_t)__popc(tiem), wsum) + tie_off[blockIdx.x];
  uint32_t takem = lessm;
  for (int j = 0; j < kVoxPerThread; ++j)
    if ((tiem >> j) & 1u) {
      if ((int64_t)tie_rank < krem) takem |= 1u << j;
      ++tie_rank;
    }
  uint32_t pos = block_excl_scan((uint32_t)__popc(takem), wsum) + out_off[blockIdx.x];
  for (int j = 0; j < kVoxPerThread; ++j)
    if ((takem >> j) & 1u) out[pos++] = base + j;
}

// S1c: nearest-neighbour squared distance for subsample s (block per s).
__global__ __launch_bounds__(kThreads) void k_nn(const float* __restrict__ mx,
                                                 const float* __restrict__ my,
                                                 const float* __restrict__ mz, int64_t ng,
                                                 int64_t stride, double* __restrict__ best) {
#pragma clang fp contract(off)
  __shared__ double sh[kThreads];
  const int64_t i = (int64_t)blockIdx.x * stride;
  const double xi = mx[i], yi = my[i], zi = mz[i];
  double b = INFINITY;
  for (int64_t j = threadIdx.x; j < ng; j += kThreads) {
    if (j == i) continue;
    const double dx = (double)mx[j] - xi, dy = (double)my[j] - yi, dz = (double)mz[j] - zi;
    const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const double d2 = (xx + yy) + zz;
    b = fmin(b, d2);
  }
  sh[threadIdx.x] = b;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) best[blockIdx.x] = sh[0];
}

// Lower median of m <= 4096 values -> sqrt, by bitonic sort in LDS.
__global__ __launch_bounds__(1024) void k_median(const double* __restrict__ best, int m,
                                                 double* __restrict__ out) {
  __shared__ double v[4096];
  for (int i = threadIdx.x; i < 4096; i += 1024) v[i] = (i < m) ? best[i] : INFINITY;
  __syncthreads();
  for (int size = 2; size <= 4096; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < 4096; i += 1024) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const double a = v[i], b = v[j];
          if ((a > b) == up) { v[i] = b; v[j] = a; }
        }
      }
      __syncthreads();
    }
  if (threadIdx.x == 0) *out = (m >= 1) ? sqrt(v[(m - 1) / 2]) : 1.0;
}

__device__ inline void quat_from_R(const double R[3][3], double q[4]) {
  const double t = R[0][0] + R[1][1] + R[2][2];
  if (t > 0.0) {
    const double s = sqrt(t + 1.0) * 2.0;
    q[0] = 0.25 * s; q[1] = (R[2][1] - R[1][2]) / s; q[2] = (R[0][2] - R[2][0]) / s;
    q[3] = (R[1][0] - R[0][1]) / s;
  } else if (R[0][0] > R[1][1] && R[0][0] > R[2][2]) {
    const double s = sqrt(1.0 + R[0][0] - R[1][1] - R[2][2]) * 2.0;
    q[0] = (R[2][1] - R[1][2]) / s; q[1] = 0.25 * s; q[2] = (R[0][1] + R[1][0]) / s;
    q[3] = (R[0][2] + R[2][0]) / s;
  } else if (R[1][1] > R[2][2]) {
    const double s = sqrt(1.0 + R[1][1] - R[0][0] - R[2][2]) * 2.0;
    q[0] = (R[0][2] - R[2][0]) / s; q[1] = (R[0][1] + R[1][0]) / s; q[2] = 0.25 * s;
    q[3] = (R[1][2] + R[2][1]) / s;
  } else {
    const double s = sqrt(1.0 + R[2][2] - R[0][0] - R[1][1]) * 2.0;
    q[0] = (R[1][0] - R[0][1]) / s; q[1] = (R[0][2] + R[2][0]) / s; q[2] = (R[1][2] + R[2][1]) / s;
    q[3] = 0.25 * s;
  }
  const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const double sg = (q[0] < 0.0) ? -1.0 : 1.0;
  for (int a = 0; a < 4; ++a) q[a] = sg * q[a] / n;
}

struct AssembleArgs {
  const float* f;
  const float* g32;
  Dims d;
  int64_t x0, y0, z0;
  const int64_t* det;
  const int64_t* cov;
  int64_t n_det, n;
  const double* s_base;   // [2]
  const unsigned long long* g99_bits;  // select state of the percentile (prefix = bits)
  double s_cap;
  uint64_t seed;
  float* theta;           // [11][n]
  const double* J6;       // [n][6] structure tensors at the seeds (k_tensor)
};

// One wave per primitive: the structure tensor at its seed voxel (S1d).
__global__ __launch_bounds__(256) void k_tensor(const float* __restrict__ f, Dims d,
                                                const int64_t* __restrict__ det,
                                                const int64_t* __restrict__ cov, int64_t n_det,
                                                int64_t n, double* __restrict__ J6) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;  // wave-uniform
  const int64_t vox = i < n_det ? det[i] : cov[i - n_det];
  const int64_t ii = vox % d.nx, jj = (vox / d.nx) % d.ny, kk = vox / (d.nx * d.ny);
  wave_structure_tensor(f, d, ii, jj, kk, J6 + 6 * i);
}

__global__ __launch_bounds__(128) void k_assemble(AssembleArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 128 + threadIdx.x;
  if (i >= a.n) return;
  const int group = i < a.n_det ? 0 : 1;
  const int64_t vox = group == 0 ? a.det[i] : a.cov[i - a.n_det];
  const int64_t n = a.n;
  // structure tensor over the clipped 7^3 box (S1d), from k_tensor
  const double* t = a.J6 + 6 * i;
  double J[3][3] = {{t[0], t[1], t[2]}, {t[1], t[3], t[4]}, {t[2], t[4], t[5]}};
  double R[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  if (J[0][0] + J[1][1] + J[2][2] >= 1e-12) {
    double A[3][3], V[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) A[r][c] = J[r][c];
    jacobi3(A, V);
    double w[3] = {A[0][0], A[1][1], A[2][2]};
    int idx[3] = {0, 1, 2};  // ascending eigenvalues
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 3; ++q)
        if (w[idx[q]] < w[idx[p]]) { int t = idx[p]; idx[p] = idx[q]; idx[q] = t; }
    // columns: e3 (smallest), e2, e1 (largest); largest-|.| component positive
    for (int col = 0; col < 3; ++col) {
      const int e = idx[col];
      int am = 0;
      double best = fabs(V[0][e]);
      for (int r = 1; r < 3; ++r)
        if (fabs(V[r][e]) > best) { best = fabs(V[r][e]); am = r; }
      const double sg = (V[am][e] < 0.0) ? -1.0 : 1.0;
      for (int r = 0; r < 3; ++r) R[r][col] = sg * V[r][e];
    }
    const double det = R[0][0] * (R[1][1] * R[2][2] - R[1][2] * R[2][1]) -
                       R[0][1] * (R[1][0] * R[2][2] - R[1][2] * R[2][0]) +
                       R[0][2] * (R[1][0] * R[2][1] - R[1][1] * R[2][0]);
    if (det < 0.0)
      for (int r = 0; r < 3; ++r) R[r][2] = -R[r][2];
  }
  // scales (S1e)
  const double sb = a.s_base[group];
  const float g99 = __uint_as_float((unsigned)a.g99_bits[0]);
  double gh = 0.0;
  if (g99 > 0.0f) gh = fmin(fmax((double)a.g32[vox] / (double)g99, 0.0), 1.0);
  const double st = fmin(sb * (1.0 + 2.0 * gh), 3.0 * sb);
  const double cap = fmax(a.s_cap, 0.25);
  const double s3[3] = {fmin(fmax(st, 0.25), cap), fmin(fmax(sb, 0.25), cap),
                        fmin(fmax(sb, 0.25), cap)};
  double q[4];
  quat_from_R(R, q);
  for (int c = 0; c < 4; ++c) a.theta[(3 + c) * n + i] = (float)q[c];
  for (int c = 0; c < 3; ++c) a.theta[(7 + c) * n + i] = (float)log(s3[c]);
  a.theta[10 * n + i] = a.f[vox];
}

// S1b jitter: centre = (voxel + u) - 1/2 per axis in double, rounded to float.
__global__ __launch_bounds__(256) void k_jitter(Dims d, int64_t x0, int64_t y0, int64_t z0,
                                                const int64_t* __restrict__ det,
                                                const int64_t* __restrict__ cov, int64_t n_det,
                                                int64_t n, uint64_t seed, float* __restrict__ theta) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int group = i < n_det ? 0 : 1;
  const int64_t vox = group == 0 ? det[i] : cov[i - n_det];
  const int64_t base[3] = {vox % d.nx + x0, (vox / d.nx) % d.ny + y0, vox / (d.nx * d.ny) + z0};
  for (int ax = 0; ax < 3; ++ax) {
    const double u = uniform01(seed, 3 + 3 * group + ax, (uint64_t)vox);
    theta[ax * n + i] = (float)(((double)base[ax] + u) - 0.5);
  }
}

__global__ void k_set_state(unsigned long long* __restrict__ st, unsigned long long a,
                            unsigned long long b) {
  if (threadIdx.x == 0) {
    st[0] = a;
    st[1] = b;
  }
}

// Dot products <U, V> and <U, U> in double (two-level, deterministic).
constexpr int kDotBlocks = 1024;
__global__ __launch_bounds__(kThreads) void k_dot_partial(const float* __restrict__ u,
                                                          const float* __restrict__ v, int64_t M,
                                                          double* __restrict__ part) {
  __shared__ double s1[kThreads], s2[kThreads];
  const int64_t per = (M + gridDim.x - 1) / gridDim.x;
  const int64_t a = (int64_t)blockIdx.x * per, e = min(M, a + per);
  double uv = 0.0, uu = 0.0;
  for (int64_t i = a + threadIdx.x; i < e; i += kThreads) {
    const double x = u[i], y = v[i];
    uv += x * y;
    uu += x * x;
  }
  s1[threadIdx.x] = uv;
  s2[threadIdx.x] = uu;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1[0];
    part[2 * blockIdx.x + 1] = s2[0];
  }
}

__global__ __launch_bounds__(kThreads) void k_kappa(const double* __restrict__ part, int np,
                                                    double* __restrict__ kappa) {
  __shared__ double s1[kThreads], s2[kThreads];
  double uv = 0.0, uu = 0.0;
  for (int i = threadIdx.x; i < np; i += kThreads) {
    uv += part[2 * i];
    uu += part[2 * i + 1];
  }
  s1[threadIdx.x] = uv;
  s2[threadIdx.x] = uu;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) kappa[0] = (s2[0] > 0.0) ? s1[0] / s2[0] : 0.0;
}

__global__ void k_scale_row(float* __restrict__ row, int64_t n, const double* __restrict__ kappa) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) row[i] = (float)((double)row[i] * kappa[0]);
}

// Min-max normalisation (Sec. III-B preprocessing).
__global__ __launch_bounds__(kThreads) void k_minmax(const float* __restrict__ f, int64_t M,
                                                     float* __restrict__ part) {
  __shared__ float lo[kThreads], hi[kThreads];
  float a = INFINITY, b = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < M;
       i += (int64_t)gridDim.x * kThreads) {
    a = fminf(a, f[i]);
    b = fmaxf(b, f[i]);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      lo[threadIdx.x] = fminf(lo[threadIdx.x], lo[threadIdx.x + w]);
      hi[threadIdx.x] = fmaxf(hi[threadIdx.x], hi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = lo[0];
    part[2 * blockIdx.x + 1] = hi[0];
  }
}

__global__ __launch_bounds__(kThreads) void k_normalize(float* __restrict__ f, int64_t M,
                                                        const float* __restrict__ part, int np) {
  float a = INFINITY, b = -INFINITY;
  for (int i = 0; i < np; ++i) {
    a = fminf(a, part[2 * i]);
    b = fmaxf(b, part[2 * i + 1]);
  }
  const float span = b - a;
  const float inv = span > 0.0f ? 1.0f / span : 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < M;
       i += (int64_t)gridDim.x * kThreads)
    f[i] = (f[i] - a) * inv;
}

unsigned grid_for(int64_t M) {
  int64_t b = (M + kThreads - 1) / kThreads;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

// ---------------------------------------------------------------------------
// Host-side sequencing (called from the ABI layer with preallocated buffers).

size_t alloc_block_count(int64_t M) { return (size_t)((M + kBlockVox - 1) / kBlockVox); }

hipError_t alloc_grad(const float* f, const gve_grid& g, float* g32, unsigned long long* counts,
                      hipStream_t s) {
  const int64_t M = g.nx * g.ny * g.nz;
  Dims d{g.nx, g.ny, g.nz};
  hipLaunchKernelGGL(k_grad, dim3(grid_for(M)), dim3(kThreads), 0, s, f, d, M, g32, counts);
  return hipGetLastError();
}

// Radix select + compaction.  mode: 0 detail, 1 coverage, 2 percentile of
// g32 (no compaction).  st: 2 u64 (prefix, rank) preset by the caller to
// (0, k); hist: 256 u64 zeroed.  For modes 0/1 writes k voxel indices to out.
hipError_t alloc_select(int mode, const float* f, const float* g32, const gve_grid& g,
                        uint64_t seed, unsigned long long* st, unsigned long long* hist,
                        uint32_t* less_cnt, uint32_t* tie_cnt, uint32_t* tie_off,
                        uint32_t* take_cnt, uint32_t* out_off, void* scan_tmp, int64_t* out,
                        hipStream_t s) {
  const int64_t M = g.nx * g.ny * g.nz;
  KeyCtx kc{f, g32, seed};
  const int top = (mode == 0) ? 56 : (mode == 1 ? 48 : 24);
  for (int shift = top; shift >= 0; shift -= 8) {
    if (mode == 0)
      hipLaunchKernelGGL(k_sel_hist<0>, dim3(grid_for(M)), dim3(kThreads), 0, s, kc, M, st, shift, hist);
    else if (mode == 1)
      hipLaunchKernelGGL(k_sel_hist<1>, dim3(grid_for(M)), dim3(kThreads), 0, s, kc, M, st, shift, hist);
    else
      hipLaunchKernelGGL(k_sel_hist<2>, dim3(grid_for(M)), dim3(kThreads), 0, s, kc, M, st, shift, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sel_step, dim3(1), dim3(64), 0, s, st, shift, hist);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (mode == 2) return hipSuccess;
  const int64_t nb = (int64_t)alloc_block_count(M);
  if (mode == 0)
    hipLaunchKernelGGL(k_sel_count<0>, dim3((unsigned)nb), dim3(kThreads), 0, s, kc, M, st, less_cnt, tie_cnt);
  else
    hipLaunchKernelGGL(k_sel_count<1>, dim3((unsigned)nb), dim3(kThreads), 0, s, kc, M, st, less_cnt, tie_cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive_u32(tie_cnt, tie_off, nb, scan_tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_take_count, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, less_cnt,
                     tie_cnt, tie_off, st, nb, take_cnt);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive_u32(take_cnt, out_off, nb, scan_tmp, s);
  if (e != hipSuccess) return e;
  if (mode == 0)
    hipLaunchKernelGGL(k_sel_write<0>, dim3((unsigned)nb), dim3(kThreads), 0, s, kc, M, st, tie_off, out_off, out);
  else
    hipLaunchKernelGGL(k_sel_write<1>, dim3((unsigned)nb), dim3(kThreads), 0, s, kc, M, st, tie_off, out_off, out);
  return hipGetLastError();
}

hipError_t alloc_spacing(const float* theta, int64_t n, int64_t first, int64_t ng, double* best,
                         double* s_base, hipStream_t s) {
  if (ng < 2) {
    // a single seed has no neighbour: unit spacing
    hipLaunchKernelGGL(k_median, dim3(1), dim3(1024), 0, s, best, 0, s_base);
    return hipGetLastError();
  }
  const int64_t stride = (ng + 4095) / 4096;
  const int64_t m = (ng + stride - 1) / stride;
  hipLaunchKernelGGL(k_nn, dim3((unsigned)m), dim3(kThreads), 0, s, theta + 0 * n + first,
                     theta + 1 * n + first, theta + 2 * n + first, ng, stride, best);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_median, dim3(1), dim3(1024), 0, s, best, (int)m, s_base);
  return hipGetLastError();
}

hipError_t alloc_jitter(const gve_grid& g, const int64_t* det, const int64_t* cov, int64_t n_det,
                        int64_t n, uint64_t seed, float* theta, hipStream_t s) {
  hipLaunchKernelGGL(k_jitter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     Dims{g.nx, g.ny, g.nz}, g.x0, g.y0, g.z0, det, cov, n_det, n, seed, theta);
  return hipGetLastError();
}

hipError_t alloc_set_state(unsigned long long* st, unsigned long long prefix,
                           unsigned long long rank, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(1), dim3(64), 0, s, st, prefix, rank);
  return hipGetLastError();
}

hipError_t alloc_assemble(const float* f, const float* g32, const gve_grid& g, const int64_t* det,
                          const int64_t* cov, int64_t n_det, int64_t n, const double* s_base,
                          const unsigned long long* g99_state, uint64_t seed, float* theta,
                          double* J6, hipStream_t s) {
  AssembleArgs a;
  a.f = f;
  a.g32 = g32;
  a.d = Dims{g.nx, g.ny, g.nz};
  a.x0 = g.x0; a.y0 = g.y0; a.z0 = g.z0;
  a.det = det;
  a.cov = cov;
  a.n_det = n_det;
  a.n = n;
  a.s_base = s_base;
  a.g99_bits = g99_state;
  int64_t mx = g.nx > g.ny ? g.nx : g.ny;
  if (g.nz > mx) mx = g.nz;
  a.s_cap = (double)mx / 16.0;
  a.seed = seed;
  a.theta = theta;
  a.J6 = J6;
  hipLaunchKernelGGL(k_tensor, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, f, a.d, det, cov,
                     n_det, n, J6);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, a);
  return hipGetLastError();
}

size_t alloc_dot_tmp_doubles() { return 2 * kDotBlocks + 8; }

hipError_t alloc_weights(const float* U, const float* f, int64_t M, float* c_row, int64_t n,
                         double* tmp, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(kThreads), 0, s, U, f, M, tmp + 8);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_kappa, dim3(1), dim3(kThreads), 0, s, tmp + 8, kDotBlocks, tmp);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scale_row, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c_row, n, tmp);
  return hipGetLastError();
}

size_t normalize_tmp_floats() { return 2 * 1024; }

hipError_t normalize_field(float* f, int64_t M, float* tmp, hipStream_t s) {
  hipLaunchKernelGGL(k_minmax, dim3(1024), dim3(kThreads), 0, s, f, M, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_normalize, dim3(grid_for(M)), dim3(kThreads), 0, s, f, M, tmp, 1024);
  return hipGetLastError();
}

}  // namespace gve
