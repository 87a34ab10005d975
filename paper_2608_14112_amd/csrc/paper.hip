// The paper's own training loop on the device (Sec. III-C eq:field, Sec. III-F,
// Table tab:training-config): the density-normalised kernel regression
//     Vt(p) = sum_i w_i a_i G_i(p) / max(sum_i w_i G_i(p), rho0)
// of 12-parameter primitives (mu, raw quaternion, log-scales, attribute a,
// weight logit b with w = sigmoid(b)), trained on a few thousand stratified,
// jittered sample points per iteration against a six-term objective.
//
// Few samples and many primitives: the samples (and a nearby partner of each
// for the smoothness term) are bucketed into a uniform grid of cells; every
// primitive visits the cells its k-sigma box overlaps and tests the points
// there (the paper buckets samples per radius bin and tests a 3^3-cell
// neighbourhood; one grid with a box-sized cell range covers every radius).
//   k_pclass_count : per 256-voxel block, voxels of the high (V > v_hi) and
//                    mid (v_occ < V <= v_hi) classes (ballot counts);
//   k_psample      : one wave per sample: class member j = floor(u n_class)
//                    found through the block prefix sums and a ballot rank
//                    inside the block, jitter, partner, trilinear value;
//   k_pcell_keys   : cell of every point;
//   k_pfwd         : per primitive, sum_i w a G and sum_i w G into the points'
//                    float64 accumulators (atomics);
//   k_pcoef        : per sample, Vt, the loss terms, and the coefficients of
//                    d(w a G) and d(w G) in dL/dtheta (quotient rule; the
//                    density floor passes no gradient);
//   k_pbwd         : per primitive, the gradient from its points (no atomics:
//                    each primitive owns its sums), the regularisers, and
//                    either the gradient (test hook) or the Adam step.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "devmath.h"

namespace gve {
namespace {

constexpr int kThreads = 256;
constexpr int kBlockVox = 256;
constexpr uint64_t kStreamPick = 20, kStreamJit = 21, kStreamPartner = 24;

// ---- primitive geometry ---------------------------------------------------------

struct PGeom {
  float mu[3];
  float P[6];      // precision xx, xy, xz, yy, yz, zz
  float half[3];   // k sqrt(Sigma_jj): the k-sigma box half-extent per axis
  float a, w;
};

__device__ inline PGeom pgeom(const float* __restrict__ th, int64_t n, int64_t i, float k) {
  PGeom g;
  g.mu[0] = th[0 * n + i];
  g.mu[1] = th[1 * n + i];
  g.mu[2] = th[2 * n + i];
  float qw = th[3 * n + i], qx = th[4 * n + i], qy = th[5 * n + i], qz = th[6 * n + i];
  const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  if (qn >= 1e-12f) {
    const float inv = 1.0f / qn;
    qw *= inv; qx *= inv; qy *= inv; qz *= inv;
  } else {
    qw = 1.f; qx = qy = qz = 0.f;
  }
  const float R[3][3] = {
      {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy)},
      {2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx)},
      {2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)}};
  float is2[3], s2[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float l = th[(7 + j) * n + i];
    is2[j] = expf(-2.f * l);
    s2[j] = expf(2.f * l);
  }
  auto prec = [&](int a, int b) {
    return R[a][0] * R[b][0] * is2[0] + R[a][1] * R[b][1] * is2[1] + R[a][2] * R[b][2] * is2[2];
  };
  g.P[0] = prec(0, 0);
  g.P[1] = prec(0, 1);
  g.P[2] = prec(0, 2);
  g.P[3] = prec(1, 1);
  g.P[4] = prec(1, 2);
  g.P[5] = prec(2, 2);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float sig = R[a][0] * R[a][0] * s2[0] + R[a][1] * R[a][1] * s2[1] + R[a][2] * R[a][2] * s2[2];
    g.half[a] = k * sqrtf(sig) * (1.0f + 1e-5f) + 1e-3f;
  }
  g.a = th[10 * n + i];
  g.w = 1.0f / (1.0f + expf(-th[11 * n + i]));
  return g;
}

__device__ inline float mahal2(const PGeom& g, float dx, float dy, float dz) {
  return g.P[0] * dx * dx + g.P[3] * dy * dy + g.P[5] * dz * dz +
         2.0f * (g.P[1] * dx * dy + g.P[2] * dx * dz + g.P[4] * dy * dz);
}

__device__ inline int cell_coord(float x, float org, float h, int nc) {
  const float c = floorf((x - org) / h);
  if (!(c > 0.f)) return 0;  // also NaN
  return c >= (float)nc ? nc - 1 : (int)c;
}

// Trilinear interpolation of the float32 volume at a world point (clamped).
__device__ inline double trilinear(const float* __restrict__ f, const gve_grid& g, double px,
                                   double py, double pz) {
  const double p[3] = {px - (double)g.x0, py - (double)g.y0, pz - (double)g.z0};
  const int64_t dim[3] = {g.nx, g.ny, g.nz};
  int64_t lo[3];
  double fr[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    double x = fmin(fmax(p[j], 0.0), (double)(dim[j] - 1));
    if (dim[j] > 1) {
      int64_t i0 = (int64_t)floor(x);
      if (i0 > dim[j] - 2) i0 = dim[j] - 2;
      lo[j] = i0;
      fr[j] = x - (double)i0;
    } else {
      lo[j] = 0;
      fr[j] = 0.0;
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const int64_t ix = min(lo[0] + dx, dim[0] - 1), iy = min(lo[1] + dy, dim[1] - 1),
                      iz = min(lo[2] + dz, dim[2] - 1);
        const double wgt = (dx ? fr[0] : 1.0 - fr[0]) * (dy ? fr[1] : 1.0 - fr[1]) *
                           (dz ? fr[2] : 1.0 - fr[2]);
        acc += wgt * (double)f[ix + g.nx * (iy + g.ny * iz)];
      }
  return acc;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Block sum of up to three doubles, one atomic per block per value.
__device__ inline void block_add3(double a, double b, double c, double* __restrict__ out) {
  __shared__ double sh[kThreads / 64][3];
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wave][0] = a;
    sh[wave][1] = b;
    sh[wave][2] = c;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w][threadIdx.x];
    if (t != 0.0) atomicAdd(&out[threadIdx.x], t);
  }
}

// ---- sampling -----------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_pclass_count(const float* __restrict__ f, int64_t M,
                                                           float v_hi, float v_occ,
                                                           uint32_t* __restrict__ cnt_hi,
                                                           uint32_t* __restrict__ cnt_mid,
                                                           int64_t nblocks) {
  const int64_t b = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (b >= nblocks) return;
  uint32_t h = 0, m = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t v = b * kBlockVox + 4 * lane + r;
    if (v < M) {
      const float x = f[v];
      h += x > v_hi ? 1u : 0u;
      m += (x > v_occ && x <= v_hi) ? 1u : 0u;
    }
  }
  h = wave_sum(h);
  m = wave_sum(m);
  if (lane == 0) {
    cnt_hi[b] = h;
    cnt_mid[b] = m;
  }
}

__device__ inline bool in_class(float x, int cls, float v_hi, float v_occ) {
  return cls == 0 ? x > v_hi : (x > v_occ && x <= v_hi);
}

struct SampleCfg {
  gve_grid g;
  int64_t M, nblocks;
  int S, n_hi, n_mid;
  uint64_t seed, it;
  float v_hi, v_occ;
};

// One wave per sample.  Points are stored as [2S][3]: sample s at row s, its
// smoothness partner at row S + s.
__global__ __launch_bounds__(kThreads) void k_psample(const float* __restrict__ f,
                                                      const uint32_t* __restrict__ off_hi,
                                                      const uint32_t* __restrict__ off_mid,
                                                      SampleCfg c, float* __restrict__ pts,
                                                      float* __restrict__ vals) {
  const int s = (int)(((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (s >= c.S) return;
  const uint64_t idx = c.it * (uint64_t)c.S + (uint64_t)s;
  const double u = uniform01(c.seed, kStreamPick, idx);
  int64_t vox;
  if (s < c.n_hi + c.n_mid) {
    const int cls = s < c.n_hi ? 0 : 1;
    const uint32_t* off = cls == 0 ? off_hi : off_mid;
    const uint64_t total = off[c.nblocks];
    uint64_t j = (uint64_t)floor(u * (double)total);
    if (j >= total) j = total - 1;
    // block b: the last with off[b] <= j
    int64_t lo = 0, hi = c.nblocks - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if ((uint64_t)off[mid] <= j) lo = mid; else hi = mid - 1;
    }
    const uint32_t r = (uint32_t)(j - off[lo]);
    // rank inside the block: lane L holds voxels 4L .. 4L+3 (ascending)
    uint32_t mine = 0;
    bool hit[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t v = lo * kBlockVox + 4 * lane + q;
      hit[q] = v < c.M && in_class(f[v], cls, c.v_hi, c.v_occ);
      mine += hit[q] ? 1u : 0u;
    }
    uint32_t incl = mine;  // inclusive prefix over lanes
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    const uint32_t excl = incl - mine;
    const bool owner = r >= excl && r < incl;
    int64_t found = 0;
    if (owner) {
      uint32_t k = r - excl;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (hit[q]) {
          if (k == 0) {
            found = lo * kBlockVox + 4 * lane + q;
            break;
          }
          --k;
        }
      }
    }
    const uint64_t ob = __builtin_amdgcn_ballot_w64(owner);
    const int src = ob ? __builtin_ffsll((long long)ob) - 1 : 0;
    vox = __shfl(found, src, 64);
  } else {
    vox = (int64_t)floor(u * (double)c.M);
    if (vox >= c.M) vox = c.M - 1;
  }
  if (lane == 0) {
    const int64_t ix = vox % c.g.nx, iy = (vox / c.g.nx) % c.g.ny, iz = vox / (c.g.nx * c.g.ny);
    const double base[3] = {(double)(c.g.x0 + ix), (double)(c.g.y0 + iy), (double)(c.g.z0 + iz)};
    double p[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      p[j] = base[j] + uniform01(c.seed, kStreamJit + j, idx) - 0.5;
      pts[3 * s + j] = (float)p[j];
      pts[3 * ((int64_t)c.S + s) + j] =
          (float)(p[j] + uniform01(c.seed, kStreamPartner + j, idx) - 0.5);
    }
    vals[s] = (float)trilinear(f, c.g, p[0], p[1], p[2]);
  }
}

__global__ __launch_bounds__(kThreads) void k_pcell_keys(const float* __restrict__ pts, int64_t np,
                                                         CellGrid cg, uint32_t* __restrict__ keys,
                                                         uint32_t* __restrict__ idx) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= np) return;
  const int cx = cell_coord(pts[3 * j + 0], cg.x0, cg.h, cg.ncx);
  const int cy = cell_coord(pts[3 * j + 1], cg.y0, cg.h, cg.ncy);
  const int cz = cell_coord(pts[3 * j + 2], cg.z0, cg.h, cg.ncz);
  keys[j] = (uint32_t)(cx + cg.ncx * (cy + cg.ncy * cz));
  idx[j] = (uint32_t)j;
}

// ---- forward / backward over the cells a primitive's box overlaps -------------------

struct PairCfg {
  CellGrid cg;
  float k2;
  int64_t S;  // points [0, S) are samples (get the numerator), [S, np) partners
};

template <typename F>
__device__ inline void for_points(const PGeom& g, const PairCfg& c, const float* __restrict__ pts,
                                  const uint32_t* __restrict__ sorted,
                                  const uint32_t* __restrict__ start, F&& fn) {
  const int x0 = cell_coord(g.mu[0] - g.half[0], c.cg.x0, c.cg.h, c.cg.ncx);
  const int x1 = cell_coord(g.mu[0] + g.half[0], c.cg.x0, c.cg.h, c.cg.ncx);
  const int y0 = cell_coord(g.mu[1] - g.half[1], c.cg.y0, c.cg.h, c.cg.ncy);
  const int y1 = cell_coord(g.mu[1] + g.half[1], c.cg.y0, c.cg.h, c.cg.ncy);
  const int z0 = cell_coord(g.mu[2] - g.half[2], c.cg.z0, c.cg.h, c.cg.ncz);
  const int z1 = cell_coord(g.mu[2] + g.half[2], c.cg.z0, c.cg.h, c.cg.ncz);
  for (int cz = z0; cz <= z1; ++cz)
    for (int cy = y0; cy <= y1; ++cy)
      for (int cx = x0; cx <= x1; ++cx) {
        const uint32_t cell = (uint32_t)(cx + c.cg.ncx * (cy + c.cg.ncy * cz));
        const uint32_t e = start[cell + 1];
        for (uint32_t j = start[cell]; j < e; ++j) {
          const uint32_t pi = sorted[j];
          const float dx = pts[3 * pi + 0] - g.mu[0];
          const float dy = pts[3 * pi + 1] - g.mu[1];
          const float dz = pts[3 * pi + 2] - g.mu[2];
          const float m2 = mahal2(g, dx, dy, dz);
          if (m2 < c.k2) fn(pi, dx, dy, dz, expf(-0.5f * m2));
        }
      }
}

__global__ __launch_bounds__(kThreads) void k_pfwd(const float* __restrict__ th, int64_t n,
                                                   PairCfg c, float k,
                                                   const float* __restrict__ pts,
                                                   const uint32_t* __restrict__ sorted,
                                                   const uint32_t* __restrict__ start,
                                                   double* __restrict__ num,
                                                   double* __restrict__ den) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const PGeom g = pgeom(th, n, i, k);
  for_points(g, c, pts, sorted, start, [&](uint32_t pi, float, float, float, float G) {
    const float wg = g.w * G;
    atomicAdd(&den[pi], (double)wg);
    if ((int64_t)pi < c.S) atomicAdd(&num[pi], (double)(wg * g.a));
  });
}

struct CoefCfg {
  int64_t S;
  double rho0, lam_rho, lam_sm, v_occ;
};

// coefA: coefficient of d(w a G) (samples only); coefB: of d(w G).
// loss[0..2] += L_val, L_rho, L_sm.
__global__ __launch_bounds__(kThreads) void k_pcoef(CoefCfg c, const double* __restrict__ num,
                                                    const double* __restrict__ den,
                                                    const float* __restrict__ vals,
                                                    float* __restrict__ coefA,
                                                    float* __restrict__ coefB,
                                                    double* __restrict__ loss,
                                                    float* __restrict__ vt_out) {
  const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double lv = 0.0, lr = 0.0, ls = 0.0;
  if (s < c.S) {
    const double d1 = den[s], d2 = den[c.S + s];
    const double D = fmax(d1, c.rho0);
    const double vt = num[s] / D;
    const double val = (double)vals[s];
    const bool occ = val > c.v_occ;
    const double u = occ ? 2.0 * (vt - val) : 0.0;
    const double v = (occ ? 2.0 * c.lam_rho * (d1 - 1.0) : 0.0) + 2.0 * c.lam_sm * (d1 - d2);
    coefA[s] = (float)(u / D);
    coefB[s] = (float)(v - (d1 > c.rho0 ? u * vt / D : 0.0));
    coefA[c.S + s] = 0.0f;
    coefB[c.S + s] = (float)(-2.0 * c.lam_sm * (d1 - d2));
    if (occ) {
      lv = (vt - val) * (vt - val);
      lr = (d1 - 1.0) * (d1 - 1.0);
    }
    ls = (d1 - d2) * (d1 - d2);
    if (vt_out) vt_out[s] = (float)vt;
  }
  block_add3(lv, lr, ls, loss);
}

struct BwdCfg {
  float k, lam_anc, lam_aniso, lam_cap, log_aniso, ell_lo, ell_hi;
  float lr, b1, b2, eps, inv_bc1, inv_bc2;
  int mode;  // 0: write the gradient; 1: Adam step
};

__global__ __launch_bounds__(kThreads) void k_pbwd(float* __restrict__ th, float* __restrict__ m,
                                                   float* __restrict__ v, int64_t n, PairCfg c,
                                                   BwdCfg b, const float* __restrict__ pts,
                                                   const uint32_t* __restrict__ sorted,
                                                   const uint32_t* __restrict__ start,
                                                   const float* __restrict__ coefA,
                                                   const float* __restrict__ coefB,
                                                   const float* __restrict__ field, gve_grid fg,
                                                   float* __restrict__ grad_out,
                                                   double* __restrict__ loss) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double la = 0.0, lan = 0.0, lc = 0.0;
  if (i < n) {
    const PGeom g = pgeom(th, n, i, b.k);
    float sgd[3] = {0.f, 0.f, 0.f}, D[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float dA = 0.f, dB = 0.f;
    for_points(g, c, pts, sorted, start, [&](uint32_t pi, float dx, float dy, float dz, float G) {
      const float cA = coefA[pi], cB = coefB[pi];
      const float e = fmaf(cA, g.a, cB);  // coefficient of d(w G)
      const float gc = e * g.w * G;
      sgd[0] = fmaf(gc, dx, sgd[0]);
      sgd[1] = fmaf(gc, dy, sgd[1]);
      sgd[2] = fmaf(gc, dz, sgd[2]);
      D[0] = fmaf(gc * dx, dx, D[0]);
      D[1] = fmaf(gc * dx, dy, D[1]);
      D[2] = fmaf(gc * dx, dz, D[2]);
      D[3] = fmaf(gc * dy, dy, D[3]);
      D[4] = fmaf(gc * dy, dz, D[4]);
      D[5] = fmaf(gc * dz, dz, D[5]);
      dA = fmaf(cA * g.w, G, dA);
      dB = fmaf(e, G, dB);
    });
    float t[12], gr[12];
#pragma unroll
    for (int a = 0; a < 12; ++a) t[a] = th[a * n + i];
    geometry_grad(&t[3], &t[7], sgd, D, gr);
    gr[10] = dA;
    gr[11] = dB * g.w * (1.0f - g.w);
    // regularisers
    const double aref = trilinear(field, fg, (double)t[0], (double)t[1], (double)t[2]);
    const double da = (double)t[10] - aref;
    gr[10] += (float)(2.0 * b.lam_anc * da);
    la = da * da;
    int jmax = 0, jmin = 0;
#pragma unroll
    for (int j = 1; j < 3; ++j) {
      if (t[7 + j] > t[7 + jmax]) jmax = j;
      if (t[7 + j] < t[7 + jmin]) jmin = j;
    }
    const float spread = t[7 + jmax] - t[7 + jmin] - b.log_aniso;
    if (spread > 0.f) {
      gr[7 + jmax] += 2.f * b.lam_aniso * spread;
      gr[7 + jmin] -= 2.f * b.lam_aniso * spread;
      lan = (double)spread * spread;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float l = t[7 + j];
      if (l > b.ell_hi) {
        gr[7 + j] += 2.f * b.lam_cap * (l - b.ell_hi);
        lc += (double)(l - b.ell_hi) * (l - b.ell_hi);
      }
      if (l < b.ell_lo) {
        gr[7 + j] -= 2.f * b.lam_cap * (b.ell_lo - l);
        lc += (double)(b.ell_lo - l) * (b.ell_lo - l);
      }
    }
    if (b.mode == 0) {
#pragma unroll
      for (int a = 0; a < 12; ++a) grad_out[a * n + i] = gr[a];
    } else {
#pragma unroll
      for (int a = 0; a < 12; ++a) {
        float mm = m[a * n + i], vv = v[a * n + i];
        mm = b.b1 * mm + (1.0f - b.b1) * gr[a];
        vv = b.b2 * vv + (1.0f - b.b2) * gr[a] * gr[a];
        m[a * n + i] = mm;
        v[a * n + i] = vv;
        th[a * n + i] = t[a] - b.lr * (mm * b.inv_bc1) / (sqrtf(vv * b.inv_bc2) + b.eps);
      }
    }
  }
  block_add3(la, lan, lc, loss);
}

__global__ __launch_bounds__(kThreads) void k_pfill_d(double* __restrict__ p, int64_t n) {
  for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * kThreads)
    p[j] = 0.0;
}

__global__ __launch_bounds__(kThreads) void k_pdensity(const double* __restrict__ num,
                                                       const double* __restrict__ den,
                                                       int64_t np, float rho0,
                                                       float* __restrict__ vt,
                                                       float* __restrict__ dn) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= np) return;
  const double d = den[j];
  if (vt) vt[j] = (float)(num[j] / fmax(d, (double)rho0));
  if (dn) dn[j] = (float)d;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

CellGrid make_cells(const gve_grid& g, float h) {
  CellGrid cg;
  cg.x0 = (float)g.x0 - 0.5f;
  cg.y0 = (float)g.y0 - 0.5f;
  cg.z0 = (float)g.z0 - 0.5f;
  cg.h = h;
  cg.ncx = (int)std::max<int64_t>(1, (int64_t)std::ceil((double)g.nx / h));
  cg.ncy = (int)std::max<int64_t>(1, (int64_t)std::ceil((double)g.ny / h));
  cg.ncz = (int)std::max<int64_t>(1, (int64_t)std::ceil((double)g.nz / h));
  return cg;
}

int64_t paper_class_blocks(int64_t M) { return (M + kBlockVox - 1) / kBlockVox; }

hipError_t paper_class_counts(const float* f, int64_t M, float v_hi, float v_occ, uint32_t* cnt_hi,
                              uint32_t* cnt_mid, hipStream_t s) {
  const int64_t nb = paper_class_blocks(M);
  hipLaunchKernelGGL(k_pclass_count, dim3(blocks_for(nb * 64)), dim3(kThreads), 0, s, f, M, v_hi,
                     v_occ, cnt_hi, cnt_mid, nb);
  return hipGetLastError();
}

hipError_t paper_sample(const float* f, const gve_grid& g, const uint32_t* off_hi,
                        const uint32_t* off_mid, int S, int n_hi, int n_mid, uint64_t seed,
                        uint64_t it, float v_hi, float v_occ, float* pts, float* vals,
                        hipStream_t s) {
  SampleCfg c;
  c.g = g;
  c.M = g.nx * g.ny * g.nz;
  c.nblocks = paper_class_blocks(c.M);
  c.S = S;
  c.n_hi = n_hi;
  c.n_mid = n_mid;
  c.seed = seed;
  c.it = it;
  c.v_hi = v_hi;
  c.v_occ = v_occ;
  hipLaunchKernelGGL(k_psample, dim3(blocks_for((int64_t)S * 64)), dim3(kThreads), 0, s, f, off_hi,
                     off_mid, c, pts, vals);
  return hipGetLastError();
}

hipError_t paper_cell_keys(const float* pts, int64_t np, const CellGrid& cg, uint32_t* keys,
                           uint32_t* idx, hipStream_t s) {
  hipLaunchKernelGGL(k_pcell_keys, dim3(blocks_for(np)), dim3(kThreads), 0, s, pts, np, cg, keys,
                     idx);
  return hipGetLastError();
}

hipError_t paper_zero(double* p, int64_t n, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n + kThreads - 1) / kThreads, 4096);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pfill_d, dim3((unsigned)blocks), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

hipError_t paper_forward(const float* th, int64_t n, const CellGrid& cg, float k, int64_t S,
                         const float* pts, const uint32_t* sorted, const uint32_t* start,
                         double* num, double* den, hipStream_t s) {
  PairCfg c;
  c.cg = cg;
  c.k2 = k * k;
  c.S = S;
  hipLaunchKernelGGL(k_pfwd, dim3(blocks_for(n)), dim3(kThreads), 0, s, th, n, c, k, pts, sorted,
                     start, num, den);
  return hipGetLastError();
}

hipError_t paper_density(const double* num, const double* den, int64_t np, float rho0, float* vt,
                         float* dn, hipStream_t s) {
  hipLaunchKernelGGL(k_pdensity, dim3(blocks_for(np)), dim3(kThreads), 0, s, num, den, np, rho0, vt,
                     dn);
  return hipGetLastError();
}

hipError_t paper_coef(int64_t S, const gve_paper_options& o, float lam_sm, const double* num,
                      const double* den, const float* vals, float* coefA, float* coefB,
                      double* loss, hipStream_t s) {
  CoefCfg c;
  c.S = S;
  c.rho0 = o.rho0;
  c.lam_rho = o.lam_rho;
  c.lam_sm = lam_sm;
  c.v_occ = o.v_occ;
  hipLaunchKernelGGL(k_pcoef, dim3(blocks_for(S)), dim3(kThreads), 0, s, c, num, den, vals, coefA,
                     coefB, loss, (float*)nullptr);
  return hipGetLastError();
}

hipError_t paper_backward(float* th, float* m, float* v, int64_t n, const CellGrid& cg,
                          const gve_paper_options& o, int mode, int64_t t, int64_t S,
                          const float* pts, const uint32_t* sorted, const uint32_t* start,
                          const float* coefA, const float* coefB, const float* field,
                          const gve_grid& fg, float* grad_out, double* loss, hipStream_t s) {
  PairCfg c;
  c.cg = cg;
  c.k2 = o.k * o.k;
  c.S = S;
  BwdCfg b;
  b.k = o.k;
  b.lam_anc = o.lam_anc;
  b.lam_aniso = o.lam_aniso;
  b.lam_cap = o.lam_cap;
  b.log_aniso = logf(o.aniso_max);
  b.ell_lo = o.ell_lo;
  b.ell_hi = o.ell_hi;
  b.lr = o.lr;
  b.b1 = o.beta1;
  b.b2 = o.beta2;
  b.eps = o.eps;
  const double tt = (double)(t > 0 ? t : 1);
  b.inv_bc1 = (float)(1.0 / (1.0 - std::pow((double)o.beta1, tt)));
  b.inv_bc2 = (float)(1.0 / (1.0 - std::pow((double)o.beta2, tt)));
  b.mode = mode;
  hipLaunchKernelGGL(k_pbwd, dim3(blocks_for(n)), dim3(kThreads), 0, s, th, m, v, n, c, b, pts,
                     sorted, start, coefA, coefB, field, fg, grad_out, loss);
  return hipGetLastError();
}

}  // namespace gve
