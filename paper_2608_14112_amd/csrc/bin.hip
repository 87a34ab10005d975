// Truncation-aware binning of primitives to voxel bricks (paper Sec. III-G:
// only pairs inside the k-sigma support contribute, so each primitive is
// visited only from the bricks its support can reach).
//
//   prep   : per primitive, normalised quaternion -> R, scales, the column
//            form of A = -(log2 e / 2) R S^-2 R^T (see Record), the k-sigma
//            bounding box
//            (|d_j| < k sqrt(Sigma_jj) bounds the ellipsoid m^2 < k^2) clipped
//            to the grid, and the number of bricks that box touches;
//   cull   : per primitive, the bricks of its box that a separating plane
//            does not part from its support, their keys and their count
//            (which replaces the box's brick count);
//   emit   : the (brick, primitive) pairs at the scanned offsets;
//   ranges : first pair of every brick in the brick-sorted list (binary search).
#include "common.h"

namespace gve {
namespace {

constexpr int kThreads = 256;

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Volume of primitive i: the last item whose first primitive is <= i.
__device__ inline int item_of_prim(const ItemDesc* __restrict__ items, int nitems, uint32_t i) {
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].prim0 <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline uint32_t prep_one(const float* __restrict__ theta, int64_t n, int64_t i,
                                    const ItemDesc& g, float k, BrickGeom bg,
                                    Record* __restrict__ rec, BoxXY* __restrict__ box,
                                    bool& degenerate) {
  const float mx = theta[0 * n + i], my = theta[1 * n + i], mz = theta[2 * n + i];
  float qw = theta[3 * n + i], qx = theta[4 * n + i], qy = theta[5 * n + i],
        qz = theta[6 * n + i];
  const float lx = theta[7 * n + i], ly = theta[8 * n + i], lz = theta[9 * n + i];
  const float c = theta[10 * n + i];
  const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  degenerate = !(qn >= 1e-12f);
  if (!degenerate) {
    const float inv = 1.0f / qn;
    qw *= inv; qx *= inv; qy *= inv; qz *= inv;
  } else {
    qw = 1.f; qx = qy = qz = 0.f;
  }
  const float r00 = 1.f - 2.f * (qy * qy + qz * qz), r01 = 2.f * (qx * qy - qw * qz),
              r02 = 2.f * (qx * qz + qw * qy);
  const float r10 = 2.f * (qx * qy + qw * qz), r11 = 1.f - 2.f * (qx * qx + qz * qz),
              r12 = 2.f * (qy * qz - qw * qx);
  const float r20 = 2.f * (qx * qz - qw * qy), r21 = 2.f * (qy * qz + qw * qx),
              r22 = 1.f - 2.f * (qx * qx + qy * qy);
  const float i0 = expf(-2.f * lx), i1 = expf(-2.f * ly), i2 = expf(-2.f * lz);
  const float s0 = expf(2.f * lx), s1 = expf(2.f * ly), s2 = expf(2.f * lz);
  // z row of the precision P = R diag(i) R^T
  const float pxz = r00 * r20 * i0 + r01 * r21 * i1 + r02 * r22 * i2;
  const float pyz = r10 * r20 * i0 + r11 * r21 * i1 + r12 * r22 * i2;
  const float pzz = r20 * r20 * i0 + r21 * r21 * i1 + r22 * r22 * i2;
  // diagonal of Sigma = R diag(s^2) R^T
  const float sxx = r00 * r00 * s0 + r01 * r01 * s1 + r02 * r02 * s2;
  const float syy = r10 * r10 * s0 + r11 * r11 * s1 + r12 * r12 * s2;
  const float szz = r20 * r20 * s0 + r21 * r21 * s1 + r22 * r22 * s2;

  // xy block of Sigma and its inverse.  det(Sigma_xy) = det(Sigma) P_zz
  // (Cauchy-Binet; the 2x2 minors of R's first two rows are its third row),
  // a sum of positive terms, so 1 / det needs no cancelling subtraction.
  const float sxy = r00 * r10 * s0 + r01 * r11 * s1 + r02 * r12 * s2;
  const float idet = (i0 * i1 * i2) / pzz;

  Record r;
  r.mu[0] = mx; r.mu[1] = my; r.mu[2] = mz;
  r.c = c;
  r.sz = sqrtf(kHalfLog2e * pzz);
  r.s[0] = -kHalfLog2e * syy * idet;
  r.s[1] = 2.0f * kHalfLog2e * sxy * idet;
  r.s[2] = -kHalfLog2e * sxx * idet;
  r.gx = -pxz / pzz;
  r.gy = -pyz / pzz;
  r.sgx = r.sz * r.gx;
  r.sgy = r.sz * r.gy;
  r.cz = __builtin_amdgcn_exp2f(-2.0f * r.sz * r.sz);
  r.spare = 0.0f;

  // conservative box: relative and absolute slack cover float32 rounding here
  const float mu3[3] = {mx, my, mz};
  const float sd[3] = {sxx, syy, szz};
  const int64_t org[3] = {g.x0, g.y0, g.z0};
  const int64_t dim[3] = {g.nx, g.ny, g.nz};
  bool empty = false;
  int lo[3], hi[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float h = k * sqrtf(sd[j]) * (1.0f + 1e-5f) + 1e-3f;
    const float a = mu3[j] - (float)org[j] - h;
    const float b = mu3[j] - (float)org[j] + h;
    if (!(a == a) || !(b == b) || !(h == h)) {  // NaN
      empty = true;
      lo[j] = 0; hi[j] = -1;
      continue;
    }
    const float fd = (float)dim[j];
    const float ac = fminf(fmaxf(ceilf(a), -1.0f), fd);
    const float bc = fminf(fmaxf(floorf(b), -1.0f), fd);
    lo[j] = clampi((int)ac, 0, (int)dim[j] - 1);
    hi[j] = clampi((int)bc, 0, (int)dim[j] - 1);
    if (ac > bc || bc < 0.f || ac > fd - 1.f) empty = true;
  }
  uint32_t cnt = 0;
  if (!empty) {
    // brick edges are powers of two; lo, hi >= 0
    const int sxy = __builtin_ctz(bg.Bxy), sz = __builtin_ctz(bg.Bz);
    cnt = (uint32_t)((hi[0] >> sxy) - (lo[0] >> sxy) + 1) *
          (uint32_t)((hi[1] >> sxy) - (lo[1] >> sxy) + 1) *
          (uint32_t)((hi[2] >> sz) - (lo[2] >> sz) + 1);
  } else {
#pragma unroll
    for (int j = 0; j < 3; ++j) { lo[j] = 1; hi[j] = 0; }
  }
  r.zlo = lo[2];
  r.zhi = hi[2];
  rec[i] = r;
  BoxXY b;
  b.lo[0] = lo[0]; b.lo[1] = lo[1];
  b.hi[0] = hi[0]; b.hi[1] = hi[1];
  box[i] = b;
  return cnt;
}

__global__ __launch_bounds__(kThreads) void k_prep(const float* __restrict__ theta, int64_t n,
                                                   const ItemDesc* __restrict__ items, int nitems,
                                                   float k, BrickGeom bg,
                                                   Record* __restrict__ rec,
                                                   uint32_t* __restrict__ count,
                                                   unsigned long long* __restrict__ total) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  uint32_t cnt = 0;
  bool degenerate = false;
  if (i < n)
    cnt = prep_one(theta, n, i, items[item_of_prim(items, nitems, (uint32_t)i)], k, bg, rec,
                   record_boxes(rec, n), degenerate);
  if (i < n) count[i] = cnt;
  // degenerate quaternions (rare): one atomic per wave that has any
  const uint64_t deg = __builtin_amdgcn_ballot_w64(degenerate);
  if (deg != 0ull && (threadIdx.x & 63) == 0)
    atomicAdd(&total[kTotalSlots], (unsigned long long)__popcll(deg));
  // 64-bit pair total (the scan itself is 32-bit): one atomic per block, into
  // one of kTotalSlots counters
  __shared__ unsigned long long wsum[kThreads / 64];
  unsigned long long w = cnt;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) w += __shfl_xor(w, d, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
#pragma unroll
    for (int v = 0; v < kThreads / 64; ++v) t += wsum[v];
    if (t) atomicAdd(&total[blockIdx.x % kTotalSlots], t);
  }
}

// ---- culling of bricks that miss the support -----------------------------
//
// A brick that meets a primitive's k-sigma box can still miss its ellipsoid
// m^2 < k^2 (the corners of a rotated ellipsoid's box).  Let C be the brick's
// part of the box (voxel centres), c its centre, h its half extents,
// d = c - mu and n = P d, the ellipsoid's normal direction at c.  Along n the
// ellipsoid m <= K reaches at most n.mu + K sqrt(n^T Sigma n) = n.mu + K sqrt(d^T P d),
// and C reaches down to n.c - sum_j |n_j| h_j, so the plane normal to n parts
// them when
//     d^T P d - sum_j |n_j| h_j > K sqrt(d^T P d).
// With K = k (1 + 1e-3) every voxel of C then has m^2 > 1.002 k^2, well
// clear of where float32 rounding could decide the cut either way, and a
// relative allowance of 1e-5 covers the rounding of the test itself.  In the
// record's scaled units (Q = -(log2 e / 2) m^2, the xy part qxy = s0 dx^2 +
// s1 dx dy + s2 dy^2, the z part -(sz t)^2 with t = dz - gx dx - gy dy) the
// scaled normal (log2 e / 2) P d is
//     (-(s0 dx + s1 dy / 2) - sz^2 t gx, -(s1 dx / 2 + s2 dy) - sz^2 t gy, sz^2 t)
// and (log2 e / 2) d^T P d = sz^2 t^2 - qxy.  The test is conservative: a brick
// it keeps may still miss (the brick kernels test every column anyway).
// (ox, oy, oz): the volume's origin minus the primitive's centre (float).
__device__ inline bool brick_meets_support(const Record& r, const BoxXY& box, float ox, float oy,
                                           float oz, BrickGeom bg, uint32_t bx, uint32_t by,
                                           uint32_t bz, float k) {
  const int bxy = bg.Bxy, bzz = bg.Bz;
  const int sxy = __builtin_ctz(bxy), sz = __builtin_ctz(bzz);  // edges are powers of two
  const int xa = max((int)(bx << sxy), box.lo[0]), xb = min((int)(bx << sxy) + bxy - 1, box.hi[0]);
  const int ya = max((int)(by << sxy), box.lo[1]), yb = min((int)(by << sxy) + bxy - 1, box.hi[1]);
  const int za = max((int)(bz << sz), r.zlo), zb = min((int)(bz << sz) + bzz - 1, r.zhi);
  const float dx = 0.5f * (float)(xa + xb) + ox;
  const float dy = 0.5f * (float)(ya + yb) + oy;
  const float dz = 0.5f * (float)(za + zb) + oz;
  const float hx = 0.5f * (float)(xb - xa), hy = 0.5f * (float)(yb - ya),
              hz = 0.5f * (float)(zb - za);
  const float t = dz - (r.gx * dx + r.gy * dy);
  const float sz2 = r.sz * r.sz;
  const float qxy = (r.s[0] * dx + r.s[1] * dy) * dx + r.s[2] * dy * dy;
  const float nx = -(r.s[0] * dx + 0.5f * r.s[1] * dy) - sz2 * t * r.gx;
  const float ny = -(0.5f * r.s[1] * dx + r.s[2] * dy) - sz2 * t * r.gy;
  const float nz = sz2 * t;
  const float mm = sz2 * t * t - qxy;
  const float side = fabsf(nx) * hx + fabsf(ny) * hy + fabsf(nz) * hz;
  // the hardware square root (within 1 ulp) is ample against the 1e-3 margin
  const float reach = (1.0f + 1e-3f) * k * sqrtf(kHalfLog2e) * __builtin_amdgcn_sqrtf(mm);
  // NaN anywhere keeps the brick
  return !(mm - side > reach + 1e-5f * (mm + side));
}

// j / d for j < 2^21 through a float reciprocal: (j + 1/2) / d lies at least
// 1/(2d) from every integer, and a reciprocal within 1 ulp times a rounded
// product moves it by less than (j + 1/2) / d * 1.5 * 2^-23 < 1/(2d), so the
// truncation is exact.
__device__ inline uint32_t div_small(uint32_t j, float inv_d) {
  return (uint32_t)(((float)j + 0.5f) * inv_d);
}

// Bricks of primitive i's box, in (z, y, x) order.
struct BoxBricks {
  uint32_t bx0, by0, bz0, nbx, nby;
  float inv_nbx, inv_nby;
  __device__ void at(uint32_t j, uint32_t& bx, uint32_t& by, uint32_t& bz) const {
    uint32_t t, u;
    if (j < (1u << 21)) {
      t = div_small(j, inv_nbx);
      u = div_small(t, inv_nby);
    } else {
      t = j / nbx;
      u = t / nby;
    }
    bx = bx0 + (j - t * nbx);
    by = by0 + (t - u * nby);
    bz = bz0 + u;
  }
};

__device__ inline BoxBricks box_bricks(const Record& r, const BoxXY& box, BrickGeom bg) {
  BoxBricks b;
  // brick edges are powers of two; box corners are >= 0
  const uint32_t sxy = (uint32_t)__builtin_ctz(bg.Bxy), sz = (uint32_t)__builtin_ctz(bg.Bz);
  b.bx0 = (uint32_t)box.lo[0] >> sxy;
  b.by0 = (uint32_t)box.lo[1] >> sxy;
  b.bz0 = (uint32_t)r.zlo >> sz;
  b.nbx = ((uint32_t)box.hi[0] >> sxy) - b.bx0 + 1;
  b.nby = ((uint32_t)box.hi[1] >> sxy) - b.by0 + 1;
  b.inv_nbx = 1.0f / (float)b.nbx;
  b.inv_nby = 1.0f / (float)b.nby;
  return b;
}

// Sixteen lanes per primitive (four primitives per wave, so that launching
// and loading cost less than the work) over the bricks of its box (box_off:
// scan of prep's box brick counts).  Keeps the bricks brick_meets_support
// does not reject, in box order, compacted by ballot within the lane group:
// their keys go to kept[box_off[i] ..] and their number to count[i].
constexpr int kGroup = 16;

__global__ __launch_bounds__(kThreads) void k_cull(const Record* __restrict__ rec, int64_t n,
                                                   const uint32_t* __restrict__ box_off,
                                                   const ItemDesc* __restrict__ items, int nitems,
                                                   BrickGeom bg, float k,
                                                   const uint32_t* __restrict__ fits,
                                                   uint32_t* __restrict__ kept,
                                                   uint32_t* __restrict__ count) {
  const int64_t i = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / kGroup;
  const int lane = threadIdx.x & 63;
  const int sub = lane & (kGroup - 1);
  const int shift = lane & ~(kGroup - 1);  // first lane of the group
  const bool live = i < n;
  // buffers sized in advance: when the box pairs do not fit, nothing is kept
  const bool room = fits == nullptr || *fits != 0u;
  uint32_t o = 0, total = 0;
  Record r{};
  BoxXY box{};
  if (live && room) {
    // the offsets, the record and the box loaded together, one wait for all
    // (pinning them here keeps their loads from following the offsets'
    // latency)
    o = box_off[i];
    total = box_off[i + 1] - o;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4* src = reinterpret_cast<const u32x4*>(rec + i);
    u32x4 q[5];
#pragma unroll
    for (int h = 0; h < 4; ++h) q[h] = src[h];
    q[4] = *reinterpret_cast<const u32x4*>(record_boxes(rec, n) + i);
    asm volatile("" ::"v"(q[0]), "v"(q[1]), "v"(q[2]), "v"(q[3]), "v"(q[4]));
    __builtin_memcpy(&r, q, sizeof(Record));
    __builtin_memcpy(&box, &q[4], sizeof(BoxXY));
  }
  if (live && !room && sub == 0) count[i] = 0;
  BoxBricks bb{};
  // the volume's descriptor, read once: origin relative to the centre, and
  // what the brick keys need
  float ox = 0.f, oy = 0.f, oz = 0.f;
  uint32_t kb0 = 0, knbx = 0, knby = 0;
  if (total > 0) {
    bb = box_bricks(r, box, bg);
    const ItemDesc& it = items[item_of_prim(items, nitems, (uint32_t)i)];
    ox = (float)it.x0 - r.mu[0];
    oy = (float)it.y0 - r.mu[1];
    oz = (float)it.z0 - r.mu[2];
    kb0 = it.brick0;
    knbx = (uint32_t)it.nbx;
    knby = (uint32_t)it.nby;
  }
  const uint64_t below = ((1ull << lane) - 1ull) & ~((1ull << shift) - 1ull);
  uint32_t nkept = 0;
  // every lane of the wave takes part in each ballot; a group idles once its
  // box is done
  for (uint32_t base = 0; __builtin_amdgcn_ballot_w64(base < total) != 0ull; base += kGroup) {
    const uint32_t j = base + (uint32_t)sub;
    bool keep = false;
    uint32_t bx = 0, by = 0, bz = 0;
    if (j < total) {
      bb.at(j, bx, by, bz);
      keep = brick_meets_support(r, box, ox, oy, oz, bg, bx, by, bz, k);
    }
    const uint64_t m = __builtin_amdgcn_ballot_w64(keep);
    // brick key: the global brick id (x fastest within the volume)
    if (keep) kept[o + nkept + (uint32_t)__popcll(m & below)] = kb0 + knbx * (by + knby * bz) + bx;
    nkept += (uint32_t)__popcll((m >> shift) & ((1ull << kGroup) - 1ull));
  }
  if (live && total > 0 && sub == 0) count[i] = nkept;
}

// Pairs at the scanned offsets from the keys k_cull kept: sixteen lanes per
// primitive.  The value of a pair is its primitive id, or, with `owner`
// (deterministic gradient sums), its emission index p, with owner[p] = the
// primitive id: the sorted emission indices then name each pair's own
// partials slot (a primitive's slots are its contiguous emission range).
__global__ __launch_bounds__(kThreads) void k_emit_kept(const uint32_t* __restrict__ offset,
                                                        int64_t n,
                                                        const uint32_t* __restrict__ box_off,
                                                        const uint32_t* __restrict__ kept,
                                                        uint32_t* __restrict__ keys,
                                                        uint32_t* __restrict__ vals,
                                                        uint32_t* __restrict__ owner,
                                                        const uint32_t* __restrict__ fits) {
  const int64_t i = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / kGroup;
  const uint32_t sub = threadIdx.x & (kGroup - 1);
  if (i >= n || (fits && *fits == 0u)) return;
  // the three loads waited for together (pinning src here keeps its load
  // from moving into the loop below, behind the offsets' latency)
  const uint32_t o = offset[i], o1 = offset[i + 1];
  uint32_t src = box_off[i];
  asm volatile("" : "+v"(src));
  const uint32_t cnt = o1 - o;
  // four strides of the group at a time, loads issued before the stores
  constexpr int kUnroll = 4;
  for (uint32_t j0 = sub; j0 < cnt; j0 += kUnroll * kGroup) {
    uint32_t key[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint32_t j = j0 + u * kGroup;
      key[u] = j < cnt ? kept[src + j] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint32_t j = j0 + u * kGroup;
      if (j < cnt) {
        keys[o + j] = key[u];
        if (owner) {
          vals[o + j] = o + j;
          owner[o + j] = (uint32_t)i;
        } else {
          vals[o + j] = (uint32_t)i;
        }
      }
    }
  }
}

// gid[j] = owner[slot[j]]: the primitive of each sorted pair, from its
// emission index.
__global__ __launch_bounds__(kThreads) void k_gather_owner(const uint32_t* __restrict__ owner,
                                                           const uint32_t* __restrict__ slot,
                                                           int64_t n,
                                                           const uint32_t* __restrict__ dn,
                                                           uint32_t* __restrict__ gid) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (dn) n = min(n, (int64_t)*dn);
  if (j < n) gid[j] = owner[slot[j]];
}

// brick_start[b] = first index whose key >= b, for b in [0, nbricks].
__global__ __launch_bounds__(kThreads) void k_ranges(const uint32_t* __restrict__ keys,
                                                     int64_t npairs,
                                                     const uint32_t* __restrict__ dn,
                                                     int64_t nbricks,
                                                     uint32_t* __restrict__ start) {
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b > nbricks) return;
  if (dn) npairs = min(npairs, (int64_t)*dn);
  int64_t lo = 0, hi = npairs;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)keys[mid] < b) lo = mid + 1; else hi = mid;
  }
  start[b] = (uint32_t)lo;
}

// Sort keys of the heaviest-first order: fewer leading zeros in the pair
// count = more work, so an ascending stable sort puts heavy bricks first and
// keeps index order within a power-of-two class.
__global__ __launch_bounds__(kThreads) void k_order_keys(const uint32_t* __restrict__ start,
                                                         int64_t nbricks,
                                                         uint32_t* __restrict__ keys,
                                                         uint32_t* __restrict__ vals) {
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b >= nbricks) return;
  keys[b] = (uint32_t)__clz((int)(start[b + 1] - start[b]));
  vals[b] = (uint32_t)b;
}

// Whether the box pairs of this binning fit the buffers sized in advance:
// fits = (sum of prep's 64-bit pair-total slots <= capacity); a binning that
// does not fit also sets the sticky flag, which only the host clears, and
// need = the largest box total seen.
// With `count` (the kept pair total, from the scan of the kept counts)
// instead of slots, the same for the pair buffers; fits then stays 0 if the
// box pairs already did not fit, and a count that does not fit is set to 0,
// so that every later kernel of the binning sees no pair.
__global__ void k_fits(const unsigned long long* __restrict__ slots, int nslots,
                       uint32_t* __restrict__ count, unsigned long long capacity,
                       uint32_t* __restrict__ fits, uint32_t* __restrict__ sticky,
                       unsigned long long* __restrict__ need) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  unsigned long long t = 0;
  if (count) {
    t = *count;
  } else {
    for (int j = 0; j < nslots; ++j) t += slots[j];
  }
  const bool ok = t <= capacity && (count == nullptr || *fits != 0u);
  *fits = ok ? 1u : 0u;
  if (!ok) *sticky = 1u;
  if (!ok && count) *count = 0u;
  if (t > *need) *need = t;
}

}  // namespace

int64_t build_items(const gve_grid* grids, const int64_t* prim_off, int nitems, int Bxy, int Bz,
                    ItemDesc* out) {
  int64_t bricks = 0, vox = 0;
  for (int i = 0; i < nitems; ++i) {
    const gve_grid& g = grids[i];
    ItemDesc d{};
    d.nx = g.nx; d.ny = g.ny; d.nz = g.nz;
    d.x0 = g.x0; d.y0 = g.y0; d.z0 = g.z0;
    d.vox = vox;
    d.nbx = (int32_t)((g.nx + Bxy - 1) / Bxy);
    d.nby = (int32_t)((g.ny + Bxy - 1) / Bxy);
    d.nbz = (int32_t)((g.nz + Bz - 1) / Bz);
    d.brick0 = (uint32_t)bricks;
    d.prim0 = (uint32_t)prim_off[i];
    out[i] = d;
    bricks += (int64_t)d.nbx * d.nby * d.nbz;
    vox += g.nx * g.ny * g.nz;
  }
  return bricks;
}

hipError_t launch_prep(const float* theta, int64_t n, const ItemDesc* items, int nitems, float k,
                       BrickGeom bg, Record* rec, uint32_t* count, unsigned long long* total,
                       hipStream_t s) {
  const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(kThreads), 0, s, theta, n, items, nitems, k, bg,
                     rec, count, total);
  return hipGetLastError();
}

hipError_t launch_cull(const Record* rec, int64_t n, const uint32_t* box_off, const ItemDesc* items,
                       int nitems, BrickGeom bg, float k, uint32_t* kept, uint32_t* count,
                       hipStream_t s, const uint32_t* fits) {
  const unsigned blocks = (unsigned)((n * kGroup + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_cull, dim3(blocks), dim3(kThreads), 0, s, rec, n, box_off, items, nitems,
                     bg, k, fits, kept, count);
  return hipGetLastError();
}

hipError_t launch_fits(const unsigned long long* slots, uint32_t* count,
                       unsigned long long capacity, uint32_t* fits, uint32_t* sticky,
                       unsigned long long* need, hipStream_t s) {
  hipLaunchKernelGGL(k_fits, dim3(1), dim3(64), 0, s, slots, kTotalSlots, count, capacity, fits,
                     sticky, need);
  return hipGetLastError();
}

hipError_t launch_emit(const uint32_t* offset, int64_t n, const uint32_t* box_off,
                       const uint32_t* kept, uint32_t* keys, uint32_t* vals, uint32_t* owner,
                       hipStream_t s, const uint32_t* fits) {
  const unsigned blocks = (unsigned)((n * kGroup + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_emit_kept, dim3(blocks), dim3(kThreads), 0, s, offset, n, box_off, kept,
                     keys, vals, owner, fits);
  return hipGetLastError();
}

hipError_t launch_gather_owner(const uint32_t* owner, const uint32_t* slot, int64_t n,
                               uint32_t* gid, hipStream_t s, const uint32_t* dn) {
  if (n <= 0) return hipSuccess;  // no pairs: nothing to gather (an empty grid is invalid)
  const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_gather_owner, dim3(blocks), dim3(kThreads), 0, s, owner, slot, n, dn, gid);
  return hipGetLastError();
}

hipError_t launch_order_keys(const uint32_t* brick_start, int64_t nbricks, uint32_t* keys,
                             uint32_t* vals, hipStream_t s) {
  const unsigned blocks = (unsigned)((nbricks + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_order_keys, dim3(blocks), dim3(kThreads), 0, s, brick_start, nbricks, keys,
                     vals);
  return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* sorted_keys, int64_t npairs, int64_t nbricks,
                         uint32_t* brick_start, hipStream_t s, const uint32_t* dn) {
  const unsigned blocks = (unsigned)((nbricks + 1 + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_ranges, dim3(blocks), dim3(kThreads), 0, s, sorted_keys, npairs, dn,
                     nbricks, brick_start);
  return hipGetLastError();
}

}  // namespace gve
