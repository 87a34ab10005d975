// Per-brick field kernels.
//
// A workgroup owns one BXY x BXY x BZ brick; lane (lx, ly) owns the voxel
// column (x, y, z0 .. z0 + BZ - 1) and keeps its BZ values in registers.  The brick's
// primitives (a contiguous run of the brick-sorted pair list, increasing
// primitive index) are read one at a time with wave-uniform scalar loads.
//
// Along a column (fixed dx, dy) the exponent is a parabola in dz (see Record):
//     Q = qxy - w^2,  w = sz t,  t = dz - (gx dx + gy dy),
// with exp(-m^2/2) = exp2(Q), and the cut m^2 < k^2 (Sec. III-C) is
// Q > -(log2 e / 2) k^2.  w advances by sz per voxel and is formed afresh at
// every voxel as w0 + zz sz (one fused multiply-add), then Q = qxy - w w (a
// second one), so rounding does not accumulate along the column.  The loop
// runs over the primitive's bounding-box z-range inside the brick only.
//
//   k_forward : Vhat on the brick (Sec. III-C eq:field, truncated).
//   k_fused   : Vhat, residual r = 2 (Vhat - V), the brick's share of
//               L = sum (Vhat - V)^2, then for every primitive of the brick the
//               ten sums of the analytic gradient (e = r G, d = p - mu):
//               sum e, sum e d (3), sum e d d^T (6 unique; the weight c,
//               common to all bricks of a primitive, is applied once per
//               primitive by the update), reduced over the workgroup with
//               cross-lane permutes and LDS,
//               then either added to the primitive's accumulators with float
//               atomics, or (deterministic mode) stored to the pair's own slot
//               of a partials array that the update kernel sums per primitive
//               in a fixed order.  Per column only sum e, sum e zz and
//               sum e zz^2 over the brick offset zz are needed, because dx and
//               dy are constant along it and dz = (z0 - mu_z) + zz.
#include <algorithm>

#include "common.h"

namespace gve {
namespace {

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// ---- cross-lane reduction of ten values ------------------------------------------
//
// v_permlane32_swap exchanges the upper half-wave of one register with the
// lower half-wave of another, v_permlane16_swap the odd rows (16 lanes) of one
// with the even rows of another; with both operands the same value, the
// folds below leave every lane holding the sum over its lane and the lane 32
// (or 16) away.
__device__ inline float fold32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ inline float fold16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// The ten sums of a pair through LDS: the wave writes v[k] to row k of its
// own 10 x kSumStride block, then lane 16 p + k (k < 10) adds the sixteen
// values 16 p .. 16 p + 15 of row k (16-byte reads, eight at a time) and the
// two folds add the four parts p, leaving sum k in lane k (lanes 10 .. 15 of
// each row repeat row 9; their sums are of no use).  About twenty vector
// instructions in place of the thirty-odd lane permutes, row-wise DPP adds
// and selects of a register-only reduction, measured 0.9 ms faster per
// 1024^3 x 1.4M pass.  The block belongs to one wave, whose LDS operations
// complete in order, so no barrier separates the writes from the reads or the
// reads from the next pair's writes.  A row stride of 68 floats puts the
// 16-byte reads of lanes k = 0 .. 7 on distinct banks.
constexpr int kSumStride = 68;
constexpr int kSumFloats = 10 * kSumStride;

__device__ inline float lds_sum10(const float (&v)[10], float* __restrict__ buf, int lane) {
#pragma unroll
  for (int k = 0; k < 10; ++k) buf[k * kSumStride + lane] = v[k];
  const int k = min(lane & 15, 9);
  const float4* src = reinterpret_cast<const float4*>(buf + k * kSumStride + (lane & 48));
  const float4 a = src[0], b = src[1];
  float s = ((a.x + a.y) + (a.z + a.w)) + ((b.x + b.y) + (b.z + b.w));
  // the second half's reads are issued once the first half is summed, so
  // that at most eight read registers are live
  asm volatile("" : "+v"(s)::"memory");
  const float4 c = src[2], d = src[3];
  s += ((c.x + c.y) + (c.z + c.w)) + ((d.x + d.y) + (d.z + d.w));
  const float h = fold32(s, s);
  return fold16(h, h);
}

// ---- per (primitive, column) setup -------------------------------------------
//
// With t0 = (z0 - mu_z) - (gx dx + gy dy) the column coordinate at the
// brick's first z and wm = sz (t0 + BZ / 2) the scaled coordinate at its
// middle, Q at brick offset zz is qxy - w w with w = wm + (zz - BZ / 2) sz.
// Anchoring at the middle halves the largest |wm|, whose rounding sets the
// error of w.  Both terms of Q are <= 0, so the sum never cancels (an
// expansion in powers of zz about the brick's first voxel would, when the
// vertex is far from it).
struct ColumnSetup {
  float qxy, wm;  // vertex height, w at the brick's middle
  int za, zb;
  uint32_t zmask;  // bit zz set when brick offset zz lies in the z-range of the box
};

template <int BZ>
__device__ inline ColumnSetup column_setup(const Record& r, float px, float py, float pz0, int iz0) {
  ColumnSetup s;
  s.za = max(r.zlo - iz0, 0);
  s.zb = min(r.zhi - iz0, BZ - 1);
  // bits za..zb (BZ <= 32; 2u << 31 wraps to 0, giving all ones)
  s.zmask = (s.zb >= s.za) ? (((2u << s.zb) - 1u) & ~((1u << s.za) - 1u)) : 0u;
  const float dx = px - r.mu[0];
  const float dy = py - r.mu[1];
  s.qxy = fmaf(r.s[0], dx, r.s[1] * dy) * dx + r.s[2] * dy * dy;
  // w = sz t at the brick's middle: the brick offset from the centre first
  // (pz0 + BZ / 2 is exact and the same for every pair of the brick), then
  // the record's scaled slopes
  s.wm = fmaf(-r.sgy, dy, fmaf(-r.sgx, dx, r.sz * ((pz0 + (float)(BZ / 2)) - r.mu[2])));
  return s;
}

// w and Q at brick offset zz.  sz is passed in a vector register so that the
// per-step constant zz can take the instruction's one scalar operand slot
// (no literal operands in three-operand instructions on this target).
__device__ inline float vreg(float x) {
  float v;
  asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
  return v;
}

template <int BZ>
__device__ inline float w_at(const ColumnSetup& s, float szv, int zz) {
  return fmaf((float)(zz - BZ / 2), szv, s.wm);
}

__device__ inline float quad_w(const ColumnSetup& s, float w) { return fmaf(-w, w, s.qxy); }

__device__ inline Record load_record(const Record* __restrict__ rec, uint32_t gid) {
  return rec[gid];
}

// True if some step of the pair (brick offsets za .. zb) has Q > thr in some
// lane whose column lies inside the volume (cols = ballot of those lanes);
// otherwise the whole (primitive, brick) pair is skipped.  Along the column Q
// peaks at the vertex (w = 0): inside [za, zb] the largest Q is qxy, else Q at
// the nearer end, computed exactly as the steps compute it.
template <int BZ>
__device__ inline bool column_hit(const ColumnSetup& s, float sz, uint64_t cols, float thr) {
  if (s.zmask == 0u) return false;
  const float wa = fmaf((float)(s.za - BZ / 2), sz, s.wm);
  const float wb = fmaf((float)(s.zb - BZ / 2), sz, s.wm);
  // za <= zb and sz > 0 give wa <= wb, so the median of (wa, wb, 0) is 0
  // clamped to [wa, wb]: the w of the segment point nearest the vertex
  const float wn = __builtin_amdgcn_fmed3f(wa, wb, 0.0f);
  return (__builtin_amdgcn_ballot_w64(fmaf(-wn, wn, s.qxy) > thr) & cols) != 0ull;
}

// With `steps` (one-wave bricks), the brick offsets at which some lane of
// pair j - j0 < kStepCap was inside the support are stored as a bit mask
// (0: the pair misses the brick), so the backward pass visits only those.
// 512 entries (2 KB) and the 2.7 KB block of the ten-sum reduction keep a
// one-wave workgroup under 5 KB of LDS, so that 8 waves per SIMD stay
// resident (a 768-entry cap, 7 waves, measured 12 % slower).
constexpr uint32_t kStepCap = 512;

// Forward steps of one pair: w, Q and exp2 at every offset of the box's
// z-range (after the compare, offsets where no lane is inside the support are
// skipped).  Returns the mask of active offsets.  (The product form the
// backward pass uses, restarted exactly every eight offsets to hold the
// values' 1e-5, measured slower here: the extra uniform branches cost more
// than the exponentials they save.)
template <int BZ>
__device__ inline uint32_t forward_steps(const ColumnSetup& s, float szv, float c, float thr,
                                         float (&acc)[BZ]) {
  uint32_t active = 0u;
  // offsets in groups of eight: a group outside the box costs one taken
  // branch instead of eight (each taken branch stalls its wave; the groups
  // made the fused pass 2.7 % faster, groups of four or 16 + 4 less so)
#pragma unroll
  for (int g0 = 0; g0 < BZ; g0 += 8) {
    if ((s.zmask >> g0) & 0xFFu) {
#pragma unroll
      for (int zz = g0; zz < g0 + 8; ++zz) {
        if ((s.zmask >> zz) & 1u) {
          const float q = quad_w(s, w_at<BZ>(s, szv, zz));
          if (__builtin_amdgcn_ballot_w64(q > thr) != 0ull) {
            active |= 1u << zz;
            const float G = (q > thr) ? __builtin_amdgcn_exp2f(q) : 0.0f;
            acc[zz] = fmaf(c, G, acc[zz]);
          }
        }
      }
    }
  }
  return active;
}

// Record prefetch: every 64 pairs each lane touches (vector load) the record
// of one of those 64 pairs, so that the pairs' scalar record loads find the
// lines in L2.  The ids of a block of 64 pairs are loaded one block ahead and
// a touched value is consumed one block later, so the vector loads never
// hold the wave up; `sink` keeps them live.
struct Touch {
  uint32_t gid;  // this lane's pair id of the next block
  float held;    // the last touched value (consumed at the next block)
  float sink;
};

// A wave visits pairs j0, j0 + stride, j0 + 2 stride, ... (< j1); its k-th
// pair is j0 + stride k.
__device__ inline void touch_begin(const uint32_t* __restrict__ pair_gid, uint32_t j0,
                                   uint32_t stride, uint32_t j1, Touch& t) {
  t.gid = pair_gid[min(j0 + stride * (threadIdx.x & 63), j1 - 1)];
  t.held = 0.0f;
  t.sink = 0.0f;
}

// At the wave's k-th pair (k a multiple of 64).
__device__ inline void touch_block(const Record* __restrict__ rec,
                                   const uint32_t* __restrict__ pair_gid, uint32_t j0,
                                   uint32_t stride, uint32_t k, uint32_t j1, Touch& t) {
  t.sink += t.held;
  t.held = reinterpret_cast<const float*>(rec + t.gid)[0];
  t.gid = pair_gid[min(j0 + stride * (k + 64 + (threadIdx.x & 63)), j1 - 1)];
}

__device__ inline void touch_end(Touch& t) {
  t.sink += t.held;
  asm volatile("" ::"v"(t.sink));
}

// Forward accumulation of the wave's pairs of one brick: jw, jw + stride, ...
// (< j1; stride > 1 when several waves split a brick's pairs).  With
// `steps`, the active offsets of pair j go to steps[j - jb] (jb = the
// brick's first pair) for j - jb < kStepCap.
template <int BZ>
__device__ inline void accumulate_brick(const Record* __restrict__ rec,
                                        const uint32_t* __restrict__ pair_gid, uint32_t jb,
                                        uint32_t jw, uint32_t stride, uint32_t j1, float px,
                                        float py, float pz0, int iz0, uint64_t cols, float thr,
                                        float (&acc)[BZ], uint32_t* __restrict__ steps) {
  Touch tc;
  if (jw < j1) touch_begin(pair_gid, jw, stride, j1, tc);
  uint32_t k = 0;
  for (uint32_t j = jw; j < j1; j += stride, ++k) {
    if ((k & 63u) == 0u) touch_block(rec, pair_gid, jw, stride, k, j1, tc);
    const uint32_t gid = __builtin_amdgcn_readfirstlane(pair_gid[j]);
    const Record r = load_record(rec, gid);
    const ColumnSetup s = column_setup<BZ>(r, px, py, pz0, iz0);
    const float szv = vreg(r.sz);
    uint32_t active = 0u;
    if (column_hit<BZ>(s, szv, cols, thr)) {
      active = forward_steps<BZ>(s, szv, r.c, thr, acc);
    }
    if (steps && j - jb < kStepCap && (threadIdx.x & 63) == 0) steps[j - jb] = active;
  }
  if (jw < j1) touch_end(tc);
}

// ---- where a brick lies --------------------------------------------------------
//
// Global brick b belongs to the last volume whose first brick is <= b; b is
// wave-uniform, so the search and the descriptor loads are scalar.
__device__ inline int item_of_brick(const ItemDesc* __restrict__ items, int nitems, uint32_t b) {
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].brick0 <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The lane's voxel column in brick b.
struct Site {
  int bx, by, bz;      // brick coordinates within its volume
  int iz0;             // first z of the brick (volume index)
  int zrem;            // voxels of the volume from iz0 on (may exceed the brick)
  float px, py, pz0;   // lane column position (world), first z
  bool col_in;         // the column lies inside the volume
  size_t org;          // brick's corner voxel (x, y, iz0) in the concatenated buffers (uniform)
  size_t plane;        // z stride
  uint32_t lbytes;     // byte offset of the lane's column from the corner (lx + nx ly) * 4

  // Address of the lane's voxel at brick offset zz: a uniform base plus a
  // 32-bit lane offset, the form global loads and stores take directly.
  template <typename T>
  __device__ T* at(T* buf, int zz) const {
    T* zb = buf + org + plane * (size_t)zz;
    return (T*)((char*)zb + lbytes);
  }
};

// c = the thread's column in the brick (x fastest): threadIdx.x, or its lane
// when several waves share the brick's columns.
template <int BXY, int BZ>
__device__ inline Site site_of(const ItemDesc* __restrict__ items, int nitems, uint32_t b,
                               uint32_t c = threadIdx.x) {
  const ItemDesc& it = items[item_of_brick(items, nitems, b)];
  const uint32_t lb = b - it.brick0;
  const uint32_t nbx = (uint32_t)it.nbx, nby = (uint32_t)it.nby;
  Site s;
  s.bx = (int)(lb % nbx);
  s.by = (int)((lb / nbx) % nby);
  s.bz = (int)(lb / (nbx * nby));
  const int ix = s.bx * BXY + (int)(c % BXY);
  const int iy = s.by * BXY + (int)(c / BXY);
  s.iz0 = s.bz * BZ;
  s.zrem = (int)it.nz - s.iz0;
  s.px = (float)(it.x0 + ix);
  s.py = (float)(it.y0 + iy);
  s.pz0 = (float)(it.z0 + s.iz0);
  s.col_in = ix < it.nx && iy < it.ny;
  s.plane = (size_t)it.nx * (size_t)it.ny;
  s.org = (size_t)it.vox + (size_t)(s.bx * BXY) + (size_t)it.nx * (size_t)(s.by * BXY) +
          s.plane * (size_t)s.iz0;
  s.lbytes = 4u * ((c % BXY) + (uint32_t)it.nx * (c / BXY));
  return s;
}

// Workgroup w -> brick when runs of consecutive bricks go to one XCD: the
// dispatcher deals workgroups round-robin over the 8 XCDs, so XCD x = w % 8
// runs its k-th workgroup (k = w / 8) on brick c C + k % C of chunk
// c = 8 (k / C) + x.  Chunks of C = 256 bricks (two rows of an 8 x 8 x 32
// brick grid at 1024^3) are small enough that the records of the primitives a
// chunk meets stay in that XCD's L2 while it works on it, and dealt in turn,
// so every XCD moves through the volume at the same pace (one contiguous
// eighth per XCD left dense regions to a few XCDs).  Bricks past the last
// whole round of 8 C keep their index (a bijection of [0, nb)).
constexpr uint32_t kXcdChunk = 256;

__device__ inline uint32_t xcd_brick(uint32_t w, uint32_t nb) {
  const uint32_t full = nb / (8u * kXcdChunk) * (8u * kXcdChunk);
  if (w >= full) return w;
  const uint32_t x = w & 7u, k = w >> 3;
  return ((k / kXcdChunk) * 8u + x) * kXcdChunk + k % kXcdChunk;
}

template <int BXY, int BZ>
__device__ __attribute__((always_inline)) inline void forward_brick(const Record* __restrict__ rec,
                                     const uint32_t* __restrict__ pair_gid,
                                     const uint32_t* __restrict__ brick_start,
                                     const ItemDesc* __restrict__ items, int nitems, uint32_t b,
                                     float thr, float* __restrict__ out) {
  const Site st = site_of<BXY, BZ>(items, nitems, b);
  float acc[BZ];
#pragma unroll
  for (int zz = 0; zz < BZ; ++zz) acc[zz] = 0.0f;
  accumulate_brick<BZ>(rec, pair_gid, brick_start[b], brick_start[b], 1u, brick_start[b + 1],
                       st.px, st.py, st.pz0, st.iz0, __builtin_amdgcn_ballot_w64(st.col_in), thr,
                       acc, nullptr);
  if (st.col_in) {
#pragma unroll
    for (int zz = 0; zz < BZ; ++zz)
      if (zz < st.zrem) *st.at(out, zz) = acc[zz];
  }
}

template <int BXY, int BZ>
__global__ __launch_bounds__(BXY* BXY) void k_forward(const Record* __restrict__ rec,
                                                  const uint32_t* __restrict__ pair_gid,
                                                  const uint32_t* __restrict__ brick_start,
                                                  const ItemDesc* __restrict__ items, int nitems,
                                                  uint32_t nbricks, int xcd, float thr,
                                                  float* __restrict__ out) {
  const uint32_t b = xcd ? xcd_brick(blockIdx.x, nbricks) : blockIdx.x;
  forward_brick<BXY, BZ>(rec, pair_gid, brick_start, items, nitems, b, thr, out);
}

// The backward steps of one pair over the brick offsets in `run`: moments
// of e = r G over zz.  CHECK skips offsets where no lane is inside the
// support; without it every offset in `run` must hold some lane inside (the
// offsets the forward pass recorded), and the steps carry no branch that
// waits on a compare.
template <int BZ, bool CHECK>
__device__ inline void backward_steps(const ColumnSetup& s, float szv, uint32_t run,
                                      const float (&res)[BZ], float thr, float& se, float& sK,
                                      float& sKK) {
#pragma unroll
  for (int g0 = 0; g0 < BZ; g0 += 8) {
    if ((run >> g0) & 0xFFu) {
#pragma unroll
      for (int zz = g0; zz < g0 + 8; ++zz) {
        if ((run >> zz) & 1u) {
          const float w = w_at<BZ>(s, szv, zz);
          const float q = quad_w(s, w);
          if (!CHECK || __builtin_amdgcn_ballot_w64(q > thr) != 0ull) {
            const float G = (q > thr) ? __builtin_amdgcn_exp2f(q) : 0.0f;
            const float e = res[zz] * G;
            se += e;
            sK = fmaf((float)zz, e, sK);
            sKK = fmaf((float)(zz * zz), e, sKK);
          }
        }
      }
    }
  }
}

// Backward steps of a recorded pair by recurrence.  Along a column Q is a
// parabola in zz: with R(zz) = exp2(Q(zz + 1) - Q(zz)) = exp2(-(2 w + sz) sz)
// and C = exp2(-2 sz^2) (the record's cz), G(zz + 1) = G(zz) R(zz) and
// R(zz + 1) = R(zz) C, two
// products per step in place of w, Q and an exp2.  The chain starts exactly
// one offset before the first recorded offset z0 (w, Q, and exp2 of Q and of
// the first difference there) and advances once per offset up to the last,
// z1; offsets between them that no lane reached add zero.  A lane whose
// starting Q is <= -100 starts at G = 0: the caller takes this path only
// when (z1 - z0 + 1) sz < reach = sqrt(100 + thr) - sqrt(-thr), and then no
// such lane can enter the support by z1 (|w| < sqrt(-thr) inside it, and |w|
// moves by sz per offset), so those lanes add nothing, as with the direct
// form; every other lane's chain keeps Q >= -100, inside the float range.
// Rounding grows along the chain, to about 1e-4 relative after 32 products:
// inside the gradient tolerance.  The forward pass, whose values must meet
// 1e-5, keeps the direct exponential.  The support test is G > T with
// T = exp2(thr).
template <int BZ>
__device__ inline void backward_steps_chain(const ColumnSetup& s, float szv, float sz, float C,
                                            int z0, int z1, const float (&res)[BZ], float T,
                                            float& se, float& sK, float& sKK) {
  const float w0 = fmaf((float)(z0 - 1 - BZ / 2), szv, s.wm);
  const float q0 = quad_w(s, w0);
  float G = q0 > -100.0f ? __builtin_amdgcn_exp2f(q0) : 0.0f;
  float R = __builtin_amdgcn_exp2f(fminf(-fmaf(2.0f, w0, sz) * sz, 100.0f));
  // offsets z0 .. z1 (z1 <= 31; 2u << 31 wraps to 0, giving all ones)
  const uint32_t span = ((2u << z1) - 1u) & ~((1u << z0) - 1u);
#pragma unroll
  for (int g0 = 0; g0 < BZ; g0 += 8) {
    if ((span >> g0) & 0xFFu) {
#pragma unroll
      for (int zz = g0; zz < g0 + 8; ++zz) {
        if ((span >> zz) & 1u) {
          // keeps the compiler from turning this uniform branch into selects
          // that would run every offset of the brick
          asm volatile("");
          G *= R;
          R *= C;
          const float e = res[zz] * (G > T ? G : 0.0f);
          se += e;
          sK = fmaf((float)zz, e, sK);
          sKK = fmaf((float)(zz * zz), e, sKK);
        }
      }
    }
  }
}

// Target values of the lane's column at brick offsets z0 .. z0 + NZ - 1
// (0 outside the volume), read as raw buffer loads: each z-plane's brick corner
// is a uniform resource base and the lane's byte offset the one per-lane
// operand, so the NZ loads share one offset register and are issued together
// (one wait per chunk rather than per voxel).  A lane whose column lies outside
// the volume passes an offset past the record count and reads 0.
constexpr int kLoadZ = 8;
// Fourth word of a gfx9-family buffer resource: 32-bit data format, no
// swizzle, no index stride (the offset is a plain byte offset).
constexpr int kBufferWord3 = 0x00020000;

__device__ inline float plane_load(const float* __restrict__ buf, const Site& st, int zz,
                                   uint32_t voff, int nrec) {
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(buf + st.org + st.plane * (size_t)zz), (short)0, nrec, kBufferWord3);
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, 0, 0));
}

template <int NZ>
__device__ inline void load_column_chunk(const float* __restrict__ field, const Site& st,
                                         uint32_t voff, int nrec, int z0, float (&t)[NZ]) {
  if (z0 + NZ <= st.zrem) {
#pragma unroll
    for (int u = 0; u < NZ; ++u) t[u] = plane_load(field, st, z0 + u, voff, nrec);
  } else {
#pragma unroll
    for (int u = 0; u < NZ; ++u)
      t[u] = z0 + u < st.zrem ? plane_load(field, st, z0 + u, voff, nrec) : 0.0f;
  }
}

// One brick of the fused pass.  VJP = false: residual r = 2 (Vhat - V) from
// the forward pass and the target `field`, loss share to brick_loss.
// VJP = true: no forward pass; r is read from `field` (an upstream gradient
// dl/dVhat), so the ten sums give the vector-Jacobian product
// sum_p r(p) dVhat(p)/dtheta.
// W > 1 (8 x 8 columns only): W waves share the brick's columns and split its
// pairs (wave w takes pairs w, w + W, ...); the forward partial sums are added
// in wave order through LDS (`comb`, W * BZ * 64 floats), after which every
// wave holds the whole field of the brick.  `comb` is then each wave's block
// of the ten-sum reduction (lds_sum10).
template <int BXY, int BZ, bool VJP, int W>
__device__ __attribute__((always_inline)) inline void fused_brick(const Record* __restrict__ rec,
                                   const uint32_t* __restrict__ pair_gid,
                                   const uint32_t* __restrict__ brick_start,
                                   const ItemDesc* __restrict__ items, int nitems, uint32_t b,
                                   float thr, const float* __restrict__ field,
                                   float* __restrict__ gacc, int64_t n, float* __restrict__ part,
                                   const uint32_t* __restrict__ pslot,
                                   float* __restrict__ brick_loss,
                                   float (*red)[10], uint32_t* __restrict__ steps,
                                   float* __restrict__ comb) {
  // `comb` holds the forward partial sums of W > 1 waves until they are
  // added, then the waves' ten-sum blocks (kSumFloats each)
  constexpr int kWaves = (BXY * BXY + 63) / 64;  // waves over the columns
  static_assert(W == 1 || kWaves == 1, "pairs are split only over one wave of columns");
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const Site st = site_of<BXY, BZ>(items, nitems, b, W > 1 ? (uint32_t)lane : threadIdx.x);
  const float px = st.px, py = st.py, pz0 = st.pz0;
  const int iz0 = st.iz0;
  const bool col_in = st.col_in;
  const uint64_t cols = __builtin_amdgcn_ballot_w64(col_in);
  const uint32_t j0 = brick_start[b], j1 = brick_start[b + 1];
  const uint32_t jw = j0 + (W > 1 ? (uint32_t)wave : 0u);  // this wave's first pair
  // target reads: lanes outside the volume read past the record count (0);
  // an inside lane's offset is below one plane and below 2^29 bytes
  static_assert(BZ % kLoadZ == 0, "brick depth must be a multiple of the load chunk");
  const uint32_t voff = col_in ? st.lbytes : 0x80000000u;
  const int nrec = (int)std::min(st.plane * 4, (size_t)0x7FFFFFFF);

  float res[BZ];
#pragma unroll
  for (int zz = 0; zz < BZ; ++zz) res[zz] = 0.0f;
  if (VJP) {
#pragma unroll
    for (int z0 = 0; z0 < BZ; z0 += kLoadZ) {
      float t[kLoadZ];
      load_column_chunk<kLoadZ>(field, st, voff, nrec, z0, t);
#pragma unroll
      for (int u = 0; u < kLoadZ; ++u) res[z0 + u] = t[u];
      asm volatile("" ::: "memory");
    }
  } else {
    accumulate_brick<BZ>(rec, pair_gid, j0, jw, (uint32_t)W, j1, px, py, pz0, iz0, cols, thr,
                         res, kWaves == 1 ? steps : nullptr);
    if (W > 1) {
      // the waves' partial sums, added in wave order
#pragma unroll
      for (int zz = 0; zz < BZ; ++zz) comb[(wave * BZ + zz) * 64 + lane] = res[zz];
      __syncthreads();
#pragma unroll
      for (int z0 = 0; z0 < BZ; z0 += 8) {
#pragma unroll
        for (int zz = z0; zz < z0 + 8; ++zz) {
          float t = 0.0f;
#pragma unroll
          for (int w = 0; w < W; ++w) t += comb[(w * BZ + zz) * 64 + lane];
          res[zz] = t;
        }
        // eight offsets at a time: the next reads wait for these sums, so
        // the loads in flight stay within 8 W registers
#pragma unroll
        for (int zz = z0; zz < z0 + 8; ++zz) asm volatile("" ::"v"(res[zz]) : "memory");
      }
      // every wave has read the partial sums before `comb` takes the waves'
      // ten-sum blocks
      __syncthreads();
    }
    // residual and this brick's share of the loss
    float lsum = 0.0f;
#pragma unroll
    for (int z0 = 0; z0 < BZ; z0 += kLoadZ) {
      float t[kLoadZ];
      load_column_chunk<kLoadZ>(field, st, voff, nrec, z0, t);
#pragma unroll
      for (int u = 0; u < kLoadZ; ++u) {
        const int zz = z0 + u;
        float r = 0.0f;
        if (col_in && zz < st.zrem) {
          const float d = res[zz] - t[u];
          lsum = fmaf(d, d, lsum);
          r = 2.0f * d;
        }
        res[zz] = r;
      }
      // one chunk of loads in flight at a time, each consumed before the
      // next is issued (the compiler would otherwise issue all of them first
      // and hold BZ more registers)
#pragma unroll
      for (int u = 0; u < kLoadZ; ++u) asm volatile("" ::"v"(res[z0 + u]));
      asm volatile("" : "+v"(lsum)::"memory");
    }
    lsum = wave_sum(lsum);
    if (W > 1) {
      if (threadIdx.x == 0) brick_loss[b] = lsum;  // every wave holds the same residual
    } else {
      if (lane == 0) red[wave][0] = lsum;
      __syncthreads();
      if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int w = 0; w < kWaves; ++w) t += red[w][0];
        brick_loss[b] = t;
      }
      __syncthreads();
    }
  }

  // support test and reach of the recurrence form of the backward steps
  const float T = __builtin_amdgcn_exp2f(thr);
  const float reach = 100.0f + thr > 0.0f ? sqrtf(100.0f + thr) - sqrtf(-thr) : 0.0f;
  for (uint32_t j = jw; j < j1; j += W) {
    const uint32_t gid = __builtin_amdgcn_readfirstlane(pair_gid[j]);
    const Record r = load_record(rec, gid);
    const ColumnSetup s = column_setup<BZ>(r, px, py, pz0, iz0);
    // the steps the forward pass found active, else the box's z-range
    const bool recorded = kWaves == 1 && !VJP && j - j0 < kStepCap;
    const uint32_t run = recorded ? __builtin_amdgcn_readfirstlane(steps[j - j0]) : s.zmask;
    const bool hit = recorded ? run != 0u : column_hit<BZ>(s, r.sz, cols, thr);
    if (kWaves == 1 && !hit) {
      // a pair whose support misses every column still owns a partials slot
      if (part && lane < 10)
        part[(size_t)pslot[j] * 10 + lane] = 0.0f;
      continue;
    }
    float v[10];
    {
      // moments of e over the brick offset zz (a literal operand per step)
      float se = 0.0f, sK = 0.0f, sKK = 0.0f;
      if (hit) {
        const float szv = vreg(r.sz);
        if (recorded) {
          const int z0 = (int)__builtin_ctz(run), z1 = 31 - (int)__builtin_clz(run);
          if ((float)(z1 - z0 + 1) * r.sz < reach)
            backward_steps_chain<BZ>(s, szv, r.sz, r.cz, z0, z1, res, T, se, sK, sKK);
          else
            backward_steps<BZ, false>(s, szv, run, res, thr, se, sK, sKK);
        } else {
          backward_steps<BZ, true>(s, szv, run, res, thr, se, sK, sKK);
        }
      }
      // dz = p_z - mu_z = ofs + zz with ofs = z0 - mu_z, so
      // sum e dz = sK + ofs se and sum e dz^2 = sKK + 2 ofs sK + ofs^2 se
      const float dx = px - r.mu[0];
      const float dy = py - r.mu[1];
      const float ofs = pz0 - r.mu[2];
      const float s1 = fmaf(ofs, se, sK);
      const float s2 = fmaf(ofs, fmaf(ofs, se, 2.0f * sK), sKK);
      const float xe = dx * se, ye = dy * se;
      v[0] = se;
      v[1] = xe;
      v[2] = ye;
      v[3] = s1;
      v[4] = dx * xe;
      v[5] = dy * xe;
      v[6] = dx * s1;
      v[7] = dy * ye;
      v[8] = dy * s1;
      v[9] = s2;
    }
    // sum a in lane a < 10 (each wave of the workgroup has its own block)
    const float sum = lds_sum10(v, comb + wave * kSumFloats, lane);
    if (kWaves == 1) {
      if (part) {
        if (lane < 10) part[(size_t)pslot[j] * 10 + lane] = sum;
      } else if (lane < 10) {
        unsafeAtomicAdd(&gacc[(int64_t)gid * kAccStride + lane], sum);
      }
    } else {
      if (lane < 10) red[wave][lane] = sum;
      __syncthreads();
      if (threadIdx.x < 10) {
        float t = 0.0f;
        for (int w = 0; w < kWaves; ++w) t += red[w][threadIdx.x];
        if (part) {
          part[(size_t)pslot[j] * 10 + threadIdx.x] = t;
        } else if (t != 0.0f) {
          unsafeAtomicAdd(&gacc[(int64_t)gid * kAccStride + threadIdx.x], t);
        }
      }
      __syncthreads();
    }
  }
}

// Floats of the fused kernels' shared block: the larger of the W > 1 forward
// partial sums and the waves' ten-sum blocks (the two are live one after the
// other).
constexpr int fused_lds_floats(int bz, bool vjp, int w, int waves) {
  const int comb = w > 1 && !vjp ? w * bz * 64 : 0;
  const int sums = w * waves * kSumFloats;
  return comb > sums ? comb : sums;
}

// One workgroup per brick (xcd: consecutive bricks grouped per XCD); W waves
// per brick split its pairs (fused_brick).
template <int BXY, int BZ, bool VJP, int W>
__global__ __launch_bounds__(BXY* BXY* W) void k_fused(const Record* __restrict__ rec,
                                                const uint32_t* __restrict__ pair_gid,
                                                const uint32_t* __restrict__ brick_start,
                                                const ItemDesc* __restrict__ items, int nitems,
                                                uint32_t nbricks, int xcd, float thr,
                                                const float* __restrict__ field,
                                                float* __restrict__ gacc, int64_t n,
                                                float* __restrict__ part,
                                                const uint32_t* __restrict__ pslot,
                                                float* __restrict__ brick_loss) {
  constexpr int kWaves = (BXY * BXY + 63) / 64;
  __shared__ float red[kWaves][10];
  __shared__ uint32_t steps[kWaves == 1 && !VJP ? kStepCap : 1];
  __shared__ __attribute__((aligned(16))) float comb[fused_lds_floats(BZ, VJP, W, kWaves)];
  const uint32_t b = xcd ? xcd_brick(blockIdx.x, nbricks) : blockIdx.x;
  fused_brick<BXY, BZ, VJP, W>(rec, pair_gid, brick_start, items, nitems, b, thr, field, gacc, n,
                               part, pslot, brick_loss, red, steps, comb);
}

// Persistent: each workgroup takes queue positions from *counter until they
// run out (every workgroup reaches that exit) and processes brick
// order[position] (heaviest first).
template <int BXY, int BZ, bool VJP, int W>
__global__ __launch_bounds__(BXY* BXY* W) void k_fused_queue(const Record* __restrict__ rec,
                                                      const uint32_t* __restrict__ pair_gid,
                                                      const uint32_t* __restrict__ brick_start,
                                                      const ItemDesc* __restrict__ items,
                                                      int nitems, uint32_t nbricks,
                                                      const uint32_t* __restrict__ order,
                                                      uint32_t* __restrict__ counter, float thr,
                                                      const float* __restrict__ field,
                                                      float* __restrict__ gacc, int64_t n,
                                                      float* __restrict__ part,
                                                      const uint32_t* __restrict__ pslot,
                                                      float* __restrict__ brick_loss) {
  constexpr int kWaves = (BXY * BXY + 63) / 64;
  __shared__ float red[kWaves][10];
  __shared__ uint32_t steps[kWaves == 1 && !VJP ? kStepCap : 1];
  __shared__ __attribute__((aligned(16))) float comb[fused_lds_floats(BZ, VJP, W, kWaves)];
  __shared__ uint32_t next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t w = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
    if (w >= nbricks) break;
    fused_brick<BXY, BZ, VJP, W>(rec, pair_gid, brick_start, items, nitems, order[w], thr,
                                 field, gacc, n, part, pslot, brick_loss, red, steps, comb);
  }
}

// Work counters of one evaluation: [0] in-support (primitive, voxel) pairs
// inside the grid (m^2 < k^2), [1] lane-voxel evaluations the brick kernels
// perform after their wave-level skips (the candidate pairs, masked lanes
// included), [2] (primitive, brick) pairs with an active step in some wave of
// the brick (the pairs whose gradient sums the fused kernel adds atomically).
template <int BXY, int BZ>
__global__ __launch_bounds__(BXY* BXY) void k_count(const Record* __restrict__ rec,
                                                const uint32_t* __restrict__ pair_gid,
                                                const uint32_t* __restrict__ brick_start,
                                                const ItemDesc* __restrict__ items, int nitems,
                                                float thr,
                                                unsigned long long* __restrict__ counts) {
  constexpr int kWaves = (BXY * BXY + 63) / 64;
  __shared__ uint32_t any[kWaves];
  const uint32_t b = blockIdx.x;
  const Site st = site_of<BXY, BZ>(items, nitems, b);
  const uint64_t cols = __builtin_amdgcn_ballot_w64(st.col_in);
  const int wave = threadIdx.x >> 6;
  unsigned long long nin = 0, ncand = 0, npair = 0;
  for (uint32_t j = brick_start[b]; j < brick_start[b + 1]; ++j) {
    const Record r = load_record(rec, __builtin_amdgcn_readfirstlane(pair_gid[j]));
    const ColumnSetup s = column_setup<BZ>(r, st.px, st.py, st.pz0, st.iz0);
    uint32_t active = 0u;
    if (column_hit<BZ>(s, r.sz, cols, thr)) {
      for (int zz = s.za; zz <= s.zb; ++zz) {
        const float q = quad_w(s, w_at<BZ>(s, r.sz, zz));
        if (__builtin_amdgcn_ballot_w64(q > thr) == 0ull) continue;
        active = 1u;
        ncand += 1;
        nin += (st.col_in && zz < st.zrem && q > thr) ? 1 : 0;
      }
    }
    // every wave of the brick walks the same pairs, so the barriers match
    if ((threadIdx.x & 63) == 0) any[wave] = active;
    if (kWaves > 1) __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t a = 0u;
      for (int w = 0; w < kWaves; ++w) a |= any[w];
      npair += a;
    }
    if (kWaves > 1) __syncthreads();
  }
  nin = wave_sum_u64(nin);
  ncand = wave_sum_u64(ncand);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&counts[0], nin);
    atomicAdd(&counts[1], ncand);
  }
  if (threadIdx.x == 0 && npair) atomicAdd(&counts[2], npair);
}

// Deterministic two-level sum of the per-brick losses in double precision.
constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 512;

__global__ __launch_bounds__(kRedThreads) void k_loss_partial(const float* __restrict__ x,
                                                              int64_t n, double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t a = (int64_t)blockIdx.x * per;
  const int64_t e = min(n, a + per);
  double s = 0.0;
  for (int64_t i = a + threadIdx.x; i < e; i += kRedThreads) s += (double)x[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kRedThreads) void k_loss_final(const double* __restrict__ part, int np,
                                                            double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += kRedThreads) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}


// Per-volume loss: one workgroup per volume sums its bricks' losses in double
// (fixed order, so deterministic).
__global__ __launch_bounds__(kRedThreads) void k_item_loss(const float* __restrict__ x,
                                                           const ItemDesc* __restrict__ items,
                                                           int nitems, int64_t nbricks,
                                                           double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  const int i = blockIdx.x;
  const int64_t a = items[i].brick0;
  const int64_t e = (i + 1 < nitems) ? (int64_t)items[i + 1].brick0 : nbricks;
  double s = 0.0;
  for (int64_t j = a + threadIdx.x; j < e; j += kRedThreads) s += (double)x[j];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = sh[0];
}

}  // namespace

#define GVE_BRICK_SHAPES(X) X(8, 8) X(8, 16) X(8, 32) X(16, 16)
// (brick edge, depth, waves per brick) of the fused kernels
#define GVE_FUSED_SHAPES(X)                                                                   \
  X(8, 8, 1) X(8, 8, 2) X(8, 8, 4) X(8, 16, 1) X(8, 16, 2) X(8, 16, 4) X(8, 32, 1) X(8, 32, 2) \
  X(8, 32, 4) X(16, 16, 1)

bool brick_shape_supported(int bxy, int bz) {
#define GVE_CASE(XY, Z) if (bxy == XY && bz == Z) return true;
  GVE_BRICK_SHAPES(GVE_CASE)
#undef GVE_CASE
  return false;
}

bool brick_waves_supported(int bxy, int bz, int waves) {
#define GVE_CASE(XY, Z, W) if (bxy == XY && bz == Z && waves == W) return true;
  GVE_FUSED_SHAPES(GVE_CASE)
#undef GVE_CASE
  return false;
}

int fused_resident_groups(int bxy, int bz, int waves, int device) {
  int per_cu = 0, cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 0;
#define GVE_CASE(XY, Z, W)                                                                    \
  if (bxy == XY && bz == Z && waves == W) {                                                   \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused_queue<XY, Z, false, W>, \
                                                     XY * XY * W, 0) != hipSuccess)           \
      return 0;                                                                               \
    return per_cu * cus;                                                                      \
  }
  GVE_FUSED_SHAPES(GVE_CASE)
#undef GVE_CASE
  return 0;
}

hipError_t launch_forward(const Record* rec, const uint32_t* pair_gid, const uint32_t* brick_start,
                          const ItemDesc* items, int nitems, BrickGeom bg, float k, float* out,
                          const Schedule& sc, hipStream_t s) {
  const float thr = -kHalfLog2e * k * k;
  if (bg.nbricks <= 0) return hipSuccess;
  const dim3 grid((unsigned)bg.nbricks);
  const int xcd = sc.kind == kSchedXcd ? 1 : 0;
#define GVE_CASE(XY, Z)                                                                       \
  if (bg.Bxy == XY && bg.Bz == Z) {                                                           \
    hipLaunchKernelGGL((k_forward<XY, Z>), grid, dim3(XY * XY), 0, s, rec, pair_gid,            \
                       brick_start, items, nitems, (uint32_t)bg.nbricks, xcd, thr, out);        \
    return hipGetLastError();                                                                 \
  }
  GVE_BRICK_SHAPES(GVE_CASE)
#undef GVE_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_fused(const Record* rec, const uint32_t* pair_gid, const uint32_t* brick_start,
                        const ItemDesc* items, int nitems, BrickGeom bg, float k,
                        const float* field, float* acc, int64_t n, float* part,
                        const uint32_t* pslot, float* brick_loss, const Schedule& sc,
                        hipStream_t s, bool vjp) {
  const float thr = -kHalfLog2e * k * k;
  if (bg.nbricks <= 0) return hipSuccess;
  const bool queue = sc.kind == kSchedQueue;
  if (queue && (!sc.order || !sc.counter || sc.persistent_groups <= 0)) return hipErrorInvalidValue;
  const dim3 grid(queue ? (unsigned)std::min<int64_t>(sc.persistent_groups, bg.nbricks)
                        : (unsigned)bg.nbricks);
  const int xcd = sc.kind == kSchedXcd ? 1 : 0;
  const uint32_t* order = sc.order;
  uint32_t* counter = sc.counter;
  const uint32_t nb = (uint32_t)bg.nbricks;
#define GVE_CASE(XY, Z, W)                                                                    \
  if (bg.Bxy == XY && bg.Bz == Z && bg.waves == W) {                                          \
    if (queue && vjp)                                                                         \
      hipLaunchKernelGGL((k_fused_queue<XY, Z, true, W>), grid, dim3(XY * XY * W), 0, s, rec,   \
                         pair_gid, brick_start, items, nitems, nb, order, counter, thr, field,  \
                         acc, n, part, pslot, brick_loss);                                     \
    else if (queue)                                                                           \
      hipLaunchKernelGGL((k_fused_queue<XY, Z, false, W>), grid, dim3(XY * XY * W), 0, s, rec,  \
                         pair_gid, brick_start, items, nitems, nb, order, counter, thr, field,  \
                         acc, n, part, pslot, brick_loss);                                     \
    else if (vjp)                                                                             \
      hipLaunchKernelGGL((k_fused<XY, Z, true, W>), grid, dim3(XY * XY * W), 0, s, rec,         \
                         pair_gid, brick_start, items, nitems, nb, xcd, thr, field, acc, n,     \
                         part, pslot, brick_loss);                                              \
    else                                                                                      \
      hipLaunchKernelGGL((k_fused<XY, Z, false, W>), grid, dim3(XY * XY * W), 0, s, rec,        \
                         pair_gid, brick_start, items, nitems, nb, xcd, thr, field, acc, n,     \
                         part, pslot, brick_loss);                                              \
    return hipGetLastError();                                                                 \
  }
  GVE_FUSED_SHAPES(GVE_CASE)
#undef GVE_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_count(const Record* rec, const uint32_t* pair_gid, const uint32_t* brick_start,
                        const ItemDesc* items, int nitems, BrickGeom bg, float k,
                        unsigned long long* counts, hipStream_t s) {
  const float thr = -kHalfLog2e * k * k;
  if (bg.nbricks <= 0) return hipSuccess;
  const dim3 grid((unsigned)bg.nbricks);
#define GVE_CASE(XY, Z)                                                                       \
  if (bg.Bxy == XY && bg.Bz == Z) {                                                           \
    hipLaunchKernelGGL((k_count<XY, Z>), grid, dim3(XY * XY), 0, s, rec, pair_gid, brick_start, \
                       items, nitems, thr, counts);                                             \
    return hipGetLastError();                                                                 \
  }
  GVE_BRICK_SHAPES(GVE_CASE)
#undef GVE_CASE
  return hipErrorInvalidValue;
}

size_t loss_reduce_tmp_doubles() { return kRedBlocks; }

hipError_t launch_loss_reduce(const float* brick_loss, int64_t nbricks, double* part, double* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_loss_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, s, brick_loss,
                     nbricks, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kRedThreads), 0, s, part, kRedBlocks, out);
  return hipGetLastError();
}

hipError_t launch_item_loss(const float* brick_loss, const ItemDesc* items, int nitems,
                            int64_t nbricks, double* out, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_item_loss, dim3((unsigned)nitems), dim3(kRedThreads), 0, s, brick_loss,
                     items, nitems, nbricks, out);
  return hipGetLastError();
}

}  // namespace gve
