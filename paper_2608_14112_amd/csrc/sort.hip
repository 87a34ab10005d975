// Stable LSD radix sort of (key, value) uint32 pairs.
//
// Sorts the (brick, primitive) overlap pairs by brick so that each brick's
// primitives form one contiguous run, in increasing primitive index (the
// pairs are emitted in primitive order and every pass is stable).  Each pass
// handles `w` <= 8 key bits:
//   1. per-tile digit histogram, stored tile-major: hist[tile * 256 + d] (one
//      coalesced row per tile);
//   2. global write offsets offs[tile * 256 + d] = (items of all smaller
//      digits) + (items of digit d in earlier tiles): column sums over
//      chunks of tiles, one workgroup scanning the chunk sums and the digit
//      totals, then the chunks' running column sums (every access a
//      coalesced row);
//   3. stable scatter: a tile is ordered by digit in LDS, consumed in rounds
//      of 256 items in index order (an item's rank among equal digits in its
//      wave comes from up to eight ballots, across waves from per-wave counts
//      in LDS), then written out run by run.
// Tiles are 4,096 items (16 rounds): at 5e7 pairs and 7-bit digits a digit's
// run in a tile averages 32 items (128 bytes of keys), so the scatter's writes
// stay close to whole lines; 2,048- and 8,192-item tiles were slower.
#include "common.h"

namespace gve {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kRounds = 16;
constexpr int kTile = kThreads * kRounds;
constexpr int kRadix = 256;

// Items to sort: n, or (with a device count) the smaller of n and *dn.  The
// launch covers n items; tiles past the device count are empty.
__device__ inline int64_t items_of(int64_t n, const uint32_t* __restrict__ dn) {
  return dn ? min(n, (int64_t)*dn) : n;
}

__global__ __launch_bounds__(kThreads) void k_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                   const uint32_t* __restrict__ dn, int shift,
                                                   uint32_t mask, int64_t ntiles,
                                                   uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[kRadix];
  n = items_of(n, dn);
  const int64_t base = (int64_t)blockIdx.x * kTile;
  if (base >= n) {  // a tile past the items (the launch covers the capacity)
    hist[(int64_t)blockIdx.x * kRadix + threadIdx.x] = 0u;
    return;
  }
  // the tile's keys, all loads issued before the first count
  uint32_t tk[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
    tk[r] = i < n ? keys[i] : 0u;
  }
  cnt[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(tk[r] >> shift) & mask], 1u);
  }
  __syncthreads();
  hist[(int64_t)blockIdx.x * kRadix + threadIdx.x] = cnt[threadIdx.x];
}

// Exclusive prefix sum of one value per thread over the block.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* __restrict__ wsum) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wave; ++w) before += wsum[w];
  return before + incl - v;
}

// Column sums of the tile-major histogram over chunks of `crows` tiles:
// csum[chunk * 256 + d] (thread d; every step reads one 1 KB row).
__global__ __launch_bounds__(kThreads) void k_col_reduce(const uint32_t* __restrict__ hist,
                                                         int64_t ntiles, int64_t crows,
                                                         uint32_t* __restrict__ csum) {
  const int64_t r0 = (int64_t)blockIdx.x * crows;
  const int64_t r1 = min(r0 + crows, ntiles);
  uint32_t s = 0;
#pragma unroll 16
  for (int64_t r = r0; r < r1; ++r) s += hist[r * kRadix + threadIdx.x];
  csum[(int64_t)blockIdx.x * kRadix + threadIdx.x] = s;
}

// One workgroup of 1024 threads: per digit, the exclusive scan over `nrows`
// (<= 256) rows of 256 counts, plus the items of all smaller digits, written
// to out (which may be in: the chunk sums are scanned in place, and a
// histogram of at most 256 tiles is scanned straight into the offsets).
// Thread (q, d) takes digit d over a quarter of the rows.
constexpr int kScanParts = 4;
constexpr int kScanThreads = kScanParts * kRadix;
__global__ __launch_bounds__(kScanThreads) void k_col_scan(const uint32_t* in, uint32_t* out,
                                                           int64_t nrows) {
  __shared__ uint32_t part[kScanParts][kRadix];
  __shared__ uint32_t wsum[kWaves];
  __shared__ uint32_t dbase[kRadix];
  const int d = threadIdx.x & (kRadix - 1);
  const int q = threadIdx.x / kRadix;
  const int64_t per = (nrows + kScanParts - 1) / kScanParts;
  const int64_t c0 = min(q * per, nrows);
  const int64_t c1 = min(c0 + per, nrows);
  uint32_t sum = 0;
#pragma unroll 16
  for (int64_t c = c0; c < c1; ++c) sum += in[c * kRadix + d];
  part[q][d] = sum;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int r = 0; r < kScanParts; ++r) {
    const uint32_t v = part[r][d];
    before += r < q ? v : 0u;
    total += v;
  }
  // digit bases: exclusive scan of the totals over the digits (the first
  // four waves, one digit per thread)
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint32_t incl = total;
  if (q == 0) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
  }
  __syncthreads();
  if (q == 0) {
    uint32_t w = 0;
    for (int v = 0; v < wave; ++v) w += wsum[v];
    dbase[d] = w + incl - total;
  }
  __syncthreads();
  uint32_t run = dbase[d] + before;
#pragma unroll 16
  for (int64_t c = c0; c < c1; ++c) {
    const uint32_t v = in[c * kRadix + d];
    out[c * kRadix + d] = run;
    run += v;
  }
}

// The chunk's running column sums: offs[t * 256 + d] for its tiles.
__global__ __launch_bounds__(kThreads) void k_col_apply(const uint32_t* __restrict__ hist,
                                                        int64_t ntiles, int64_t crows,
                                                        const uint32_t* __restrict__ cbase,
                                                        uint32_t* __restrict__ offs) {
  const int64_t r0 = (int64_t)blockIdx.x * crows;
  const int64_t r1 = min(r0 + crows, ntiles);
  uint32_t run = cbase[(int64_t)blockIdx.x * kRadix + threadIdx.x];
#pragma unroll 16
  for (int64_t r = r0; r < r1; ++r) {
    const uint32_t v = hist[r * kRadix + threadIdx.x];
    offs[r * kRadix + threadIdx.x] = run;
    run += v;
  }
}

// Stable scatter of one tile: the tile is first ordered by digit in LDS
// (rounds of 256 items in index order; an item's rank among equal digits in
// its wave from the ballots, across waves from per-wave counts), then written
// out in that order, so each digit's run of the tile lands as one contiguous
// stretch of the output.  Two barriers per round: the per-round counts and
// staged totals alternate between two buffers, so each round's second phase
// also prepares the next (four barriers per round before: binning 1.64 ->
// 1.60 ms at 5e7 pairs).
__global__ __launch_bounds__(kThreads) void k_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, int64_t n,
    const uint32_t* __restrict__ dn, int shift, uint32_t mask, int wbits, int64_t ntiles,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ offs,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout) {
  n = items_of(n, dn);
  if ((int64_t)blockIdx.x * kTile >= n) return;  // a tile past the items: nothing to move
  // the tile's items, all loads issued at once (the rounds below are
  // separated by barriers, which would otherwise expose one load latency
  // per round)
  const int64_t base = (int64_t)blockIdx.x * kTile;
  uint32_t tk[kRounds], tv[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
    tk[r] = i < n ? kin[i] : 0u;
    tv[r] = i < n ? vin[i] : 0u;
  }
  __shared__ uint32_t skey[kTile], sval[kTile];
  __shared__ uint32_t bstart[kRadix];         // tile-local start of each digit
  // per round (two buffers, alternating): items of each digit staged before
  // the round, and the round's count per digit of each wave, one byte per
  // wave (at most 64) in one word per digit
  __shared__ uint32_t run[2][kRadix];
  __shared__ uint32_t wcnt[2][kRadix];
  __shared__ uint32_t wsum[kWaves];
  __shared__ uint32_t delta[kRadix];          // output position - tile-local position, per digit
  static_assert(kWaves == 4, "four wave counts per word");
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint32_t mine = hist[(int64_t)blockIdx.x * kRadix + threadIdx.x];
  const uint32_t out0 = offs[(int64_t)blockIdx.x * kRadix + threadIdx.x];
  const uint32_t start = block_exclusive_scan(mine, wsum);
  bstart[threadIdx.x] = start;
  delta[threadIdx.x] = out0 - start;
  run[0][threadIdx.x] = 0;
  wcnt[0][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int b = r & 1;
    const int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
    const bool valid = i < n;
    const uint32_t key = tk[r], val = tv[r];
    const uint32_t d = valid ? (key >> shift) & mask : 0u;
    // lanes holding the same digit (invalid lanes excluded)
    uint64_t same = __ballot(valid);
    for (int bit = 0; bit < wbits; ++bit) {
      uint64_t bal = __ballot((d >> bit) & 1u);
      same &= ((d >> bit) & 1u) ? bal : ~bal;
    }
    const uint32_t rank_in_wave = __popcll(same & lt_mask);
    if (valid && rank_in_wave == 0)
      reinterpret_cast<uint8_t*>(&wcnt[b][d])[wave] = (uint8_t)__popcll(same);
    __syncthreads();
    if (valid) {
      // byte w of c * 0x01010100 = counts of waves 0 .. w - 1 (sums <= 192)
      const uint32_t c = wcnt[b][d];
      const uint32_t before = ((c * 0x01010100u) >> (8 * wave)) & 0xFFu;
      const uint32_t pos = bstart[d] + run[b][d] + before + rank_in_wave;
      skey[pos] = key;
      sval[pos] = val;
    }
    // digit threadIdx.x: the next round's staged count, and the other
    // buffer's counts cleared (last read in the previous round)
    {
      const uint32_t c = wcnt[b][threadIdx.x];
      const uint32_t add = (((c * 0x01010100u) >> 24) & 0xFFu) + (c >> 24);
      run[b ^ 1][threadIdx.x] = run[b][threadIdx.x] + add;
      wcnt[b ^ 1][threadIdx.x] = 0;
    }
    __syncthreads();
  }
  const int64_t cnt = (n - base) < kTile ? (n - base) : kTile;
  for (int j = threadIdx.x; j < cnt; j += kThreads) {
    const uint32_t key = skey[j];
    const uint32_t pos = (uint32_t)j + delta[(key >> shift) & mask];
    kout[pos] = key;
    vout[pos] = sval[j];
  }
}

int64_t ntiles_of(int64_t n) { return (n + kTile - 1) / kTile; }

// At most 256 chunks of tiles, so that one workgroup scans the chunk sums.
int64_t chunk_rows(int64_t ntiles) { return (ntiles + kRadix - 1) / kRadix; }

}  // namespace

// Room for a sort of any item count up to n: the histogram and the offsets
// (256 per tile), and the chunk sums sized for the largest chunk count, 256
// (the count for fewer items can be larger: 512 tiles make 256 chunks of 2,
// 513 tiles 171 chunks of 3).
size_t sort_hist_bytes(int64_t n) {
  int64_t t = ntiles_of(n > 0 ? n : 1);
  int64_t h = (int64_t)kRadix * t;
  return (2 * (size_t)h + (size_t)kRadix * kRadix) * sizeof(uint32_t) + 256;
}

hipError_t radix_sort_pairs(uint32_t* keys[2], uint32_t* vals[2], int64_t n, int bits,
                            void* hist_mem, int* which, hipStream_t s, const uint32_t* dn) {
  *which = 0;
  if (n <= 1 || bits <= 0) return hipSuccess;
  const int64_t t = ntiles_of(n);
  const int64_t h = (int64_t)kRadix * t;
  uint32_t* hist = static_cast<uint32_t*>(hist_mem);
  uint32_t* offs = hist + h;
  uint32_t* csum = offs + h;  // [chunks <= 256][256]
  const int64_t crows = chunk_rows(t);
  const int64_t nchunks = (t + crows - 1) / crows;
  const int passes = (bits + 7) / 8;
  const int w = (bits + passes - 1) / passes;
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * w;
    const int wb = (shift + w <= bits) ? w : (bits - shift);
    const uint32_t mask = (1u << wb) - 1u;
    hipLaunchKernelGGL(k_hist, dim3((unsigned)t), dim3(kThreads), 0, s, keys[cur], n, dn, shift,
                       mask, t, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (t <= kRadix) {
      // one tile per chunk: the chunk sums would be the histogram's rows
      hipLaunchKernelGGL(k_col_scan, dim3(1), dim3(kScanThreads), 0, s, hist, offs, t);
    } else {
      hipLaunchKernelGGL(k_col_reduce, dim3((unsigned)nchunks), dim3(kThreads), 0, s, hist, t,
                         crows, csum);
      hipLaunchKernelGGL(k_col_scan, dim3(1), dim3(kScanThreads), 0, s, csum, csum, nchunks);
      hipLaunchKernelGGL(k_col_apply, dim3((unsigned)nchunks), dim3(kThreads), 0, s, hist, t,
                         crows, csum, offs);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)t), dim3(kThreads), 0, s, keys[cur], vals[cur], n,
                       dn, shift, mask, wb, t, hist, offs, keys[cur ^ 1], vals[cur ^ 1]);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur ^= 1;
  }
  *which = cur;
  return hipSuccess;
}

}  // namespace gve
