// C ABI of libgve.so: argument validation, device memory, and the order in
// which the binning, field and update kernels are queued on the caller's
// stream.  Declarations and contracts are in include/gve.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "devmath.h"

using gve::Scratch;

// Device memory of the allocation-free entry point (gve_loss_grad_static):
// every workspace buffer of one loss-and-gradient call is carved from it.
// Each device the library runs on holds its own copy until the process ends;
// host code reaches a device's copy only through the address that
// hipGetSymbolAddress returns for it (scratch_address below).
constexpr size_t kStaticScratchBytes = GVE_STATIC_SCRATCH_BYTES;
static_assert(kStaticScratchBytes % 256 == 0, "static scratch size");
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Zero columns [off, off + cnt) of an [rows][ld] float array.
__global__ void k_zero_cols(float* __restrict__ p, int64_t ld, int64_t off, int64_t cnt, int rows) {
  const int64_t total = cnt * rows;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x)
    p[(i / cnt) * ld + off + i % cnt] = 0.0f;
}

// Address of `scratch` on each device, resolved once per device with that
// device current (gve_create).  A failed lookup is remembered as its error.
std::mutex g_scratch_mu;
std::map<int, std::pair<void*, hipError_t>> g_scratch_addr;

void resolve_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr.count(device)) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_scratch_addr[device] = std::make_pair(e == hipSuccess ? ptr : nullptr, e);
}

std::pair<void*, hipError_t> scratch_address(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it == g_scratch_addr.end()) return std::make_pair(nullptr, hipErrorNotInitialized);
  return it->second;
}

gve_status fail(const gve_ctx* ctx, gve_status st, const std::string& msg) {
  if (ctx) const_cast<gve_ctx*>(ctx)->last_error = msg;
  return st;
}

gve_status from_hip(const gve_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return GVE_OK;
  const gve_status st = (e == hipErrorOutOfMemory) ? GVE_ERR_OUT_OF_MEMORY : GVE_ERR_DEVICE;
  return fail(ctx, st, std::string(what) + ": " + hipGetErrorString(e));
}

#define TRY_HIP(ctx, call)                                         \
  do {                                                             \
    hipError_t e_ = (call);                                        \
    if (e_ != hipSuccess) return from_hip((ctx), e_, #call);       \
  } while (0)

#define TRY(call)                        \
  do {                                   \
    gve_status s_ = (call);              \
    if (s_ != GVE_OK) return s_;         \
  } while (0)

// A buffer of the allocation-free entry point: the next 256-byte aligned
// piece of the context's fixed region, or UNSUPPORTED when it does not fit.
gve_status carve(gve_ctx* ctx, Scratch& s, size_t bytes) {
  const size_t off = (ctx->arena_used + 255) & ~(size_t)255;
  if (bytes > ctx->arena_cap || off > ctx->arena_cap - bytes)
    return fail(ctx, GVE_ERR_UNSUPPORTED,
                "the workload needs more than the " + std::to_string(ctx->arena_cap >> 20) +
                    " MiB of static scratch of the allocation-free entry point (at least " +
                    std::to_string((off + bytes + 1048575) >> 20) + " MiB)");
  s.ptr = ctx->arena_base + off;
  s.bytes = bytes;
  ctx->arena_used = off + bytes;
  return GVE_OK;
}

// Grow-only device buffer.  Synchronises before freeing the old allocation.
gve_status ensure(gve_ctx* ctx, Scratch& s, size_t bytes) {
  if (s.bytes >= bytes && s.ptr) return GVE_OK;
  if (ctx->arena_base) return carve(ctx, s, bytes);
  if (s.ptr) {
    TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    TRY_HIP(ctx, hipFree(s.ptr));
    s.ptr = nullptr;
    s.bytes = 0;
  }
  size_t want = bytes + bytes / 4 + 256;
  TRY_HIP(ctx, hipMalloc(&s.ptr, want));
  s.bytes = want;
  return GVE_OK;
}

// Small device block: [0] loss (double), [2] clamp count and [3] non-finite
// parameter count (u64, cumulative), [4 .. 6] work counters of the counting
// pass, [16 ..] loss-reduction partials, then kTotalSlots pair-total counters
// and the degenerate-quaternion counter (u64).  Zeroed when first allocated.
gve_status ensure_dloss(gve_ctx* ctx) {
  if (ctx->ws.dloss.ptr) return GVE_OK;
  const size_t nd = 16 + gve::loss_reduce_tmp_doubles() + gve::kTotalSlots + 1;
  TRY(ensure(ctx, ctx->ws.dloss, sizeof(double) * nd));
  TRY_HIP(ctx, gve::fill_u64(static_cast<unsigned long long*>(ctx->ws.dloss.ptr), (int64_t)nd,
                             ctx->stream));
  return GVE_OK;
}

unsigned long long* pair_total_slots(gve_ctx* ctx) {
  return reinterpret_cast<unsigned long long*>(ctx->ws.dloss.ptr) + 16 +
         gve::loss_reduce_tmp_doubles();
}

gve_status validate_options(const gve_ctx* ctx, const gve_options& o) {
  if (!(o.k > 0.0f) || !std::isfinite(o.k) || o.k > 64.0f)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "k must be finite, > 0 and <= 64");
  if (o.brick != 0) {  // brick 0: automatic (brick_z and brick_waves are then not used)
    const int bz = o.brick_z == 0 ? o.brick : o.brick_z;
    if (!gve::brick_shape_supported(o.brick, bz))
      return fail(ctx, GVE_ERR_UNSUPPORTED,
                  "brick shape must be 8x8x8, 8x8x16, 8x8x32 or 16x16x16");
    if (!gve::brick_waves_supported(o.brick, bz, o.brick_waves == 0 ? 1 : o.brick_waves))
      return fail(ctx, GVE_ERR_UNSUPPORTED,
                  "brick_waves must be 0 or 1, or 2 or 4 with 8 x 8 columns");
  }
  if (!(o.lr >= 0.0f) || !std::isfinite(o.lr))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "lr must be finite and >= 0");
  if (!(o.beta1 >= 0.0f && o.beta1 < 1.0f) || !(o.beta2 >= 0.0f && o.beta2 < 1.0f))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "beta1, beta2 must lie in [0, 1)");
  if (!(o.eps > 0.0f) || !std::isfinite(o.eps))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "eps must be finite and > 0");
  if (o.deterministic != 0 && o.deterministic != 1)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "deterministic must be 0 or 1");
  if (o.schedule < GVE_SCHED_INDEX || o.schedule > GVE_SCHED_QUEUE)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "schedule must be 0, 1 or 2");
  if (std::isnan(o.ell_min) || std::isnan(o.ell_max) || o.ell_min > o.ell_max)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "ell_min must be <= ell_max");
  return GVE_OK;
}

gve_status validate_grid(const gve_ctx* ctx, const gve_grid& g) {
  if (g.nx <= 0 || g.ny <= 0 || g.nz <= 0)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "grid dimensions must be positive");
  const int64_t lim = (int64_t)1 << 24;  // voxel coordinates exact in float32
  if (g.nx > lim || g.ny > lim || g.nz > lim || std::llabs(g.x0) > lim || std::llabs(g.y0) > lim ||
      std::llabs(g.z0) > lim || std::llabs(g.x0) + g.nx > lim || std::llabs(g.y0) + g.ny > lim ||
      std::llabs(g.z0) + g.nz > lim)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "grid extent and origin must stay below 2^24");
  const double vox = (double)g.nx * (double)g.ny * (double)g.nz;
  if (vox > 1.6e10) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "grid too large");
  return GVE_OK;
}

// Brick shape and schedule of the next binning: the options', or with
// options.brick = 0 the automatic choice (select_auto).
int brick_xy(const gve_ctx* ctx) { return ctx->opt.brick == 0 ? ctx->auto_bxy : ctx->opt.brick; }
int brick_z(const gve_ctx* ctx) {
  if (ctx->opt.brick == 0) return ctx->auto_bz;
  return ctx->opt.brick_z == 0 ? brick_xy(ctx) : ctx->opt.brick_z;
}
int sched_of(const gve_ctx* ctx) {
  return ctx->opt.brick == 0 ? ctx->auto_sched : ctx->opt.schedule;
}
int waves_of(const gve_ctx* ctx) {
  if (ctx->opt.brick == 0) return ctx->auto_waves;
  return ctx->opt.brick_waves == 0 ? 1 : ctx->opt.brick_waves;
}

struct Vol;
gve_status select_auto(gve_ctx* ctx, const gve_params* p, const float* d_field, const Vol& vol,
                       bool tune);

int bits_for(int64_t nbricks) {
  int b = 0;
  while (((int64_t)1 << b) < nbricks) ++b;
  return b;
}

// A set of volumes and the primitive ranges that belong to each.
struct Vol {
  const gve_grid* grids;
  const int64_t* prim_off;  // [n + 1]
  int n;
};

struct Binned {
  gve::BrickGeom bg;
  const gve::ItemDesc* items = nullptr;  // device
  int nitems = 0;
  gve::Schedule sched;
  const uint32_t* gid = nullptr;   // primitive of each sorted pair
  const uint32_t* slot = nullptr;  // its emission index (deterministic sums), else null
  const uint32_t* start = nullptr;
  const uint32_t* sorted_keys = nullptr;  // brick key of each sorted pair
  int64_t npairs = 0;      // pairs (-1: counted on the device only)
  int64_t capacity = 0;    // pairs the buffers hold (>= npairs)
  int64_t box_total = -1;  // box pairs before culling (synchronous binning)
  const uint32_t* fits = nullptr;  // device flag of an asynchronous binning
};

// Volume descriptors on the device for the current brick shape.  The upload
// is followed by a synchronisation, so the host copy (which the device copy
// mirrors) is never rewritten while a transfer from it is pending.
gve_status upload_items(gve_ctx* ctx, const Vol& vol, int Bxy, int Bz, int64_t* nbricks) {
  std::vector<gve::ItemDesc> h((size_t)vol.n);
  *nbricks = gve::build_items(vol.grids, vol.prim_off, vol.n, Bxy, Bz, h.data());
  const bool same = h.size() == ctx->items_host.size() && ctx->ws.items.ptr &&
                    std::memcmp(h.data(), ctx->items_host.data(),
                                sizeof(gve::ItemDesc) * h.size()) == 0;
  if (same) return GVE_OK;
  TRY(ensure(ctx, ctx->ws.items, sizeof(gve::ItemDesc) * h.size()));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ctx->items_host.swap(h);
  TRY_HIP(ctx, hipMemcpyAsync(ctx->ws.items.ptr, ctx->items_host.data(),
                              sizeof(gve::ItemDesc) * ctx->items_host.size(),
                              hipMemcpyHostToDevice, ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return GVE_OK;
}

int resident_groups(gve_ctx* ctx, int bxy, int bz, int waves) {
  const std::array<int, 3> key = {bxy, bz, waves};
  auto it = ctx->resident.find(key);
  if (it != ctx->resident.end()) return it->second;
  const int r = gve::fused_resident_groups(bxy, bz, waves, ctx->device);
  ctx->resident[key] = r;
  return r;
}

// prep -> (scan -> cull ->) scan -> emit -> radix sort -> brick ranges (->
// heaviest-first order for the queue schedule).  Reads the box pair total (and
// with culling the kept total) back to the host, small synchronising copies
// that size the pair buffers.
// Destination of a copy of the emitted (unsorted) pair list, for inspection.
struct EmitCopy {
  uint32_t* keys = nullptr;
  uint32_t* vals = nullptr;
  int64_t capacity = 0;
  bool fits = false;  // set when the list fitted and was copied
};

bool same_items(const std::vector<gve::ItemDesc>& a, const std::vector<gve::ItemDesc>& b) {
  return a.size() == b.size() &&
         (a.empty() || std::memcmp(a.data(), b.data(), sizeof(gve::ItemDesc) * a.size()) == 0);
}

// Flags of the asynchronous binning in the small device block: [7] fits
// (u32) and sticky (u32), [8] the largest box pair total and [9] the largest
// kept pair total seen (u64).
uint32_t* fits_flag(gve_ctx* ctx) {
  return reinterpret_cast<uint32_t*>(static_cast<unsigned long long*>(ctx->ws.dloss.ptr) + 7);
}
uint32_t* sticky_flag(gve_ctx* ctx) { return fits_flag(ctx) + 1; }
unsigned long long* need_slot(gve_ctx* ctx) {
  return static_cast<unsigned long long*>(ctx->ws.dloss.ptr) + 8;
}
unsigned long long* need_pairs_slot(gve_ctx* ctx) {
  return static_cast<unsigned long long*>(ctx->ws.dloss.ptr) + 9;
}

// prep -> scan -> cull -> scan -> emit -> radix sort -> brick ranges (->
// heaviest-first order for the queue schedule).
//
// Synchronous (async = false): reads the box pair total and the kept total
// back to the host (two small synchronising copies) and sizes the pair
// buffers from them.  Asynchronous (async = true, refinement after its first
// iteration): no host read; the buffers hold ctx->pair_cap pairs, every
// count after the cull is read on the device, and a binning whose box pairs
// exceed the capacity keeps no pair and raises the fits / sticky flags (the
// caller redoes the work with larger buffers).  out->npairs = -1 then.
gve_status bin_vol(gve_ctx* ctx, const gve_params* p, const Vol& vol, Binned* out,
                   EmitCopy* ec = nullptr, bool async = false) {
  TRY(select_auto(ctx, p, nullptr, vol, false));
  hipStream_t s = ctx->stream;
  auto& ws = ctx->ws;
  const int64_t n = p->n;
  gve::BrickGeom bg;
  bg.Bxy = brick_xy(ctx);
  bg.Bz = brick_z(ctx);
  bg.waves = waves_of(ctx);
  TRY(upload_items(ctx, vol, bg.Bxy, bg.Bz, &bg.nbricks));
  if (bg.nbricks >= ((int64_t)1 << 31))
    return fail(ctx, GVE_ERR_UNSUPPORTED, "too many bricks for 32-bit brick keys");
  // capacity sized for these volumes and this brick shape only
  if (async && (ctx->box_cap <= 0 || !same_items(ctx->pair_cap_items, ctx->items_host)))
    async = false;
  const gve::ItemDesc* items = static_cast<const gve::ItemDesc*>(ws.items.ptr);
  TRY(ensure(ctx, ws.scan_tmp, gve::scan_tmp_bytes(n + 1)));
  TRY(ensure_dloss(ctx));
  unsigned long long* total = pair_total_slots(ctx);
  TRY_HIP(ctx, gve::fill_u64(total, gve::kTotalSlots + 1, s));
  TRY_HIP(ctx, gve::launch_prep(p->theta, n, items, vol.n, ctx->opt.k, bg, p->rec, p->count,
                                total, s));
  // Culling drops bricks a separating plane parts from the support.  The box
  // total bounds the kept total, so below the limit every 32-bit scan is
  // exact.  Deterministic sums address a pair's partials by its emission
  // index, which the sort carries as the value.
  const bool slots = ctx->opt.deterministic != 0;
  unsigned char* hp = static_cast<unsigned char*>(ws.h_pinned);
  TRY(ensure(ctx, ws.box_off, sizeof(uint32_t) * (size_t)(n + 1)));
  uint32_t* box_off = static_cast<uint32_t*>(ws.box_off.ptr);
  TRY_HIP(ctx, gve::scan_exclusive_u32(p->count, box_off, n, ws.scan_tmp.ptr, s));
  unsigned long long cap = 0;       // pairs the buffers hold
  const uint32_t* fits = nullptr;   // device flag of the asynchronous binning
  const uint32_t* dn = nullptr;     // device pair count (asynchronous)
  if (async) {
    cap = (unsigned long long)ctx->box_cap;
    TRY_HIP(ctx, gve::launch_fits(total, nullptr, cap, fits_flag(ctx), sticky_flag(ctx),
                                  need_slot(ctx), s));
    fits = fits_flag(ctx);
    dn = p->offset + n;
  } else {
    static_assert(sizeof(unsigned long long) * (gve::kTotalSlots + 1) <= 512,
                  "pinned staging size");
    TRY_HIP(ctx, hipMemcpyAsync(hp, total, sizeof(unsigned long long) * (gve::kTotalSlots + 1),
                                hipMemcpyDeviceToHost, s));
    TRY_HIP(ctx, hipStreamSynchronize(s));
    unsigned long long box_total = 0;
    for (int j = 0; j < gve::kTotalSlots; ++j)
      box_total += reinterpret_cast<const unsigned long long*>(hp)[j];
    ctx->stats.n_degenerate_q =
        (int64_t) reinterpret_cast<const unsigned long long*>(hp)[gve::kTotalSlots];
    if (box_total >= 0xFFFFFFF0ull)
      return fail(ctx, GVE_ERR_UNSUPPORTED,
                  "more than 2^32 (primitive, brick) pairs; use larger bricks or a smaller k");
    cap = box_total;
    out->box_total = (int64_t)box_total;
  }
  // the kept keys wait in the sort's second key buffer until emission
  TRY(ensure(ctx, ws.keys[1], sizeof(uint32_t) * (size_t)(cap > 0 ? cap : 1)));
  uint32_t* kept = static_cast<uint32_t*>(ws.keys[1].ptr);
  TRY_HIP(ctx, gve::launch_cull(p->rec, n, box_off, items, vol.n, bg, ctx->opt.k, kept, p->count,
                                s, fits));
  TRY_HIP(ctx, gve::scan_exclusive_u32(p->count, p->offset, n, ws.scan_tmp.ptr, s));
  unsigned long long T = cap;       // pairs (synchronous) or capacity (asynchronous)
  if (async) {
    T = (unsigned long long)ctx->pair_cap;
    TRY_HIP(ctx, gve::launch_fits(nullptr, p->offset + n, T, fits_flag(ctx), sticky_flag(ctx),
                                  need_pairs_slot(ctx), s));
  } else {
    TRY_HIP(ctx, hipMemcpyAsync(hp + 8, p->offset + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    TRY_HIP(ctx, hipStreamSynchronize(s));
    T = *reinterpret_cast<uint32_t*>(hp + 8);
  }
  const size_t pair_bytes = sizeof(uint32_t) * (size_t)(T > 0 ? T : 1);
  for (int b = 0; b < 2; ++b) {
    TRY(ensure(ctx, ws.keys[b], pair_bytes));  // keys[1] already holds >= T: kept
    TRY(ensure(ctx, ws.vals[b], pair_bytes));
  }
  const bool queue = sched_of(ctx) == GVE_SCHED_QUEUE;
  TRY(ensure(ctx, ws.sort_hist,
             gve::sort_hist_bytes(std::max<int64_t>((int64_t)T, queue ? bg.nbricks : 0))));
  TRY(ensure(ctx, ws.brick_start, sizeof(uint32_t) * (size_t)(bg.nbricks + 1)));
  uint32_t* keys[2] = {static_cast<uint32_t*>(ws.keys[0].ptr), static_cast<uint32_t*>(ws.keys[1].ptr)};
  uint32_t* vals[2] = {static_cast<uint32_t*>(ws.vals[0].ptr), static_cast<uint32_t*>(ws.vals[1].ptr)};
  uint32_t* owner = nullptr;
  if (slots) {
    TRY(ensure(ctx, ws.owner, pair_bytes));
    TRY(ensure(ctx, ws.slot_gid, pair_bytes));
    owner = static_cast<uint32_t*>(ws.owner.ptr);
  }
  TRY_HIP(ctx, gve::launch_emit(p->offset, n, box_off, kept, keys[0], vals[0], owner, s, fits));
  if (ec) {
    ec->fits = !async && (int64_t)T <= ec->capacity;
    if (ec->fits && T > 0) {
      TRY_HIP(ctx, hipMemcpyAsync(ec->keys, keys[0], sizeof(uint32_t) * (size_t)T,
                                  hipMemcpyDeviceToDevice, s));
      TRY_HIP(ctx, hipMemcpyAsync(ec->vals, vals[0], sizeof(uint32_t) * (size_t)T,
                                  hipMemcpyDeviceToDevice, s));
    }
  }
  int which = 0;
  TRY_HIP(ctx, gve::radix_sort_pairs(keys, vals, (int64_t)T, bits_for(bg.nbricks), ws.sort_hist.ptr,
                                     &which, s, dn));
  uint32_t* start = static_cast<uint32_t*>(ws.brick_start.ptr);
  TRY_HIP(ctx, gve::launch_ranges(keys[which], (int64_t)T, bg.nbricks, start, s, dn));
  out->sched = gve::Schedule();
  out->sched.kind = sched_of(ctx);
  if (queue) {
    const size_t ob = sizeof(uint32_t) * (size_t)std::max<int64_t>(bg.nbricks, 1);
    for (int b = 0; b < 2; ++b) {
      TRY(ensure(ctx, ws.order_keys[b], ob));
      TRY(ensure(ctx, ws.order_vals[b], ob));
    }
    TRY(ensure(ctx, ws.queue, 256));
    uint32_t* ok[2] = {static_cast<uint32_t*>(ws.order_keys[0].ptr),
                       static_cast<uint32_t*>(ws.order_keys[1].ptr)};
    uint32_t* ov[2] = {static_cast<uint32_t*>(ws.order_vals[0].ptr),
                       static_cast<uint32_t*>(ws.order_vals[1].ptr)};
    TRY_HIP(ctx, gve::launch_order_keys(start, bg.nbricks, ok[0], ov[0], s));
    int ow = 0;
    TRY_HIP(ctx, gve::radix_sort_pairs(ok, ov, bg.nbricks, 6, ws.sort_hist.ptr, &ow, s));
    out->sched.order = ov[ow];
    out->sched.counter = static_cast<uint32_t*>(ws.queue.ptr);
    out->sched.persistent_groups = resident_groups(ctx, bg.Bxy, bg.Bz, bg.waves);
    if (out->sched.persistent_groups <= 0)
      return fail(ctx, GVE_ERR_DEVICE, "occupancy query for the persistent launch failed");
  }
  out->bg = bg;
  out->items = items;
  out->nitems = vol.n;
  out->gid = vals[which];
  out->slot = nullptr;
  if (slots) {
    uint32_t* g = static_cast<uint32_t*>(ws.slot_gid.ptr);
    TRY_HIP(ctx, gve::launch_gather_owner(owner, vals[which], (int64_t)T, g, s, dn));
    out->slot = vals[which];
    out->gid = g;
  }
  out->start = start;
  out->sorted_keys = keys[which];
  out->npairs = async ? -1 : (int64_t)T;
  out->capacity = (int64_t)T;
  out->fits = fits;
  ctx->stats.n_primitives = n;
  ctx->stats.n_bricks = bg.nbricks;
  ctx->stats.bin_brick = bg.Bxy;
  ctx->stats.bin_brick_z = bg.Bz;
  ctx->stats.bin_schedule = sched_of(ctx);
  ctx->stats.bin_waves = bg.waves;
  if (!async) ctx->stats.n_overlaps = (int64_t)T;
  return GVE_OK;
}

// Records of every primitive (the prep kernel alone, no pair list): what the
// dense reference path reads.
gve_status prep_only(gve_ctx* ctx, const gve_params* p, const gve_grid& g) {
  const int64_t off[2] = {0, p->n};
  int64_t nbricks = 0;
  TRY(upload_items(ctx, Vol{&g, off, 1}, brick_xy(ctx), brick_z(ctx), &nbricks));
  TRY(ensure_dloss(ctx));
  unsigned long long* total = pair_total_slots(ctx);
  TRY_HIP(ctx, gve::fill_u64(total, gve::kTotalSlots + 1, ctx->stream));
  gve::BrickGeom bg;
  bg.Bxy = brick_xy(ctx);
  bg.Bz = brick_z(ctx);
  bg.nbricks = nbricks;
  const gve::ItemDesc* items = static_cast<const gve::ItemDesc*>(ctx->ws.items.ptr);
  TRY_HIP(ctx, gve::launch_prep(p->theta, p->n, items, 1, ctx->opt.k, bg, p->rec, p->count, total,
                                ctx->stream));
  return GVE_OK;
}

// The dense path launches one workgroup row per 64 primitives.
gve_status check_dense(const gve_ctx* ctx, const gve_params* p) {
  if ((p->n + 63) / 64 > 65535)
    return fail(ctx, GVE_ERR_UNSUPPORTED, "dense path: at most 65535 * 64 primitives");
  return GVE_OK;
}

gve_status bin(gve_ctx* ctx, const gve_params* p, const gve_grid& g, Binned* out) {
  const int64_t off[2] = {0, p->n};
  return bin_vol(ctx, p, Vol{&g, off, 1}, out);
}

// Launch the fused kernel over a binning (resets the queue counter first).
gve_status fused(gve_ctx* ctx, const gve_params* p, const Binned& bn, const float* d_field,
                 float* part, float* brick_loss, bool vjp) {
  if (bn.sched.kind == gve::kSchedQueue)
    TRY_HIP(ctx, gve::fill_u32(bn.sched.counter, 1, ctx->stream));
  TRY_HIP(ctx, gve::launch_fused(p->rec, bn.gid, bn.start, bn.items, bn.nitems, bn.bg,
                                 ctx->opt.k, d_field, p->acc, p->n, part, bn.slot, brick_loss,
                                 bn.sched, ctx->stream, vjp));
  return GVE_OK;
}

// Loss of every volume of a binning into out[0 .. nitems).
gve_status losses(gve_ctx* ctx, const Binned& bn, const float* brick_loss, double* out) {
  double* dl = static_cast<double*>(ctx->ws.dloss.ptr);
  if (bn.nitems == 1)
    TRY_HIP(ctx, gve::launch_loss_reduce(brick_loss, bn.bg.nbricks, dl + 16, out, ctx->stream));
  else
    TRY_HIP(ctx, gve::launch_item_loss(brick_loss, bn.items, bn.nitems, bn.bg.nbricks, out,
                                       ctx->stream));
  return GVE_OK;
}

gve_status check_ctx_params(const gve_ctx* ctx, const gve_params* p) {
  if (!ctx) return GVE_ERR_INVALID_ARGUMENT;
  if (!p) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "params is NULL");
  const_cast<gve_ctx*>(ctx)->last_error.clear();
  return GVE_OK;
}

gve_status set_device(const gve_ctx* ctx) {
  TRY_HIP(ctx, hipSetDevice(ctx->device));
  return GVE_OK;
}

// Partials buffer for deterministic gradients (nullptr selects atomics).
gve_status partials_for(gve_ctx* ctx, int64_t npairs, float** part) {
  *part = nullptr;
  if (!ctx->opt.deterministic) return GVE_OK;
  TRY(ensure(ctx, ctx->ws.partials, sizeof(float) * 10 * (size_t)(npairs > 0 ? npairs : 1)));
  *part = static_cast<float*>(ctx->ws.partials.ptr);
  return GVE_OK;
}

// Fused forward + squared error + backward into p->acc (or the partials),
// the loss of each volume into d_loss_out[0 .. vol.n).
gve_status loss_and_sums_vol(gve_ctx* ctx, const gve_params* p, const float* d_field, const Vol& vol,
                             double* d_loss_out, float** part_out) {
  Binned bn;
  TRY(bin_vol(ctx, p, vol, &bn));
  TRY(ensure(ctx, ctx->ws.brick_loss, sizeof(float) * (size_t)std::max<int64_t>(bn.bg.nbricks, 1)));
  float* bl = static_cast<float*>(ctx->ws.brick_loss.ptr);
  float* part = nullptr;
  TRY(partials_for(ctx, bn.capacity, &part));
  *part_out = part;
  TRY(fused(ctx, p, bn, d_field, part, bl, false));
  TRY(losses(ctx, bn, bl, d_loss_out));
  return GVE_OK;
}

gve_status loss_and_sums(gve_ctx* ctx, const gve_params* p, const float* d_field, const gve_grid& g,
                         double* d_loss_out, float** part_out) {
  const int64_t off[2] = {0, p->n};
  return loss_and_sums_vol(ctx, p, d_field, Vol{&g, off, 1}, d_loss_out, part_out);
}

unsigned long long* clamp_counter(gve_ctx* ctx) {
  return reinterpret_cast<unsigned long long*>(ctx->ws.dloss.ptr) + 2;
}

}  // namespace

namespace gve {

hipError_t fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t fill_u32(uint32_t* p, int64_t n, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t fill_u64(unsigned long long* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace gve

extern "C" {

const char* gve_status_string(gve_status s) {
  switch (s) {
    case GVE_OK: return "ok";
    case GVE_ERR_INVALID_ARGUMENT: return "invalid argument";
    case GVE_ERR_BUDGET_INFEASIBLE: return "budget infeasible";
    case GVE_ERR_OUT_OF_MEMORY: return "out of device memory";
    case GVE_ERR_DEVICE: return "device error";
    case GVE_ERR_NUMERIC: return "non-finite value";
    case GVE_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* gve_last_error(const gve_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

gve_status gve_default_options(gve_options* opt) {
  if (!opt) return GVE_ERR_INVALID_ARGUMENT;
  opt->k = 3.0f;
  opt->brick = 8;
  opt->lr = 8e-3f;
  opt->beta1 = 0.9f;
  opt->beta2 = 0.999f;
  opt->eps = 1e-8f;
  opt->ell_min = -INFINITY;
  opt->ell_max = INFINITY;
  opt->brick_z = 32;
  opt->schedule = GVE_SCHED_XCD;
  opt->deterministic = 0;
  opt->brick_waves = 1;
  return GVE_OK;
}

gve_status gve_create(gve_ctx** out, const gve_options* opt, void* hip_stream) {
  if (!out) return GVE_ERR_INVALID_ARGUMENT;
  gve_options o;
  gve_default_options(&o);
  if (opt) o = *opt;
  gve_ctx* ctx = new (std::nothrow) gve_ctx();
  if (!ctx) return GVE_ERR_OUT_OF_MEMORY;
  gve_status st = validate_options(ctx, o);
  if (st != GVE_OK) {
    delete ctx;
    return st;
  }
  ctx->opt = o;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&ctx->device) != hipSuccess || hipHostMalloc(&ctx->ws.h_pinned, 512) != hipSuccess) {
    delete ctx;
    return GVE_ERR_DEVICE;
  }
  resolve_scratch(ctx->device);
  *out = ctx;
  return GVE_OK;
}

gve_status gve_destroy(gve_ctx* ctx) {
  if (!ctx) return GVE_ERR_INVALID_ARGUMENT;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  auto& ws = ctx->ws;
  Scratch* all[] = {&ws.keys[0], &ws.keys[1], &ws.vals[0], &ws.vals[1], &ws.brick_start,
                    &ws.brick_loss, &ws.scan_tmp, &ws.sort_hist, &ws.dloss, &ws.clamp_count,
                    &ws.grad_tmp, &ws.alloc, &ws.voxf, &ws.partials, &ws.mlp,
                    &ws.sat, &ws.feat, &ws.theta_base, &ws.items, &ws.order_keys[0],
                    &ws.order_keys[1], &ws.order_vals[0], &ws.order_vals[1], &ws.queue,
                    &ws.p_cls, &ws.p_pts, &ws.p_acc, &ws.p_coef, &ws.p_keys[0], &ws.p_keys[1],
                    &ws.p_idx[0], &ws.p_idx[1], &ws.p_start, &ws.p_loss, &ws.dense, &ws.snap,
                    &ws.box_off, &ws.owner, &ws.slot_gid};
  static_assert(sizeof(all) / sizeof(all[0]) * sizeof(Scratch) + sizeof(void*) ==
                    sizeof(gve::Workspace),
                "every scratch buffer of the workspace is freed");
  for (Scratch* s : all)
    if (s->ptr) hipFree(s->ptr);
  if (ws.h_pinned) hipHostFree(ws.h_pinned);
  for (hipEvent_t e : ctx->events) hipEventDestroy(e);
  delete ctx;
  return GVE_OK;
}

gve_status gve_set_options(gve_ctx* ctx, const gve_options* opt) {
  if (!ctx || !opt) return GVE_ERR_INVALID_ARGUMENT;
  TRY(validate_options(ctx, *opt));
  ctx->opt = *opt;
  return GVE_OK;
}

gve_status gve_get_options(const gve_ctx* ctx, gve_options* opt) {
  if (!ctx || !opt) return GVE_ERR_INVALID_ARGUMENT;
  *opt = ctx->opt;
  return GVE_OK;
}

gve_status gve_params_create(gve_ctx* ctx, int64_t n, gve_params** out) {
  if (!ctx || !out) return GVE_ERR_INVALID_ARGUMENT;
  if (n < 1 || n >= ((int64_t)1 << 31))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "primitive count must be in [1, 2^31)");
  TRY(set_device(ctx));
  gve_params* p = new (std::nothrow) gve_params();
  if (!p) return GVE_ERR_OUT_OF_MEMORY;
  p->n = n;
  p->device = ctx->device;
  const size_t f11 = sizeof(float) * 11 * (size_t)n;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMalloc(&p->theta, f11);
  if (e == hipSuccess) e = hipMalloc(&p->m, f11);
  if (e == hipSuccess) e = hipMalloc(&p->v, f11);
  if (e == hipSuccess) e = hipMalloc(&p->acc, sizeof(float) * gve::kAccStride * (size_t)n);
  if (e == hipSuccess) e = hipMalloc(&p->rec, gve::record_bytes(n));
  if (e == hipSuccess) e = hipMalloc(&p->count, sizeof(uint32_t) * (size_t)n);
  if (e == hipSuccess) e = hipMalloc(&p->offset, sizeof(uint32_t) * (size_t)(n + 1));
  if (e == hipSuccess) e = gve::fill_f32(p->theta, 11 * n, 0.0f, ctx->stream);
  if (e == hipSuccess) e = gve::fill_f32(p->m, 11 * n, 0.0f, ctx->stream);
  if (e == hipSuccess) e = gve::fill_f32(p->v, 11 * n, 0.0f, ctx->stream);
  if (e == hipSuccess) e = gve::fill_f32(p->acc, gve::kAccStride * n, 0.0f, ctx->stream);
  if (e != hipSuccess) {
    gve_params_destroy(p);
    return from_hip(ctx, e, "gve_params_create");
  }
  *out = p;
  return GVE_OK;
}

gve_status gve_params_destroy(gve_params* p) {
  if (!p) return GVE_ERR_INVALID_ARGUMENT;
  hipSetDevice(p->device);
  hipDeviceSynchronize();
  void* bufs[] = {p->theta, p->m, p->v, p->acc, p->rec, p->count, p->offset};
  for (void* b : bufs)
    if (b) hipFree(b);
  delete p;
  return GVE_OK;
}

gve_status gve_params_size(const gve_params* p, int64_t* n) {
  if (!p || !n) return GVE_ERR_INVALID_ARGUMENT;
  *n = p->n;
  return GVE_OK;
}

gve_status gve_params_reset_adam(gve_ctx* ctx, gve_params* p) {
  TRY(check_ctx_params(ctx, p));
  TRY(set_device(ctx));
  TRY_HIP(ctx, gve::fill_f32(p->m, 11 * p->n, 0.0f, ctx->stream));
  TRY_HIP(ctx, gve::fill_f32(p->v, 11 * p->n, 0.0f, ctx->stream));
  p->t = 0;
  return GVE_OK;
}

gve_status gve_params_upload(gve_ctx* ctx, gve_params* p, const float* h_soa) {
  TRY(check_ctx_params(ctx, p));
  if (!h_soa) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "h_soa is NULL");
  TRY(set_device(ctx));
  TRY_HIP(ctx, hipMemcpyAsync(p->theta, h_soa, sizeof(float) * 11 * (size_t)p->n,
                              hipMemcpyHostToDevice, ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return gve_params_reset_adam(ctx, p);
}

gve_status gve_params_copy_from_device(gve_ctx* ctx, gve_params* p, const float* d_soa) {
  TRY(check_ctx_params(ctx, p));
  if (!d_soa) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_soa is NULL");
  TRY(set_device(ctx));
  TRY_HIP(ctx, hipMemcpyAsync(p->theta, d_soa, sizeof(float) * 11 * (size_t)p->n,
                              hipMemcpyDeviceToDevice, ctx->stream));
  return gve_params_reset_adam(ctx, p);
}

gve_status gve_params_download(gve_ctx* ctx, const gve_params* p, float* h_soa) {
  TRY(check_ctx_params(ctx, p));
  if (!h_soa) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "h_soa is NULL");
  TRY(set_device(ctx));
  TRY_HIP(ctx, hipMemcpyAsync(h_soa, p->theta, sizeof(float) * 11 * (size_t)p->n,
                              hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return GVE_OK;
}

gve_status gve_params_device(gve_params* p, float** d_soa) {
  if (!p || !d_soa) return GVE_ERR_INVALID_ARGUMENT;
  *d_soa = p->theta;
  return GVE_OK;
}

gve_status gve_params_adam_state(gve_params* p, float** d_m, float** d_v, int64_t* t) {
  if (!p) return GVE_ERR_INVALID_ARGUMENT;
  if (d_m) *d_m = p->m;
  if (d_v) *d_v = p->v;
  if (t) *t = p->t;
  return GVE_OK;
}

gve_status gve_params_set_step(gve_params* p, int64_t t) {
  if (!p || t < 0) return GVE_ERR_INVALID_ARGUMENT;
  p->t = t;
  return GVE_OK;
}

gve_status gve_evaluate(gve_ctx* ctx, const gve_params* p, gve_grid g, float* d_out) {
  TRY(check_ctx_params(ctx, p));
  if (!d_out) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_out is NULL");
  TRY(validate_grid(ctx, g));
  TRY(set_device(ctx));
  Binned bn;
  TRY(bin(ctx, p, g, &bn));
  TRY_HIP(ctx, gve::launch_forward(p->rec, bn.gid, bn.start, bn.items, bn.nitems, bn.bg,
                                   ctx->opt.k, d_out, bn.sched, ctx->stream));
  return GVE_OK;
}

gve_status gve_loss_grad(gve_ctx* ctx, const gve_params* p, const float* d_field, gve_grid g,
                         float* d_grad, double* h_loss) {
  TRY(check_ctx_params(ctx, p));
  if (!d_field) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_field is NULL");
  TRY(validate_grid(ctx, g));
  TRY(set_device(ctx));
  gve_params* pm = const_cast<gve_params*>(p);
  TRY(ensure_dloss(ctx));
  {
    // the allocation-free path never tunes (tuning allocates)
    const int64_t off[2] = {0, p->n};
    TRY(select_auto(ctx, p, d_field, Vol{&g, off, 1}, ctx->arena_base == nullptr));
  }
  TRY_HIP(ctx, gve::fill_f32(pm->acc, gve::kAccStride * p->n, 0.0f, ctx->stream));
  double* dl = static_cast<double*>(ctx->ws.dloss.ptr);
  float* part = nullptr;
  TRY(loss_and_sums(ctx, p, d_field, g, dl, &part));
  if (d_grad) {
    TRY_HIP(ctx, gve::launch_update(0, pm->theta, pm->m, pm->v, pm->acc, part, p->offset, nullptr,
                                    d_grad, p->n, p->t, ctx->opt, nullptr, ctx->stream));
  } else {
    TRY_HIP(ctx, gve::fill_f32(pm->acc, gve::kAccStride * p->n, 0.0f, ctx->stream));
  }
  if (h_loss) {
    TRY_HIP(ctx, hipMemcpyAsync(ctx->ws.h_pinned, dl, sizeof(double), hipMemcpyDeviceToHost,
                                ctx->stream));
    TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *h_loss = *static_cast<double*>(ctx->ws.h_pinned);
    ctx->stats.last_loss = *h_loss;
    if (!std::isfinite(*h_loss)) return fail(ctx, GVE_ERR_NUMERIC, "loss is not finite");
  }
  return GVE_OK;
}

namespace {

// For the duration of one allocation-free call: the context works on an empty
// workspace whose buffers are carved from the device's static scratch (the
// host staging buffer is shared), with its own host copy of the volume
// descriptors; the context's own workspace and descriptors are restored on
// every exit.
struct StaticScope {
  gve_ctx* ctx;
  gve::Workspace saved;
  std::vector<gve::ItemDesc> saved_items;
  StaticScope(gve_ctx* c, void* base) : ctx(c), saved(c->ws) {
    saved_items.swap(ctx->items_host);
    gve::Workspace fresh;
    fresh.h_pinned = saved.h_pinned;
    ctx->ws = fresh;
    ctx->arena_base = static_cast<char*>(base);
    ctx->arena_cap = kStaticScratchBytes;
    ctx->arena_used = 0;
  }
  ~StaticScope() {
    ctx->ws = saved;
    ctx->items_host.swap(saved_items);
    ctx->arena_base = nullptr;
    ctx->arena_cap = ctx->arena_used = 0;
  }
};

}  // namespace

gve_status gve_loss_grad_static(gve_ctx* ctx, const gve_params* p, const float* d_field,
                                gve_grid g, float* d_grad, double* h_loss) {
  TRY(check_ctx_params(ctx, p));
  const auto addr = scratch_address(ctx->device);
  if (!addr.first)
    return from_hip(ctx, addr.second == hipSuccess ? hipErrorInvalidSymbol : addr.second,
                    "static scratch address (hipGetSymbolAddress)");
  StaticScope scope(ctx, addr.first);
  return gve_loss_grad(ctx, p, d_field, g, d_grad, h_loss);
}

gve_status gve_dense_evaluate(gve_ctx* ctx, const gve_params* p, gve_grid g, float* d_out) {
  TRY(check_ctx_params(ctx, p));
  if (!d_out) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_out is NULL");
  TRY(validate_grid(ctx, g));
  TRY(check_dense(ctx, p));
  TRY(set_device(ctx));
  TRY(prep_only(ctx, p, g));
  TRY_HIP(ctx, gve::launch_dense_forward(p->rec, p->n, g, ctx->opt.k, nullptr, d_out, nullptr,
                                         ctx->stream));
  return GVE_OK;
}

gve_status gve_dense_loss_grad(gve_ctx* ctx, const gve_params* p, const float* d_field,
                               gve_grid g, float* d_grad, double* h_loss) {
  TRY(check_ctx_params(ctx, p));
  if (!d_field) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_field is NULL");
  TRY(validate_grid(ctx, g));
  TRY(check_dense(ctx, p));
  TRY(set_device(ctx));
  gve_params* pm = const_cast<gve_params*>(p);
  const int64_t M = g.nx * g.ny * g.nz;
  const int64_t nblk = gve::dense_blocks(g);
  TRY(ensure(ctx, ctx->ws.dense, sizeof(float) * (size_t)M));
  TRY(ensure(ctx, ctx->ws.brick_loss, sizeof(float) * (size_t)nblk));
  TRY(prep_only(ctx, p, g));
  float* resid = static_cast<float*>(ctx->ws.dense.ptr);
  float* bl = static_cast<float*>(ctx->ws.brick_loss.ptr);
  double* dl = static_cast<double*>(ctx->ws.dloss.ptr);
  TRY_HIP(ctx, gve::launch_dense_forward(p->rec, p->n, g, ctx->opt.k, d_field, resid, bl,
                                         ctx->stream));
  TRY_HIP(ctx, gve::launch_loss_reduce(bl, nblk, dl + 16, dl, ctx->stream));
  if (d_grad) {
    TRY_HIP(ctx, gve::fill_f32(pm->acc, gve::kAccStride * p->n, 0.0f, ctx->stream));
    TRY_HIP(ctx, gve::launch_dense_backward(p->rec, p->n, g, ctx->opt.k, resid, pm->acc,
                                            ctx->stream));
    TRY_HIP(ctx, gve::launch_update(0, pm->theta, pm->m, pm->v, pm->acc, nullptr, p->offset,
                                    nullptr, d_grad, p->n, p->t, ctx->opt, nullptr, ctx->stream));
  }
  if (h_loss) {
    TRY_HIP(ctx, hipMemcpyAsync(ctx->ws.h_pinned, dl, sizeof(double), hipMemcpyDeviceToHost,
                                ctx->stream));
    TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *h_loss = *static_cast<double*>(ctx->ws.h_pinned);
    ctx->stats.last_loss = *h_loss;
    if (!std::isfinite(*h_loss)) return fail(ctx, GVE_ERR_NUMERIC, "loss is not finite");
  }
  return GVE_OK;
}

gve_status gve_vjp(gve_ctx* ctx, const gve_params* p, const float* d_upstream, gve_grid g,
                   float* d_grad) {
  TRY(check_ctx_params(ctx, p));
  if (!d_upstream || !d_grad)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_upstream and d_grad are required");
  TRY(validate_grid(ctx, g));
  TRY(set_device(ctx));
  TRY(ensure_dloss(ctx));
  gve_params* pm = const_cast<gve_params*>(p);
  Binned bn;
  TRY(bin(ctx, p, g, &bn));
  TRY(ensure(ctx, ctx->ws.brick_loss, sizeof(float) * (size_t)std::max<int64_t>(bn.bg.nbricks, 1)));
  float* part = nullptr;
  TRY(partials_for(ctx, bn.capacity, &part));
  if (!part) TRY_HIP(ctx, gve::fill_f32(pm->acc, gve::kAccStride * p->n, 0.0f, ctx->stream));
  TRY(fused(ctx, p, bn, d_upstream, part, static_cast<float*>(ctx->ws.brick_loss.ptr), true));
  TRY_HIP(ctx, gve::launch_update(0, pm->theta, pm->m, pm->v, pm->acc, part, p->offset, nullptr,
                                  d_grad, p->n, p->t, ctx->opt, nullptr, ctx->stream));
  return GVE_OK;
}

gve_status gve_adam_step(gve_ctx* ctx, gve_params* p, const float* d_grad) {
  TRY(check_ctx_params(ctx, p));
  if (!d_grad) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_grad is NULL");
  TRY(set_device(ctx));
  TRY(ensure_dloss(ctx));
  p->t += 1;
  TRY_HIP(ctx, gve::launch_update(2, p->theta, p->m, p->v, p->acc, nullptr, nullptr, d_grad,
                                  nullptr, p->n, p->t,
                                  ctx->opt, clamp_counter(ctx), ctx->stream));
  ctx->stats.iterations = p->t;
  return GVE_OK;
}

namespace {

struct ExportHeader {
  char magic[4];
  uint32_t version;
  int64_t n;
  int64_t grid[6];
  float k, vmin, vmax, pad;
};
static_assert(sizeof(ExportHeader) <= 256, "export header");
constexpr int64_t kMaxRecords = (int64_t)1 << 40;  // keeps every size product in range
constexpr size_t kLutOffset = 256;  // 256 RGBA float32 = 4096 bytes
static_assert(kLutOffset + 4096 <= GVE_EXPORT_HEADER, "export header size");

struct CheckpointHeader {
  char magic[4];
  uint32_t version;
  int64_t n;
  int64_t t;
  double elapsed;
};

}  // namespace

size_t gve_export_size(int64_t n) { return GVE_EXPORT_HEADER + 48 * (size_t)(n > 0 ? n : 0); }

gve_status gve_export(gve_ctx* ctx, const gve_params* p, gve_grid g, float vmin, float vmax,
                      void* h_buf, size_t buf_bytes) {
  TRY(check_ctx_params(ctx, p));
  if (!h_buf || buf_bytes < gve_export_size(p->n))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "buffer smaller than gve_export_size(n)");
  TRY(set_device(ctx));
  const int64_t n = p->n;
  std::vector<float> theta((size_t)11 * n);
  TRY_HIP(ctx, hipMemcpyAsync(theta.data(), p->theta, sizeof(float) * theta.size(),
                              hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  char* out = static_cast<char*>(h_buf);
  std::memset(out, 0, GVE_EXPORT_HEADER);
  ExportHeader h{};
  std::memcpy(h.magic, "GVE1", 4);
  h.version = 1;
  h.n = n;
  const int64_t gv[6] = {g.nx, g.ny, g.nz, g.x0, g.y0, g.z0};
  for (int i = 0; i < 6; ++i) h.grid[i] = gv[i];
  h.k = ctx->opt.k;
  h.vmin = vmin;
  h.vmax = vmax;
  std::memcpy(out, &h, sizeof h);
  float lut[1024];
  for (int i = 0; i < 256; ++i) {
    const float v = (float)i / 255.0f;
    lut[4 * i + 0] = v; lut[4 * i + 1] = v; lut[4 * i + 2] = v; lut[4 * i + 3] = v;
  }
  std::memcpy(out + kLutOffset, lut, sizeof lut);
  // the caller's buffer need not be float-aligned: build records, then copy
  std::vector<float> rec((size_t)12 * n);
  for (int64_t i = 0; i < n; ++i) {
    float* r = rec.data() + 12 * i;
    r[0] = theta[0 * n + i]; r[1] = theta[1 * n + i]; r[2] = theta[2 * n + i];
    r[3] = theta[7 * n + i]; r[4] = theta[8 * n + i]; r[5] = theta[9 * n + i];
    r[6] = theta[3 * n + i]; r[7] = theta[4 * n + i]; r[8] = theta[5 * n + i];
    r[9] = theta[6 * n + i];
    r[10] = theta[10 * n + i];  // scalar attribute a = c
    r[11] = 1.0f;               // weight w
  }
  std::memcpy(out + GVE_EXPORT_HEADER, rec.data(), sizeof(float) * rec.size());
  return GVE_OK;
}

gve_status gve_import(gve_ctx* ctx, const void* h_buf, size_t buf_bytes, gve_params** out,
                      gve_grid* g_out) {
  if (!ctx || !out) return GVE_ERR_INVALID_ARGUMENT;
  ctx->last_error.clear();
  if (!h_buf || buf_bytes < GVE_EXPORT_HEADER)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "buffer shorter than the export header");
  ExportHeader h;
  std::memcpy(&h, h_buf, sizeof h);
  if (std::memcmp(h.magic, "GVE1", 4) != 0 || h.version != 1 || h.n < 1 || h.n > kMaxRecords ||
      buf_bytes < gve_export_size(h.n))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "not a version-1 export of the stated size");
  const int64_t n = h.n;
  std::vector<float> rec((size_t)12 * n);
  std::memcpy(rec.data(), static_cast<const char*>(h_buf) + GVE_EXPORT_HEADER,
              sizeof(float) * rec.size());
  std::vector<float> theta((size_t)11 * n);
  for (int64_t i = 0; i < n; ++i) {
    const float* r = rec.data() + 12 * i;
    theta[0 * n + i] = r[0]; theta[1 * n + i] = r[1]; theta[2 * n + i] = r[2];
    theta[7 * n + i] = r[3]; theta[8 * n + i] = r[4]; theta[9 * n + i] = r[5];
    theta[3 * n + i] = r[6]; theta[4 * n + i] = r[7]; theta[5 * n + i] = r[8];
    theta[6 * n + i] = r[9];
    theta[10 * n + i] = r[10] * r[11];
  }
  gve_params* p = nullptr;
  TRY(gve_params_create(ctx, n, &p));
  const gve_status st = gve_params_upload(ctx, p, theta.data());
  if (st != GVE_OK) {
    gve_params_destroy(p);
    return st;
  }
  if (g_out) *g_out = gve_grid{h.grid[0], h.grid[1], h.grid[2], h.grid[3], h.grid[4], h.grid[5]};
  *out = p;
  return GVE_OK;
}

size_t gve_checkpoint_size(int64_t n) {
  return sizeof(CheckpointHeader) + 3 * 11 * sizeof(float) * (size_t)(n > 0 ? n : 0);
}

gve_status gve_checkpoint_save(gve_ctx* ctx, const gve_params* p, double elapsed_s, void* h_buf,
                               size_t buf_bytes) {
  TRY(check_ctx_params(ctx, p));
  if (!h_buf || buf_bytes < gve_checkpoint_size(p->n))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "buffer smaller than gve_checkpoint_size(n)");
  TRY(set_device(ctx));
  CheckpointHeader h{};
  std::memcpy(h.magic, "GVC1", 4);
  h.version = 1;
  h.n = p->n;
  h.t = p->t;
  h.elapsed = elapsed_s;
  char* out = static_cast<char*>(h_buf);
  std::memcpy(out, &h, sizeof h);
  const size_t block = 11 * sizeof(float) * (size_t)p->n;
  char* body = out + sizeof h;
  TRY_HIP(ctx, hipMemcpyAsync(body, p->theta, block, hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(ctx, hipMemcpyAsync(body + block, p->m, block, hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(ctx, hipMemcpyAsync(body + 2 * block, p->v, block, hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return GVE_OK;
}

gve_status gve_checkpoint_load(gve_ctx* ctx, const void* h_buf, size_t buf_bytes,
                               gve_params** out, double* elapsed_s) {
  if (!ctx || !out) return GVE_ERR_INVALID_ARGUMENT;
  ctx->last_error.clear();
  if (!h_buf || buf_bytes < sizeof(CheckpointHeader))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "buffer shorter than the checkpoint header");
  CheckpointHeader h;
  std::memcpy(&h, h_buf, sizeof h);
  if (std::memcmp(h.magic, "GVC1", 4) != 0 || h.version != 1 || h.n < 1 || h.n > kMaxRecords ||
      h.t < 0 ||
      buf_bytes < gve_checkpoint_size(h.n))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "not a version-1 checkpoint of the stated size");
  TRY(set_device(ctx));
  gve_params* p = nullptr;
  TRY(gve_params_create(ctx, h.n, &p));
  const size_t block = 11 * sizeof(float) * (size_t)h.n;
  const char* body = static_cast<const char*>(h_buf) + sizeof h;
  hipError_t e = hipMemcpyAsync(p->theta, body, block, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(p->m, body + block, block, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->v, body + 2 * block, block, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    gve_params_destroy(p);
    return from_hip(ctx, e, "gve_checkpoint_load");
  }
  p->t = h.t;
  if (elapsed_s) *elapsed_s = h.elapsed;
  *out = p;
  return GVE_OK;
}

gve_status gve_set_timing(gve_ctx* ctx, int32_t enable) {
  if (!ctx) return GVE_ERR_INVALID_ARGUMENT;
  ctx->timing = enable != 0;
  return GVE_OK;
}

gve_status gve_probe(gve_ctx* ctx, gve_probe_rates* h_out) {
  if (!ctx) return GVE_ERR_INVALID_ARGUMENT;
  ctx->last_error.clear();
  if (!h_out) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "h_out is NULL");
  TRY(set_device(ctx));
  const int64_t n = (int64_t)1 << 28;  // floats: 1 GiB
  float* buf = nullptr;
  if (hipMalloc(&buf, sizeof(float) * (size_t)n) != hipSuccess)
    return fail(ctx, GVE_ERR_OUT_OF_MEMORY, "probe buffer (1 GiB)");
  struct Free {
    float* p;
    ~Free() { hipFree(p); }
  } guard{buf};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TRY_HIP(ctx, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(ctx, GVE_ERR_DEVICE, "hipEventCreate");
  }
  struct Events {
    hipEvent_t a, b;
    ~Events() {
      hipEventDestroy(a);
      hipEventDestroy(b);
    }
  } events{e0, e1};
  hipStream_t s = ctx->stream;
  // 8 waves per SIMD on 256 CUs: 2,048 blocks of 4 waves
  const int blocks = 2048;
  const double threads = (double)blocks * gve::probe_threads();
  const double chains = gve::probe_chains();
  auto timed = [&](int kind, int64_t len, int iters, int nblocks, double* ms) -> gve_status {
    TRY_HIP(ctx, gve::launch_probe(kind, buf, len, iters, nblocks, s));  // warm-up
    std::vector<float> t;
    for (int r = 0; r < 5; ++r) {
      TRY_HIP(ctx, hipEventRecord(e0, s));
      TRY_HIP(ctx, gve::launch_probe(kind, buf, len, iters, nblocks, s));
      TRY_HIP(ctx, hipEventRecord(e1, s));
      TRY_HIP(ctx, hipEventSynchronize(e1));
      float v = 0.0f;
      TRY_HIP(ctx, hipEventElapsedTime(&v, e0, e1));
      t.push_back(v);
    }
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return GVE_OK;
  };
  TRY_HIP(ctx, hipMemsetAsync(buf, 0, sizeof(float) * (size_t)n, s));
  double ms = 0.0;
  const int it_fma = 16384, it_exp = 4096, it_atomic = 256;
  TRY(timed(gve::kProbeFma, n, it_fma, blocks, &ms));
  h_out->fma_flops_per_s = 2.0 * chains * it_fma * threads / (ms * 1e-3);
  TRY(timed(gve::kProbeExp, n, it_exp, blocks, &ms));
  h_out->exp_per_s = chains * it_exp * threads / (ms * 1e-3);
  TRY(timed(gve::kProbeCopy, n, 1, blocks * 4, &ms));
  h_out->copy_bytes_per_s = (double)sizeof(float) * (double)n / (ms * 1e-3);
  const int64_t lines = (int64_t)1 << 20;
  TRY_HIP(ctx, gve::fill_f32(buf, gve::kAccStride * lines, 0.0f, s));
  TRY(timed(gve::kProbeAtomic, gve::kAccStride * lines, it_atomic, blocks, &ms));
  h_out->atomic_instr_per_s = (threads / 64.0) * it_atomic / (ms * 1e-3);
  return GVE_OK;
}

gve_status gve_count_pairs(gve_ctx* ctx, const gve_params* p, gve_grid g, int64_t* h_in_support,
                           int64_t* h_candidates) {
  TRY(check_ctx_params(ctx, p));
  if (!h_in_support || !h_candidates)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "output pointers are required");
  TRY(validate_grid(ctx, g));
  TRY(set_device(ctx));
  Binned bn;
  TRY(bin(ctx, p, g, &bn));
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(ctx->ws.dloss.ptr) + 4;
  TRY_HIP(ctx, gve::fill_u64(cnt, 3, ctx->stream));
  TRY_HIP(ctx, gve::launch_count(p->rec, bn.gid, bn.start, bn.items, bn.nitems, bn.bg, ctx->opt.k,
                                 cnt, ctx->stream));
  TRY_HIP(ctx, hipMemcpyAsync(ctx->ws.h_pinned, cnt, 24, hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const unsigned long long* hc = static_cast<unsigned long long*>(ctx->ws.h_pinned);
  *h_in_support = (int64_t)hc[0];
  *h_candidates = (int64_t)hc[1];
  ctx->stats.n_in_support = (int64_t)hc[0];
  ctx->stats.n_candidates = (int64_t)hc[1];
  ctx->stats.n_atomics = (int64_t)hc[2];
  return GVE_OK;
}

gve_status gve_bin_pairs(gve_ctx* ctx, const gve_params* p, gve_grid g, uint32_t* d_emit_keys,
                         uint32_t* d_emit_vals, uint32_t* d_keys, uint32_t* d_vals,
                         uint32_t* d_brick_start, int64_t capacity, int64_t* h_npairs,
                         int64_t* h_nbricks) {
  TRY(check_ctx_params(ctx, p));
  if (!h_npairs || !h_nbricks)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "h_npairs and h_nbricks are required");
  const bool copy = d_emit_keys && d_emit_vals && d_keys && d_vals && d_brick_start;
  if (copy && capacity < 0) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "capacity must be >= 0");
  TRY(validate_grid(ctx, g));
  TRY(set_device(ctx));
  const int64_t off[2] = {0, p->n};
  EmitCopy ec;
  ec.keys = d_emit_keys;
  ec.vals = d_emit_vals;
  ec.capacity = copy ? capacity : -1;
  Binned bn;
  TRY(bin_vol(ctx, p, Vol{&g, off, 1}, &bn, &ec));
  if (copy && ec.fits) {
    hipStream_t s = ctx->stream;
    const size_t T = (size_t)bn.npairs;
    if (T > 0) {
      TRY_HIP(ctx, hipMemcpyAsync(d_keys, bn.sorted_keys, sizeof(uint32_t) * T,
                                  hipMemcpyDeviceToDevice, s));
      TRY_HIP(ctx, hipMemcpyAsync(d_vals, bn.slot ? bn.slot : bn.gid, sizeof(uint32_t) * T,
                                  hipMemcpyDeviceToDevice, s));
    }
    TRY_HIP(ctx, hipMemcpyAsync(d_brick_start, bn.start,
                                sizeof(uint32_t) * (size_t)(bn.bg.nbricks + 1),
                                hipMemcpyDeviceToDevice, s));
  }
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *h_npairs = bn.npairs;
  *h_nbricks = bn.bg.nbricks;
  if (copy && !ec.fits)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "capacity is smaller than the pair count");
  return GVE_OK;
}

namespace {

// Capacity of the asynchronous binning from a box pair total: a quarter
// more, so that the primitives can grow for many iterations before a
// binning no longer fits.
int64_t pair_capacity(int64_t box_total) { return box_total + box_total / 4 + 4096; }

// Restart point of a refinement (parameters, Adam moments and the clamp and
// non-finite counters), taken before its first asynchronously binned
// iteration.
gve_status snapshot(gve_ctx* ctx, gve_params* p, bool save) {
  const size_t f11 = sizeof(float) * 11 * (size_t)p->n;
  TRY(ensure(ctx, ctx->ws.snap, 3 * f11 + 64));
  char* sp = static_cast<char*>(ctx->ws.snap.ptr);
  void* dev[3] = {p->theta, p->m, p->v};
  for (int a = 0; a < 3; ++a) {
    void* dst = save ? (void*)(sp + a * f11) : dev[a];
    const void* src = save ? (const void*)dev[a] : (const void*)(sp + a * f11);
    TRY_HIP(ctx, hipMemcpyAsync(dst, src, f11, hipMemcpyDeviceToDevice, ctx->stream));
  }
  void* cnt = clamp_counter(ctx);  // clamp and non-finite counts, 16 bytes
  TRY_HIP(ctx, hipMemcpyAsync(save ? (void*)(sp + 3 * f11) : cnt,
                              save ? (const void*)cnt : (const void*)(sp + 3 * f11), 16,
                              hipMemcpyDeviceToDevice, ctx->stream));
  return GVE_OK;
}

// Iterations [first, last) of a refinement; asynchronous binning when allowed.
gve_status refine_iters(gve_ctx* ctx, gve_params* p, const float* d_field, const Vol& vol,
                        int32_t first, int32_t last, double* hist, bool timing, bool async) {
  hipStream_t s = ctx->stream;
  for (int32_t it = first; it < last; ++it) {
    hipEvent_t* ev = timing ? &ctx->events[4 * (size_t)it] : nullptr;
    if (timing) TRY_HIP(ctx, hipEventRecord(ev[0], s));
    Binned bn;
    TRY(bin_vol(ctx, p, vol, &bn, nullptr, async));
    if (bn.box_total >= 0) {
      // sized synchronously: later iterations bin into buffers of this capacity
      const bool same = same_items(ctx->pair_cap_items, ctx->items_host);
      ctx->box_cap = same ? std::max(ctx->box_cap, pair_capacity(bn.box_total))
                          : pair_capacity(bn.box_total);
      ctx->pair_cap = same ? std::max(ctx->pair_cap, pair_capacity(bn.npairs))
                           : pair_capacity(bn.npairs);
      ctx->pair_cap_items = ctx->items_host;
    }
    TRY(ensure(ctx, ctx->ws.brick_loss,
               sizeof(float) * (size_t)std::max<int64_t>(bn.bg.nbricks, 1)));
    float* bl = static_cast<float*>(ctx->ws.brick_loss.ptr);
    float* part = nullptr;
    TRY(partials_for(ctx, bn.capacity, &part));
    if (timing) TRY_HIP(ctx, hipEventRecord(ev[1], s));
    TRY(fused(ctx, p, bn, d_field, part, bl, false));
    if (timing) TRY_HIP(ctx, hipEventRecord(ev[2], s));
    TRY(losses(ctx, bn, bl, hist + (size_t)it * vol.n));
    p->t += 1;
    TRY_HIP(ctx, gve::launch_update(1, p->theta, p->m, p->v, p->acc, part, p->offset, nullptr,
                                    nullptr, p->n, p->t, ctx->opt, clamp_counter(ctx), s, bn.fits));
    if (timing) TRY_HIP(ctx, hipEventRecord(ev[3], s));
  }
  return GVE_OK;
}

// End of a refinement: stage timers, clamp and non-finite counts, loss
// history (synchronises).
gve_status refine_finish(gve_ctx* ctx, gve_params* p, const Vol& vol, int32_t iters,
                         const double* hist, double* h_loss_hist, bool timing) {
  ctx->stats.iterations = p->t;
  hipStream_t s = ctx->stream;
  if (timing) {
    TRY_HIP(ctx, hipStreamSynchronize(s));
    double tb = 0, tf = 0, tu = 0;
    for (int32_t it = 0; it < iters; ++it) {
      hipEvent_t* ev = &ctx->events[4 * (size_t)it];
      float a = 0, b = 0, c = 0;
      TRY_HIP(ctx, hipEventElapsedTime(&a, ev[0], ev[1]));
      TRY_HIP(ctx, hipEventElapsedTime(&b, ev[1], ev[2]));
      TRY_HIP(ctx, hipEventElapsedTime(&c, ev[2], ev[3]));
      tb += a; tf += b; tu += c;
    }
    ctx->stats.timed_iterations = iters;
    ctx->stats.ms_bin = tb;
    ctx->stats.ms_fused = tf;
    ctx->stats.ms_update = tu;
  }
  if (iters <= 0) return GVE_OK;
  const size_t nl = (size_t)vol.n * (size_t)iters;
  TRY_HIP(ctx, hipMemcpyAsync(ctx->ws.h_pinned, clamp_counter(ctx),
                              2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  if (h_loss_hist)
    TRY_HIP(ctx, hipMemcpyAsync(h_loss_hist, hist, sizeof(double) * nl, hipMemcpyDeviceToHost, s));
  TRY_HIP(ctx, hipStreamSynchronize(s));
  const unsigned long long* hc = static_cast<unsigned long long*>(ctx->ws.h_pinned);
  ctx->stats.n_clamped = (int64_t)hc[0];
  const int64_t bad_before = ctx->stats.n_nonfinite;
  ctx->stats.n_nonfinite = (int64_t)hc[1];
  if (ctx->stats.n_nonfinite > bad_before)
    return fail(ctx, GVE_ERR_NUMERIC,
                std::to_string(ctx->stats.n_nonfinite - bad_before) +
                    " parameter values became non-finite during refinement");
  if (h_loss_hist) {
    double last = 0.0;
    for (int i = 0; i < vol.n; ++i) last += h_loss_hist[(size_t)(iters - 1) * vol.n + i];
    ctx->stats.last_loss = last;
    for (size_t i = 0; i < nl; ++i)
      if (!std::isfinite(h_loss_hist[i])) return fail(ctx, GVE_ERR_NUMERIC, "loss is not finite");
  }
  return GVE_OK;
}

// `iters` fused iterations over a volume set; h_loss_hist [iters][vol.n].
// The first iteration bins synchronously (sizing the pair buffers); the
// others bin asynchronously into buffers of that capacity, so that an
// iteration queues its kernels without waiting for the device.  They run in
// chunks of kCheckEvery iterations, each from a restart point: should a
// binning of the chunk not fit (the sticky flag, read after the chunk), the
// chunk is rolled back and redone with synchronous binning and larger
// buffers, with the same result.
constexpr int32_t kCheckEvery = 64;

gve_status refine_vol(gve_ctx* ctx, gve_params* p, const float* d_field, const Vol& vol,
                      int32_t iters, double* h_loss_hist) {
  TRY(set_device(ctx));
  TRY(ensure_dloss(ctx));
  if (iters > 0) TRY(select_auto(ctx, p, d_field, vol, true));
  const size_t nl = (size_t)vol.n * (size_t)(iters > 0 ? iters : 1);
  TRY(ensure(ctx, ctx->ws.grad_tmp, sizeof(double) * nl));
  double* hist = static_cast<double*>(ctx->ws.grad_tmp.ptr);
  TRY_HIP(ctx, gve::fill_f32(p->acc, gve::kAccStride * p->n, 0.0f, ctx->stream));
  const bool timing = ctx->timing && iters > 0;
  if (timing) {
    while ((int64_t)ctx->events.size() < 4 * (int64_t)iters) {
      hipEvent_t e;
      TRY_HIP(ctx, hipEventCreate(&e));
      ctx->events.push_back(e);
    }
  }
  hipStream_t s = ctx->stream;
  const int32_t first_async = std::min<int32_t>(1, iters);
  TRY(refine_iters(ctx, p, d_field, vol, 0, first_async, hist, timing, false));
  for (int32_t c0 = first_async; c0 < iters; c0 += kCheckEvery) {
    const int32_t c1 = std::min(iters, c0 + kCheckEvery);
    const int64_t t_restart = p->t;
    TRY(snapshot(ctx, p, true));
    TRY(refine_iters(ctx, p, d_field, vol, c0, c1, hist, timing, true));
    // flags [7]; needs [8], [9]
    TRY_HIP(ctx, hipMemcpyAsync(ctx->ws.h_pinned, fits_flag(ctx), 3 * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, s));
    TRY_HIP(ctx, hipStreamSynchronize(s));
    const unsigned long long* hc = static_cast<unsigned long long*>(ctx->ws.h_pinned);
    if (reinterpret_cast<const uint32_t*>(hc)[1]) {
      TRY_HIP(ctx, gve::fill_u32(sticky_flag(ctx), 1, s));
      TRY(snapshot(ctx, p, false));
      TRY_HIP(ctx, gve::fill_f32(p->acc, gve::kAccStride * p->n, 0.0f, s));
      p->t = t_restart;
      ctx->box_cap = std::max(ctx->box_cap, pair_capacity((int64_t)hc[1]));
      ctx->pair_cap = std::max(ctx->pair_cap, pair_capacity((int64_t)hc[2]));
      ctx->stats.n_resized += 1;
      TRY(refine_iters(ctx, p, d_field, vol, c0, c1, hist, timing, false));
    }
  }
  if (iters > 0) {
    // pair and degenerate-quaternion counts of the last (asynchronous) binning
    unsigned char* hp = static_cast<unsigned char*>(ctx->ws.h_pinned);
    TRY_HIP(ctx, hipMemcpyAsync(hp, p->offset + p->n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    TRY_HIP(ctx, hipMemcpyAsync(hp + 8, pair_total_slots(ctx) + gve::kTotalSlots,
                                sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    TRY_HIP(ctx, hipStreamSynchronize(s));
    ctx->stats.n_overlaps = (int64_t) * reinterpret_cast<const uint32_t*>(hp);
    ctx->stats.n_degenerate_q = (int64_t) * reinterpret_cast<const unsigned long long*>(hp + 8);
  }
  return refine_finish(ctx, p, vol, iters, hist, h_loss_hist, timing);
}

}  // namespace

gve_status gve_refine(gve_ctx* ctx, gve_params* p, const float* d_field, gve_grid g,
                      int32_t iters, double* h_loss_hist) {
  TRY(check_ctx_params(ctx, p));
  if (!d_field) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_field is NULL");
  if (iters < 0) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "iters must be >= 0");
  TRY(validate_grid(ctx, g));
  const int64_t off[2] = {0, p->n};
  return refine_vol(ctx, p, d_field, Vol{&g, off, 1}, iters, h_loss_hist);
}

gve_status gve_normalize(gve_ctx* ctx, float* d_field, int64_t n) {
  if (!ctx) return GVE_ERR_INVALID_ARGUMENT;
  ctx->last_error.clear();
  if (!d_field || n <= 0) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "need a field of n > 0 values");
  TRY(set_device(ctx));
  TRY(ensure(ctx, ctx->ws.alloc, sizeof(float) * gve::normalize_tmp_floats()));
  TRY_HIP(ctx, gve::normalize_field(d_field, n, static_cast<float*>(ctx->ws.alloc.ptr),
                                    ctx->stream));
  return GVE_OK;
}

gve_status gve_allocate(gve_ctx* ctx, const float* d_field, gve_grid g, int64_t budget,
                        uint64_t seed, gve_params** out, gve_alloc_info* info) {
  if (!ctx) return GVE_ERR_INVALID_ARGUMENT;
  ctx->last_error.clear();
  if (!d_field || !out) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_field and out are required");
  if (budget < 1 || budget >= ((int64_t)1 << 31))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "budget must be in [1, 2^31)");
  TRY(validate_grid(ctx, g));
  TRY(set_device(ctx));
  hipStream_t s = ctx->stream;
  const int64_t M = g.nx * g.ny * g.nz;
  const int64_t nb = (int64_t)gve::alloc_block_count(M);
  const int64_t n_det = (int64_t)std::floor(0.55 * (double)budget + 0.5);
  const int64_t n_cov = budget - n_det;
  // carve the allocation scratch
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t o_counts = take(16), o_st = take(48), o_hist = take(256 * 8), o_sb = take(16),
               o_best = take(4096 * 8), o_dot = take(sizeof(double) * gve::alloc_dot_tmp_doubles()),
               o_less = take(4 * (nb + 1)), o_tie = take(4 * (nb + 1)), o_toff = take(4 * (nb + 1)),
               o_take = take(4 * (nb + 1)), o_ooff = take(4 * (nb + 1)), o_det = take(8 * n_det),
               o_cov = take(8 * n_cov), o_j6 = take(6 * sizeof(double) * (size_t)budget);
  TRY(ensure(ctx, ctx->ws.alloc, off));
  TRY(ensure(ctx, ctx->ws.voxf, sizeof(float) * (size_t)M));
  TRY(ensure(ctx, ctx->ws.scan_tmp, gve::scan_tmp_bytes(nb + 1)));
  char* base = static_cast<char*>(ctx->ws.alloc.ptr);
  auto U64 = [&](size_t o) { return reinterpret_cast<unsigned long long*>(base + o); };
  auto U32 = [&](size_t o) { return reinterpret_cast<uint32_t*>(base + o); };
  auto I64 = [&](size_t o) { return reinterpret_cast<int64_t*>(base + o); };
  auto F64 = [&](size_t o) { return reinterpret_cast<double*>(base + o); };
  float* g32 = static_cast<float*>(ctx->ws.voxf.ptr);

  // S1a: gradient magnitude and domain counts; feasibility (Sec. V-B)
  TRY_HIP(ctx, gve::fill_u64(U64(o_counts), 2, s));
  TRY_HIP(ctx, gve::fill_u64(U64(o_hist), 256, s));
  TRY_HIP(ctx, gve::alloc_grad(d_field, g, g32, U64(o_counts), s));
  TRY_HIP(ctx, hipMemcpyAsync(ctx->ws.h_pinned, U64(o_counts), 16, hipMemcpyDeviceToHost, s));
  TRY_HIP(ctx, hipStreamSynchronize(s));
  const int64_t n_occ = (int64_t) static_cast<unsigned long long*>(ctx->ws.h_pinned)[0];
  const int64_t n_el = (int64_t) static_cast<unsigned long long*>(ctx->ws.h_pinned)[1];
  gve_alloc_info inf{};
  inf.n_detail = n_det;
  inf.n_coverage = n_cov;
  inf.n_eligible = n_el;
  inf.n_occupied = n_occ;
  int64_t shortfall = n_det - n_el;
  if (n_cov - n_occ > shortfall) shortfall = n_cov - n_occ;
  if (shortfall > 0) {
    inf.shortfall = shortfall;
    if (info) *info = inf;
    return fail(ctx, GVE_ERR_BUDGET_INFEASIBLE,
                "budget needs " + std::to_string(shortfall) + " more distinct seed voxels");
  }
  // S1b: the two draws and the 99th percentile of |grad V| over V > 0.02
  unsigned long long* st_det = U64(o_st);
  unsigned long long* st_cov = st_det + 2;
  unsigned long long* st_g99 = st_det + 4;
  const int64_t r99 = (int64_t)std::floor(0.99 * (double)(n_occ - 1));
  TRY_HIP(ctx, gve::alloc_set_state(st_det, 0ull, (unsigned long long)n_det, s));
  TRY_HIP(ctx, gve::alloc_set_state(st_cov, 0ull, (unsigned long long)n_cov, s));
  TRY_HIP(ctx, gve::alloc_set_state(st_g99, 0ull, (unsigned long long)(r99 + 1), s));
  int64_t* det = I64(o_det);
  int64_t* cov = I64(o_cov);
  TRY_HIP(ctx, gve::alloc_select(0, d_field, g32, g, seed, st_det, U64(o_hist), U32(o_less),
                                 U32(o_tie), U32(o_toff), U32(o_take), U32(o_ooff),
                                 ctx->ws.scan_tmp.ptr, det, s));
  TRY_HIP(ctx, gve::alloc_select(1, d_field, g32, g, seed, st_cov, U64(o_hist), U32(o_less),
                                 U32(o_tie), U32(o_toff), U32(o_take), U32(o_ooff),
                                 ctx->ws.scan_tmp.ptr, cov, s));
  TRY_HIP(ctx, gve::alloc_select(2, d_field, g32, g, seed, st_g99, U64(o_hist), nullptr, nullptr,
                                 nullptr, nullptr, nullptr, nullptr, nullptr, s));
  gve_params* p = nullptr;
  TRY(gve_params_create(ctx, budget, &p));
  auto cleanup = [&](gve_status st) {
    gve_params_destroy(p);
    return st;
  };
  gve_status st = GVE_OK;
#define TRY_A(call)                                                        \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess) return cleanup(from_hip(ctx, e_, #call));        \
  } while (0)
  TRY_A(gve::alloc_jitter(g, det, cov, n_det, budget, seed, p->theta, s));
  // S1c: group spacing
  double* sb = F64(o_sb);
  TRY_A(gve::alloc_spacing(p->theta, budget, 0, n_det, F64(o_best), sb, s));
  TRY_A(gve::alloc_spacing(p->theta, budget, n_det, n_cov, F64(o_best), sb + 1, s));
  // S1d/S1e: frames, scales, values
  TRY_A(gve::alloc_assemble(d_field, g32, g, det, cov, n_det, budget, sb, st_g99, seed, p->theta,
                            F64(o_j6), s));
  // weights: U = sum a_i G_i on the grid (g32's buffer is free now), kappa
  Binned bn;
  st = bin(ctx, p, g, &bn);
  if (st != GVE_OK) return cleanup(st);
  TRY_A(gve::launch_forward(p->rec, bn.gid, bn.start, bn.items, bn.nitems, bn.bg, ctx->opt.k, g32,
                            bn.sched, s));
  TRY_A(gve::alloc_weights(g32, d_field, M, p->theta + 10 * budget, budget, F64(o_dot), s));
#undef TRY_A
  // report
  double* hp = static_cast<double*>(ctx->ws.h_pinned);
  hipError_t e = hipMemcpyAsync(hp, sb, 16, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hp + 2, F64(o_dot), 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hp + 3, st_g99, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return cleanup(from_hip(ctx, e, "gve_allocate readback"));
  inf.s_base_detail = hp[0];
  inf.s_base_coverage = hp[1];
  inf.kappa = hp[2];
  unsigned long long gb;
  std::memcpy(&gb, hp + 3, 8);
  float g99f;
  const uint32_t gb32 = (uint32_t)gb;
  std::memcpy(&g99f, &gb32, 4);
  inf.g99 = g99f;
  if (info) *info = inf;
  *out = p;
  return GVE_OK;
}

gve_status gve_get_stats(const gve_ctx* ctx, gve_stats* out) {
  if (!ctx || !out) return GVE_ERR_INVALID_ARGUMENT;
  *out = ctx->stats;
  const gve::Workspace& w = ctx->ws;
  const gve::Scratch* all[] = {&w.keys[0], &w.keys[1], &w.vals[0], &w.vals[1], &w.brick_start,
                               &w.brick_loss, &w.scan_tmp, &w.box_off, &w.owner, &w.slot_gid,
                               &w.sort_hist, &w.dloss,
                               &w.clamp_count, &w.grad_tmp, &w.alloc, &w.voxf, &w.partials,
                               &w.mlp, &w.sat, &w.feat, &w.theta_base, &w.items,
                               &w.order_keys[0], &w.order_keys[1], &w.order_vals[0],
                               &w.order_vals[1], &w.queue, &w.p_cls, &w.p_pts, &w.p_acc,
                               &w.p_coef, &w.p_keys[0], &w.p_keys[1], &w.p_idx[0], &w.p_idx[1],
                               &w.p_start, &w.p_loss, &w.dense, &w.snap};
  static_assert(sizeof(all) / sizeof(all[0]) * sizeof(gve::Scratch) + sizeof(void*) ==
                    sizeof(gve::Workspace),
                "every scratch buffer of the workspace is counted");
  int64_t bytes = 0;
  for (const gve::Scratch* s : all) bytes += s->ptr ? (int64_t)s->bytes : 0;
  out->workspace_bytes = bytes;
  return GVE_OK;
}

}  // extern "C"

// ===========================================================================
// Learned warm start
// ===========================================================================

struct gve_mlp {
  int device = 0;
  float* w = nullptr;      // [GVE_MLP_NWEIGHT] float32 master weights
  float* m = nullptr;      // Adam moments
  float* v = nullptr;
  float* stats = nullptr;  // fmean[16] fstd[16] tmean[11] tstd[11]
  int64_t t = 0;
};

namespace {

constexpr int kDin = 16, kDh = 128, kDout = 11;
constexpr int64_t kW1 = 0, kB1 = 2048, kW2 = 2176, kB2 = 18560, kW3 = 18688, kB3 = 20096;
constexpr int64_t kMlpRows = 65536;  // rows per forward / backward chunk
static_assert(kB3 + kDout == GVE_MLP_NWEIGHT, "weight layout");

struct MlpBuf {
  float *Xs, *Ts, *Z1, *H1, *Z2, *H2, *Y, *dY, *grad, *split;
  size_t split_floats;
  double *part, *acc;
};

gve_status mlp_buffers(gve_ctx* ctx, int64_t rows, int64_t nacc, MlpBuf* b) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t r = (size_t)rows;
  const size_t split_floats = (size_t)((rows + 511) / 512) * kDh * kDh;
  const size_t oXs = take(4 * r * kDin), oTs = take(4 * r * kDout), oZ1 = take(4 * r * kDh),
               oH1 = take(4 * r * kDh), oZ2 = take(4 * r * kDh), oH2 = take(4 * r * kDh),
               oY = take(4 * r * kDout), odY = take(4 * r * kDout), og = take(4 * GVE_MLP_NWEIGHT),
               osp = take(4 * split_floats), opart = take(8 * 64), oacc = take(8 * (size_t)nacc);
  TRY(ensure(ctx, ctx->ws.mlp, off));
  char* base = static_cast<char*>(ctx->ws.mlp.ptr);
  auto F32 = [&](size_t o) { return reinterpret_cast<float*>(base + o); };
  b->Xs = F32(oXs); b->Ts = F32(oTs); b->Z1 = F32(oZ1); b->H1 = F32(oH1); b->Z2 = F32(oZ2);
  b->H2 = F32(oH2); b->Y = F32(oY); b->dY = F32(odY); b->grad = F32(og); b->split = F32(osp);
  b->split_floats = split_floats;
  b->part = reinterpret_cast<double*>(base + opart);
  b->acc = reinterpret_cast<double*>(base + oacc);
  return GVE_OK;
}

// Y = network(Xs) for `rows` standardised inputs; activations kept in b.
gve_status mlp_fwd(gve_ctx* ctx, const gve_mlp* m, const float* Xs, int64_t rows, MlpBuf& b,
                   float* Y) {
  hipStream_t s = ctx->stream;
  const int R = (int)rows;
  TRY_HIP(ctx, gve::mlp_gemm(false, true, 1, R, kDh, kDin, Xs, kDin, m->w + kW1, kDin, b.Z1, kDh,
                             m->w + kB1, b.H1, nullptr, 0, s));
  TRY_HIP(ctx, gve::mlp_gemm(false, true, 1, R, kDh, kDh, b.H1, kDh, m->w + kW2, kDh, b.Z2, kDh,
                             m->w + kB2, b.H2, nullptr, 0, s));
  TRY_HIP(ctx, gve::mlp_gemm(false, true, 0, R, kDout, kDh, b.H2, kDh, m->w + kW3, kDh, Y, kDout,
                             m->w + kB3, nullptr, nullptr, 0, s));
  return GVE_OK;
}

// Gradients of the mean squared error into b.grad, given b.dY (= dL/dY).
gve_status mlp_bwd(gve_ctx* ctx, const gve_mlp* m, const float* Xs, int64_t rows, MlpBuf& b) {
  hipStream_t s = ctx->stream;
  const int R = (int)rows;
  float* g = b.grad;
  TRY_HIP(ctx, gve::mlp_gemm(true, false, 0, kDout, kDh, R, b.dY, kDout, b.H2, kDh, g + kW3, kDh,
                             nullptr, nullptr, b.split, b.split_floats, s));
  TRY_HIP(ctx, gve::mlp_colsum(b.dY, R, kDout, g + kB3, s));
  // dH2 reuses H2's buffer after dW3 has consumed it (stream order)
  float* dH2 = b.H2;
  TRY_HIP(ctx, gve::mlp_gemm(false, false, 0, R, kDh, kDout, b.dY, kDout, m->w + kW3, kDh, dH2, kDh,
                             nullptr, nullptr, nullptr, 0, s));
  TRY_HIP(ctx, gve::mlp_gelu_back(dH2, b.Z2, rows * kDh, s));
  TRY_HIP(ctx, gve::mlp_gemm(true, false, 0, kDh, kDh, R, dH2, kDh, b.H1, kDh, g + kW2, kDh,
                             nullptr, nullptr, b.split, b.split_floats, s));
  TRY_HIP(ctx, gve::mlp_colsum(dH2, R, kDh, g + kB2, s));
  float* dH1 = b.H1;
  TRY_HIP(ctx, gve::mlp_gemm(false, false, 0, R, kDh, kDh, dH2, kDh, m->w + kW2, kDh, dH1, kDh,
                             nullptr, nullptr, nullptr, 0, s));
  TRY_HIP(ctx, gve::mlp_gelu_back(dH1, b.Z1, rows * kDh, s));
  TRY_HIP(ctx, gve::mlp_gemm(true, false, 0, kDh, kDin, R, dH1, kDh, Xs, kDin, g + kW1, kDin,
                             nullptr, nullptr, b.split, b.split_floats, s));
  TRY_HIP(ctx, gve::mlp_colsum(dH1, R, kDh, g + kB1, s));
  return GVE_OK;
}

// Loss L of p on the field (forward + fused pass), read back to the host.
gve_status eval_loss(gve_ctx* ctx, const gve_params* p, const float* d_field, const gve_grid& g,
                     double* out) {
  double* dl = static_cast<double*>(ctx->ws.dloss.ptr);
  float* part = nullptr;
  TRY(loss_and_sums(ctx, p, d_field, g, dl, &part));
  if (!part) TRY_HIP(ctx, gve::fill_f32(const_cast<gve_params*>(p)->acc, gve::kAccStride * p->n, 0.0f, ctx->stream));
  TRY_HIP(ctx, hipMemcpyAsync(ctx->ws.h_pinned, dl, sizeof(double), hipMemcpyDeviceToHost,
                              ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *out = *static_cast<double*>(ctx->ws.h_pinned);
  return GVE_OK;
}

}  // namespace

extern "C" {

gve_status gve_mlp_create(gve_ctx* ctx, uint64_t seed, gve_mlp** out) {
  if (!ctx || !out) return GVE_ERR_INVALID_ARGUMENT;
  ctx->last_error.clear();
  TRY(set_device(ctx));
  gve_mlp* m = new (std::nothrow) gve_mlp();
  if (!m) return GVE_ERR_OUT_OF_MEMORY;
  m->device = ctx->device;
  hipError_t e = hipMalloc(&m->w, sizeof(float) * GVE_MLP_NWEIGHT);
  if (e == hipSuccess) e = hipMalloc(&m->m, sizeof(float) * GVE_MLP_NWEIGHT);
  if (e == hipSuccess) e = hipMalloc(&m->v, sizeof(float) * GVE_MLP_NWEIGHT);
  if (e == hipSuccess) e = hipMalloc(&m->stats, sizeof(float) * 54);
  if (e != hipSuccess) {
    gve_mlp_destroy(m);
    return from_hip(ctx, e, "gve_mlp_create");
  }
  std::vector<float> h(GVE_MLP_NFLAT, 0.0f);
  // He-uniform: U(-b, b), b = sqrt(6 / fan_in); uniform from a counter hash
  auto fill = [&](int64_t off, int64_t count, int fan_in, uint64_t stream) {
    const double bnd = std::sqrt(6.0 / fan_in);
    for (int64_t i = 0; i < count; ++i) {
      const uint64_t r = gve::hash_bits(seed, stream, (uint64_t)i);
      const double u = (double)((r >> 11) + 1) * 0x1.0p-53;
      h[off + i] = (float)((2.0 * u - 1.0) * bnd);
    }
  };
  fill(kW1, kB1 - kW1, kDin, 11);
  fill(kW2, kB2 - kW2, kDh, 12);
  fill(kW3, kB3 - kW3, kDh, 13);
  for (int c = 0; c < 16; ++c) h[GVE_MLP_NWEIGHT + 16 + c] = 1.0f;
  for (int c = 0; c < 11; ++c) h[GVE_MLP_NWEIGHT + 32 + 11 + c] = 1.0f;
  *out = m;
  const gve_status st = gve_mlp_import(ctx, m, h.data());
  if (st != GVE_OK) {
    gve_mlp_destroy(m);
    *out = nullptr;
  }
  return st;
}

gve_status gve_mlp_destroy(gve_mlp* m) {
  if (!m) return GVE_ERR_INVALID_ARGUMENT;
  hipSetDevice(m->device);
  hipDeviceSynchronize();
  void* bufs[] = {m->w, m->m, m->v, m->stats};
  for (void* b : bufs)
    if (b) hipFree(b);
  delete m;
  return GVE_OK;
}

gve_status gve_mlp_export(gve_ctx* ctx, const gve_mlp* m, float* h_flat) {
  if (!ctx || !m || !h_flat) return GVE_ERR_INVALID_ARGUMENT;
  TRY(set_device(ctx));
  TRY_HIP(ctx, hipMemcpyAsync(h_flat, m->w, sizeof(float) * GVE_MLP_NWEIGHT,
                              hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(ctx, hipMemcpyAsync(h_flat + GVE_MLP_NWEIGHT, m->stats, sizeof(float) * 54,
                              hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return GVE_OK;
}

gve_status gve_mlp_import(gve_ctx* ctx, gve_mlp* m, const float* h_flat) {
  if (!ctx || !m || !h_flat) return GVE_ERR_INVALID_ARGUMENT;
  TRY(set_device(ctx));
  TRY_HIP(ctx, hipMemcpyAsync(m->w, h_flat, sizeof(float) * GVE_MLP_NWEIGHT,
                              hipMemcpyHostToDevice, ctx->stream));
  TRY_HIP(ctx, hipMemcpyAsync(m->stats, h_flat + GVE_MLP_NWEIGHT, sizeof(float) * 54,
                              hipMemcpyHostToDevice, ctx->stream));
  TRY_HIP(ctx, gve::fill_f32(m->m, GVE_MLP_NWEIGHT, 0.0f, ctx->stream));
  TRY_HIP(ctx, gve::fill_f32(m->v, GVE_MLP_NWEIGHT, 0.0f, ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  m->t = 0;
  return GVE_OK;
}

gve_status gve_mlp_forward(gve_ctx* ctx, const gve_mlp* m, const float* d_X, int64_t n, float* d_Y) {
  if (!ctx || !m) return GVE_ERR_INVALID_ARGUMENT;
  ctx->last_error.clear();
  if (!d_X || !d_Y || n < 1) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "need d_X, d_Y and n >= 1");
  TRY(set_device(ctx));
  MlpBuf b;
  TRY(mlp_buffers(ctx, std::min(n, kMlpRows), 1, &b));
  for (int64_t r0 = 0; r0 < n; r0 += kMlpRows) {
    const int64_t rows = std::min(kMlpRows, n - r0);
    TRY(mlp_fwd(ctx, m, d_X + r0 * kDin, rows, b, d_Y + r0 * kDout));
  }
  return GVE_OK;
}

gve_status gve_mlp_loss_grad(gve_ctx* ctx, const gve_mlp* m, const float* d_X, const float* d_T,
                             int64_t n, float* d_grad, double* h_loss) {
  if (!ctx || !m) return GVE_ERR_INVALID_ARGUMENT;
  ctx->last_error.clear();
  if (!d_X || !d_T || n < 1) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "need d_X, d_T and n >= 1");
  if (n > kMlpRows) return fail(ctx, GVE_ERR_UNSUPPORTED, "at most 65536 rows per call");
  TRY(set_device(ctx));
  MlpBuf b;
  TRY(mlp_buffers(ctx, n, 1, &b));
  hipStream_t s = ctx->stream;
  TRY(mlp_fwd(ctx, m, d_X, n, b, b.Y));
  const double inv = 1.0 / ((double)n * kDout);
  TRY_HIP(ctx, gve::fill_u64(reinterpret_cast<unsigned long long*>(b.acc), 1, s));
  TRY_HIP(ctx, gve::mlp_mse_grad(b.Y, d_T, n * kDout, (float)inv, b.dY, b.part, b.acc, inv, s));
  if (d_grad) {
    TRY(mlp_bwd(ctx, m, d_X, n, b));
    TRY_HIP(ctx, hipMemcpyAsync(d_grad, b.grad, sizeof(float) * GVE_MLP_NWEIGHT,
                                hipMemcpyDeviceToDevice, s));
  }
  if (h_loss) {
    TRY_HIP(ctx, hipMemcpyAsync(ctx->ws.h_pinned, b.acc, 8, hipMemcpyDeviceToHost, s));
    TRY_HIP(ctx, hipStreamSynchronize(s));
    *h_loss = *static_cast<double*>(ctx->ws.h_pinned);
  }
  return GVE_OK;
}

gve_status gve_mlp_train(gve_ctx* ctx, gve_mlp* m, const float* d_X, const float* d_T, int64_t n,
                         int32_t epochs, int32_t batch, float lr, uint64_t seed,
                         double* h_epoch_loss) {
  if (!ctx || !m) return GVE_ERR_INVALID_ARGUMENT;
  ctx->last_error.clear();
  if (!d_X || !d_T || n < 1 || epochs < 0 || batch < 1 || batch > kMlpRows || !(lr >= 0.0f) ||
      n >= ((int64_t)1 << 31))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT,
                "need d_X, d_T, 1 <= n < 2^31, epochs >= 0, 1 <= batch <= 65536, lr >= 0");
  TRY(set_device(ctx));
  hipStream_t s = ctx->stream;
  MlpBuf b;
  TRY(mlp_buffers(ctx, batch, std::max(epochs, 1), &b));
  float* fmean = m->stats;
  float* fstd = m->stats + 16;
  float* tmean = m->stats + 32;
  float* tstd = m->stats + 43;
  TRY_HIP(ctx, gve::mlp_colstats(d_X, n, kDin, fmean, fstd, s));
  TRY_HIP(ctx, gve::mlp_colstats(d_T, n, kDout, tmean, tstd, s));
  TRY_HIP(ctx, gve::fill_u64(reinterpret_cast<unsigned long long*>(b.acc), std::max(epochs, 1), s));
  // shuffle buffers: the pair ping-pong buffers of the binning are reused
  auto& ws = ctx->ws;
  for (int i = 0; i < 2; ++i) {
    TRY(ensure(ctx, ws.keys[i], sizeof(uint32_t) * (size_t)n));
    TRY(ensure(ctx, ws.vals[i], sizeof(uint32_t) * (size_t)n));
  }
  TRY(ensure(ctx, ws.sort_hist, gve::sort_hist_bytes(n)));
  uint32_t* keys[2] = {static_cast<uint32_t*>(ws.keys[0].ptr), static_cast<uint32_t*>(ws.keys[1].ptr)};
  uint32_t* vals[2] = {static_cast<uint32_t*>(ws.vals[0].ptr), static_cast<uint32_t*>(ws.vals[1].ptr)};
  const int64_t nb = (n + batch - 1) / batch;
  for (int32_t ep = 0; ep < epochs; ++ep) {
    TRY_HIP(ctx, gve::mlp_perm_keys(keys[0], vals[0], n, seed, (uint64_t)ep, s));
    int which = 0;
    TRY_HIP(ctx, gve::radix_sort_pairs(keys, vals, n, 32, ws.sort_hist.ptr, &which, s));
    const uint32_t* perm = vals[which];
    for (int64_t bi = 0; bi < nb; ++bi) {
      const int64_t r0 = bi * batch;
      const int64_t rows = std::min((int64_t)batch, n - r0);
      TRY_HIP(ctx, gve::mlp_standardize(d_X, perm + r0, rows, kDin, fmean, fstd, b.Xs, s));
      TRY_HIP(ctx, gve::mlp_standardize(d_T, perm + r0, rows, kDout, tmean, tstd, b.Ts, s));
      TRY(mlp_fwd(ctx, m, b.Xs, rows, b, b.Y));
      const double inv = 1.0 / ((double)rows * kDout);
      TRY_HIP(ctx, gve::mlp_mse_grad(b.Y, b.Ts, rows * kDout, (float)inv, b.dY, b.part, b.acc + ep,
                                     inv / (double)nb, s));
      TRY(mlp_bwd(ctx, m, b.Xs, rows, b));
      m->t += 1;
      TRY_HIP(ctx, gve::mlp_adam(m->w, m->m, m->v, b.grad, GVE_MLP_NWEIGHT, lr, 0.9f, 0.999f, 1e-8f,
                                 m->t, s));
    }
  }
  if (h_epoch_loss && epochs > 0) {
    TRY_HIP(ctx, hipMemcpyAsync(h_epoch_loss, b.acc, sizeof(double) * (size_t)epochs,
                                hipMemcpyDeviceToHost, s));
  }
  TRY_HIP(ctx, hipStreamSynchronize(s));
  return GVE_OK;
}

gve_status gve_features(gve_ctx* ctx, const gve_params* p, const float* d_field, gve_grid g,
                        int64_t n_detail, double g99, float* d_X) {
  TRY(check_ctx_params(ctx, p));
  if (!d_field || !d_X) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_field and d_X are required");
  if (n_detail < 0 || n_detail > p->n || !(g99 >= 0.0))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "need 0 <= n_detail <= n and g99 >= 0");
  TRY(validate_grid(ctx, g));
  TRY(set_device(ctx));
  const int64_t M = g.nx * g.ny * g.nz;
  // summed-area tables of V and V^2, then the primitives' structure tensors
  TRY(ensure(ctx, ctx->ws.sat, sizeof(double) * (2 * (size_t)M + 6 * (size_t)p->n)));
  double* s1 = static_cast<double*>(ctx->ws.sat.ptr);
  double* s2 = s1 + M;
  double* J6 = s2 + M;
  TRY_HIP(ctx, gve::mlp_sat(d_field, g, s1, s2, ctx->stream));
  TRY_HIP(ctx, gve::mlp_features(d_field, p->theta, p->n, n_detail, g, g99, ctx->opt.k, s1, s2, J6,
                                 d_X, ctx->stream));
  return GVE_OK;
}

gve_status gve_targets(gve_ctx* ctx, const gve_params* alloc, const gve_params* refined,
                       float* d_T) {
  TRY(check_ctx_params(ctx, alloc));
  if (!refined || !d_T) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "refined and d_T are required");
  if (refined->n != alloc->n) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "sizes differ");
  TRY(set_device(ctx));
  TRY_HIP(ctx, gve::mlp_targets(alloc->theta, refined->theta, alloc->n, d_T, ctx->stream));
  return GVE_OK;
}

gve_status gve_warmstart(gve_ctx* ctx, const gve_mlp* m, gve_params* p, const float* d_field,
                         gve_grid g, int64_t n_detail, double g99, int32_t* applied,
                         double* h_losses) {
  TRY(check_ctx_params(ctx, p));
  if (!m || !d_field || !applied)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "network, field and applied are required");
  TRY(validate_grid(ctx, g));
  TRY(set_device(ctx));
  hipStream_t s = ctx->stream;
  const int64_t n = p->n;
  TRY(ensure_dloss(ctx));
  TRY(ensure(ctx, ctx->ws.feat, sizeof(float) * (size_t)n * (kDin + kDout)));
  TRY(ensure(ctx, ctx->ws.theta_base, sizeof(float) * 11 * (size_t)n));
  float* X = static_cast<float*>(ctx->ws.feat.ptr);
  float* Y = X + (size_t)n * kDin;
  float* base = static_cast<float*>(ctx->ws.theta_base.ptr);
  TRY(gve_features(ctx, p, d_field, g, n_detail, g99, X));
  TRY_HIP(ctx, gve::mlp_standardize(X, nullptr, n, kDin, m->stats, m->stats + 16, X, s));
  TRY(gve_mlp_forward(ctx, m, X, n, Y));
  TRY_HIP(ctx, hipMemcpyAsync(base, p->theta, sizeof(float) * 11 * (size_t)n,
                              hipMemcpyDeviceToDevice, s));
  double L[4] = {NAN, NAN, NAN, NAN};
  TRY(eval_loss(ctx, p, d_field, g, &L[0]));
  const float alphas[3] = {1.0f, 0.5f, 0.25f};
  int32_t chosen = 0;
  for (int a = 0; a < 3 && !chosen; ++a) {
    TRY_HIP(ctx, gve::mlp_apply_delta(p->theta, base, Y, n, m->stats + 32, m->stats + 43,
                                      alphas[a], s));
    TRY(eval_loss(ctx, p, d_field, g, &L[a + 1]));
    if (std::isfinite(L[a + 1]) && L[a + 1] < L[0]) chosen = a + 1;
  }
  if (!chosen)
    TRY_HIP(ctx, hipMemcpyAsync(p->theta, base, sizeof(float) * 11 * (size_t)n,
                                hipMemcpyDeviceToDevice, s));
  TRY(gve_params_reset_adam(ctx, p));
  TRY_HIP(ctx, hipStreamSynchronize(s));
  *applied = chosen;
  if (h_losses)
    for (int i = 0; i < 4; ++i) h_losses[i] = L[i];
  return GVE_OK;
}

}  // extern "C"

// ---- batched volumes ------------------------------------------------------------

struct gve_batch {
  int device = 0;
  std::vector<gve_grid> grids;
  std::vector<int64_t> prim_off, vox_off;  // [n_items + 1]
  gve_params* params = nullptr;
};

namespace {

Vol vol_of(const gve_batch* b) {
  return Vol{b->grids.data(), b->prim_off.data(), (int)b->grids.size()};
}

gve_status check_batch(const gve_ctx* ctx, const gve_batch* b) {
  if (!ctx) return GVE_ERR_INVALID_ARGUMENT;
  const_cast<gve_ctx*>(ctx)->last_error.clear();
  if (!b) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "batch is NULL");
  if (b->device != ctx->device)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "batch and context are on different devices");
  return GVE_OK;
}

}  // namespace

gve_status gve_batch_create(gve_ctx* ctx, int32_t n_items, const gve_grid* h_grids,
                            const int64_t* h_counts, gve_batch** out) {
  if (!ctx || !out) return GVE_ERR_INVALID_ARGUMENT;
  ctx->last_error.clear();
  if (n_items < 1 || n_items > (1 << 20) || !h_grids || !h_counts)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "need 1 <= n_items <= 2^20, grids and counts");
  int64_t prims = 0, vox = 0;
  for (int32_t i = 0; i < n_items; ++i) {
    TRY(validate_grid(ctx, h_grids[i]));
    if (h_counts[i] < 1) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "every count must be >= 1");
    prims += h_counts[i];
    vox += h_grids[i].nx * h_grids[i].ny * h_grids[i].nz;
    if (prims >= ((int64_t)1 << 31))
      return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "more than 2^31 - 1 primitives in the batch");
    if (vox > ((int64_t)1 << 36)) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "batch too large");
  }
  gve_batch* b = new (std::nothrow) gve_batch();
  if (!b) return GVE_ERR_OUT_OF_MEMORY;
  b->device = ctx->device;
  b->grids.assign(h_grids, h_grids + n_items);
  b->prim_off.assign((size_t)n_items + 1, 0);
  b->vox_off.assign((size_t)n_items + 1, 0);
  for (int32_t i = 0; i < n_items; ++i) {
    b->prim_off[i + 1] = b->prim_off[i] + h_counts[i];
    b->vox_off[i + 1] = b->vox_off[i] + h_grids[i].nx * h_grids[i].ny * h_grids[i].nz;
  }
  const gve_status st = gve_params_create(ctx, prims, &b->params);
  if (st != GVE_OK) {
    delete b;
    return st;
  }
  *out = b;
  return GVE_OK;
}

void gve_batch_destroy(gve_batch* b) {
  if (!b) return;
  if (b->params) gve_params_destroy(b->params);
  delete b;
}

gve_status gve_batch_params(gve_batch* b, gve_params** out) {
  if (!b || !out) return GVE_ERR_INVALID_ARGUMENT;
  *out = b->params;
  return GVE_OK;
}

gve_status gve_batch_offsets(const gve_batch* b, int64_t* h_prim_off, int64_t* h_vox_off) {
  if (!b) return GVE_ERR_INVALID_ARGUMENT;
  if (h_prim_off) std::copy(b->prim_off.begin(), b->prim_off.end(), h_prim_off);
  if (h_vox_off) std::copy(b->vox_off.begin(), b->vox_off.end(), h_vox_off);
  return GVE_OK;
}

namespace {

gve_status item_copy(gve_ctx* ctx, const gve_batch* b, int32_t item, gve_params* other,
                     bool into_batch) {
  TRY(check_batch(ctx, b));
  if (!other) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "params is NULL");
  if (item < 0 || item >= (int32_t)b->grids.size())
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "item out of range");
  const int64_t off = b->prim_off[item], cnt = b->prim_off[item + 1] - off;
  if (other->n != cnt)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "params size differs from the item's count");
  TRY(set_device(ctx));
  const int64_t N = b->params->n;
  const size_t w = sizeof(float) * (size_t)cnt, ld = sizeof(float) * (size_t)N;
  float* bt = b->params->theta + off;
  if (into_batch) {
    TRY_HIP(ctx, hipMemcpy2DAsync(bt, ld, other->theta, w, w, 11, hipMemcpyDeviceToDevice,
                                  ctx->stream));
    const int64_t blocks = std::min<int64_t>((11 * cnt + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_cols, dim3((unsigned)blocks), dim3(256), 0, ctx->stream,
                       b->params->m, N, off, cnt, 11);
    TRY_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(k_zero_cols, dim3((unsigned)blocks), dim3(256), 0, ctx->stream,
                       b->params->v, N, off, cnt, 11);
    TRY_HIP(ctx, hipGetLastError());
  } else {
    TRY_HIP(ctx, hipMemcpy2DAsync(other->theta, w, bt, ld, w, 11, hipMemcpyDeviceToDevice,
                                  ctx->stream));
  }
  return GVE_OK;
}

}  // namespace

gve_status gve_batch_set_item(gve_ctx* ctx, gve_batch* b, int32_t item, const gve_params* src) {
  return item_copy(ctx, b, item, const_cast<gve_params*>(src), true);
}

gve_status gve_batch_get_item(gve_ctx* ctx, const gve_batch* b, int32_t item, gve_params* dst) {
  return item_copy(ctx, b, item, dst, false);
}

gve_status gve_batch_evaluate(gve_ctx* ctx, const gve_batch* b, float* d_out) {
  TRY(check_batch(ctx, b));
  if (!d_out) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_out is NULL");
  TRY(set_device(ctx));
  Binned bn;
  TRY(bin_vol(ctx, b->params, vol_of(b), &bn));
  TRY_HIP(ctx, gve::launch_forward(b->params->rec, bn.gid, bn.start, bn.items, bn.nitems, bn.bg,
                                   ctx->opt.k, d_out, bn.sched, ctx->stream));
  return GVE_OK;
}

gve_status gve_batch_loss_grad(gve_ctx* ctx, const gve_batch* b, const float* d_fields,
                               float* d_grad, double* h_loss) {
  TRY(check_batch(ctx, b));
  if (!d_fields) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_fields is NULL");
  TRY(set_device(ctx));
  TRY(ensure_dloss(ctx));
  gve_params* pm = b->params;
  TRY(select_auto(ctx, pm, d_fields, vol_of(b), true));
  const int ni = (int)b->grids.size();
  TRY(ensure(ctx, ctx->ws.grad_tmp, sizeof(double) * (size_t)ni));
  double* dl = static_cast<double*>(ctx->ws.grad_tmp.ptr);
  TRY_HIP(ctx, gve::fill_f32(pm->acc, gve::kAccStride * pm->n, 0.0f, ctx->stream));
  float* part = nullptr;
  TRY(loss_and_sums_vol(ctx, pm, d_fields, vol_of(b), dl, &part));
  if (d_grad) {
    TRY_HIP(ctx, gve::launch_update(0, pm->theta, pm->m, pm->v, pm->acc, part, pm->offset, nullptr,
                                    d_grad, pm->n, pm->t, ctx->opt, nullptr, ctx->stream));
  } else {
    TRY_HIP(ctx, gve::fill_f32(pm->acc, gve::kAccStride * pm->n, 0.0f, ctx->stream));
  }
  if (h_loss) {
    TRY_HIP(ctx, hipMemcpyAsync(h_loss, dl, sizeof(double) * (size_t)ni, hipMemcpyDeviceToHost,
                                ctx->stream));
    TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double tot = 0.0;
    for (int i = 0; i < ni; ++i) tot += h_loss[i];
    ctx->stats.last_loss = tot;
    if (!std::isfinite(tot)) return fail(ctx, GVE_ERR_NUMERIC, "loss is not finite");
  }
  return GVE_OK;
}

gve_status gve_batch_refine(gve_ctx* ctx, gve_batch* b, const float* d_fields, int32_t iters,
                            double* h_loss) {
  TRY(check_batch(ctx, b));
  if (!d_fields) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_fields is NULL");
  if (iters < 0) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "iters must be >= 0");
  return refine_vol(ctx, b->params, d_fields, vol_of(b), iters, h_loss);
}

gve_status gve_batch_count_pairs(gve_ctx* ctx, const gve_batch* b, int64_t* h_in_support,
                                 int64_t* h_candidates) {
  TRY(check_batch(ctx, b));
  if (!h_in_support || !h_candidates)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "output pointers are required");
  TRY(set_device(ctx));
  Binned bn;
  TRY(bin_vol(ctx, b->params, vol_of(b), &bn));
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(ctx->ws.dloss.ptr) + 4;
  TRY_HIP(ctx, gve::fill_u64(cnt, 3, ctx->stream));
  TRY_HIP(ctx, gve::launch_count(b->params->rec, bn.gid, bn.start, bn.items, bn.nitems, bn.bg,
                                 ctx->opt.k, cnt, ctx->stream));
  TRY_HIP(ctx, hipMemcpyAsync(ctx->ws.h_pinned, cnt, 24, hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const unsigned long long* hc = static_cast<unsigned long long*>(ctx->ws.h_pinned);
  *h_in_support = (int64_t)hc[0];
  *h_candidates = (int64_t)hc[1];
  ctx->stats.n_in_support = (int64_t)hc[0];
  ctx->stats.n_candidates = (int64_t)hc[1];
  ctx->stats.n_atomics = (int64_t)hc[2];
  return GVE_OK;
}

// ---- autotuner -----------------------------------------------------------------

namespace {

// Restores the context's options on every exit unless committed.
struct OptionsGuard {
  gve_ctx* ctx;
  gve_options saved;
  bool keep = false;
  explicit OptionsGuard(gve_ctx* c) : ctx(c), saved(c->opt) {}
  ~OptionsGuard() {
    if (!keep) ctx->opt = saved;
  }
};

// One timed unit of the tuner: binning + fused kernel + per-volume loss.
gve_status tune_pass(gve_ctx* ctx, const gve_params* p, const float* d_field, const Vol& vol) {
  Binned bn;
  TRY(bin_vol(ctx, p, vol, &bn));
  TRY(ensure(ctx, ctx->ws.brick_loss, sizeof(float) * (size_t)std::max<int64_t>(bn.bg.nbricks, 1)));
  float* bl = static_cast<float*>(ctx->ws.brick_loss.ptr);
  float* part = nullptr;
  TRY(partials_for(ctx, bn.capacity, &part));
  TRY(fused(ctx, p, bn, d_field, part, bl, false));
  TRY(ensure(ctx, ctx->ws.grad_tmp, sizeof(double) * (size_t)vol.n));
  TRY(losses(ctx, bn, bl, static_cast<double*>(ctx->ws.grad_tmp.ptr)));
  return GVE_OK;
}

int bucket(double x, double per_octave) {
  return (int)std::lround(std::log2(std::max(x, 1e-6)) * per_octave);
}

// Times every brick shape, waves per brick and schedule on the workload (a
// warm-up pass, then the median of `reps` passes) and returns the fastest as
// (brick, brick_z, schedule, waves).  Entries go to h_table while it has room.  The context's
// options are restored on return; the passes' gradient sums are cleared.
gve_status tune_candidates(gve_ctx* ctx, gve_params* P, const float* d_field, const Vol& vol,
                           int32_t reps, gve_tune_entry* h_table, int32_t table_len,
                           int32_t* written, std::array<int, 4>* best) {
  // (brick, depth, waves per brick)
  static const int shapes[][3] = {{8, 8, 1},  {8, 8, 2},  {8, 8, 4},  {8, 16, 1}, {8, 16, 2},
                                  {8, 16, 4}, {8, 32, 1}, {8, 32, 2}, {8, 32, 4}, {16, 16, 1}};
  static const int scheds[] = {GVE_SCHED_INDEX, GVE_SCHED_XCD, GVE_SCHED_QUEUE};
  OptionsGuard guard(ctx);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TRY_HIP(ctx, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(ctx, GVE_ERR_DEVICE, "hipEventCreate");
  }
  struct Events {
    hipEvent_t a, b;
    ~Events() {
      hipEventDestroy(a);
      hipEventDestroy(b);
    }
  } events{e0, e1};
  float best_ms = INFINITY;
  *written = 0;
  for (const auto& sh : shapes) {
    for (int sc : scheds) {
      ctx->opt = guard.saved;
      ctx->opt.brick = sh[0];
      ctx->opt.brick_z = sh[1];
      ctx->opt.brick_waves = sh[2];
      ctx->opt.schedule = sc;
      TRY(tune_pass(ctx, P, d_field, vol));  // warm-up
      std::vector<float> ms;
      for (int32_t r = 0; r < reps; ++r) {
        TRY_HIP(ctx, hipEventRecord(e0, ctx->stream));
        TRY(tune_pass(ctx, P, d_field, vol));
        TRY_HIP(ctx, hipEventRecord(e1, ctx->stream));
        TRY_HIP(ctx, hipEventSynchronize(e1));
        float t = 0.0f;
        TRY_HIP(ctx, hipEventElapsedTime(&t, e0, e1));
        ms.push_back(t);
      }
      std::sort(ms.begin(), ms.end());
      const float med = ms[ms.size() / 2];
      if (*written < table_len)
        h_table[(*written)++] = gve_tune_entry{sh[0], sh[1], sc, med, sh[2]};
      if (med < best_ms) {
        best_ms = med;
        *best = {sh[0], sh[1], sc, sh[2]};
      }
    }
  }
  // the tuning passes added their sums to the accumulators (atomics mode)
  TRY_HIP(ctx, gve::fill_f32(P->acc, gve::kAccStride * P->n, 0.0f, ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return GVE_OK;
}

// The workload an automatic choice belongs to: primitive count, then every
// volume's dimensions and primitive range.
std::vector<int64_t> auto_key(const Vol& vol, const gve_params* p) {
  std::vector<int64_t> k = {p->n};
  for (int i = 0; i < vol.n; ++i) {
    const gve_grid& g = vol.grids[i];
    k.insert(k.end(), {g.nx, g.ny, g.nz, vol.prim_off[i + 1] - vol.prim_off[i]});
  }
  return k;
}

// options.brick = 0: picks the brick shape and schedule for the workload
// (the volumes' voxel count and the primitive count): the choice made
// earlier for it, else, when tuning is allowed and a target field is given,
// the tuner's choice (then kept), else 8 x 8 x 32 bricks in XCD chunks.
gve_status select_auto(gve_ctx* ctx, const gve_params* p, const float* d_field, const Vol& vol,
                       bool tune) {
  if (ctx->opt.brick != 0) return GVE_OK;
  const auto key = auto_key(vol, p);
  auto hit = ctx->auto_choice.find(key);
  std::array<int, 4> c = {8, 32, GVE_SCHED_XCD, 1};
  if (hit != ctx->auto_choice.end()) {
    c = hit->second;
  } else if (tune && d_field) {
    TRY(ensure_dloss(ctx));
    int32_t written = 0;
    TRY(tune_candidates(ctx, const_cast<gve_params*>(p), d_field, vol, 3, nullptr, 0, &written,
                        &c));
    ctx->auto_choice[key] = c;
  }
  ctx->auto_bxy = c[0];
  ctx->auto_bz = c[1];
  ctx->auto_sched = c[2];
  ctx->auto_waves = c[3];
  return GVE_OK;
}

}  // namespace

gve_status gve_autotune(gve_ctx* ctx, const gve_params* p, const float* d_field, gve_grid g,
                        const gve_batch* b, int32_t reps, gve_tune_entry* h_table,
                        int32_t table_len, int32_t* n_written) {
  if (!ctx) return GVE_ERR_INVALID_ARGUMENT;
  ctx->last_error.clear();
  if (n_written) *n_written = 0;
  if (!d_field) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "field is NULL");
  if (reps < 1 || reps > 1000) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "reps must be in [1, 1000]");
  if (table_len < 0 || (table_len > 0 && !h_table))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "table_len > 0 needs a table");
  const int64_t single_off[2] = {0, p ? p->n : 0};
  Vol vol;
  gve_params* P;
  int64_t M = 0;
  if (b) {
    TRY(check_batch(ctx, b));
    vol = vol_of(b);
    P = b->params;
    M = b->vox_off.back();
  } else {
    TRY(check_ctx_params(ctx, p));
    TRY(validate_grid(ctx, g));
    vol = Vol{&g, single_off, 1};
    P = const_cast<gve_params*>(p);
    M = g.nx * g.ny * g.nz;
  }
  TRY(set_device(ctx));
  TRY(ensure_dloss(ctx));
  OptionsGuard guard(ctx);
  // cache key: box coverage per voxel measured at 8x8x8
  ctx->opt.brick = 8;
  ctx->opt.brick_z = 8;
  ctx->opt.brick_waves = 1;
  ctx->opt.schedule = GVE_SCHED_INDEX;
  {
    Binned bn;
    TRY(bin_vol(ctx, P, vol, &bn));
  }
  const double cover = (double)ctx->stats.n_overlaps * 512.0 / (double)M;
  const std::array<int, 4> key = {vol.n, bucket((double)M, 1.0), bucket((double)P->n, 1.0),
                                  bucket(cover, 2.0)};
  auto hit = ctx->tuned.find(key);
  std::array<int, 4> c{};
  int32_t written = 0;
  if (hit != ctx->tuned.end()) {
    c = hit->second;
  } else {
    TRY(tune_candidates(ctx, P, d_field, vol, reps, h_table, table_len, &written, &c));
    ctx->tuned[key] = c;
  }
  gve_options best = guard.saved;
  if (guard.saved.brick == 0) {
    // automatic mode stays on; the choice becomes this workload's
    ctx->auto_choice[auto_key(vol, P)] = c;
    ctx->auto_bxy = c[0];
    ctx->auto_bz = c[1];
    ctx->auto_sched = c[2];
    ctx->auto_waves = c[3];
  } else {
    best.brick = c[0];
    best.brick_z = c[1];
    best.schedule = c[2];
    best.brick_waves = c[3];
    ctx->opt = best;
    guard.keep = true;
  }
  if (n_written) *n_written = written;
  return GVE_OK;
}

// ---- the paper's own training loop --------------------------------------------------

struct gve_paper {
  int64_t n = 0;
  int device = 0;
  float* theta = nullptr;  // [12][n]
  float* m = nullptr;
  float* v = nullptr;
  int64_t t = 0;
};

namespace {

constexpr int kPRows = 12;

gve_status paper_validate(const gve_ctx* ctx, const gve_paper_options* o) {
  if (!o) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "options are NULL");
  if (!(o->k > 0.f) || !(o->k <= 64.f) || !(o->rho0 > 0.f) || !std::isfinite(o->rho0))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "need 0 < k <= 64 and rho0 > 0");
  if (o->samples < 1 || o->samples > (1 << 26))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "samples must be in [1, 2^26]");
  if (!(o->frac_hi >= 0.f) || !(o->frac_mid >= 0.f) || o->frac_hi + o->frac_mid > 1.f)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "class fractions must be >= 0 and sum to <= 1");
  if (!(o->cell >= 1.f) || !std::isfinite(o->cell))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "cell must be >= 1 voxel");
  if (!(o->aniso_max > 1.f) || !(o->eps > 0.f) || !(o->lr >= 0.f))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "need aniso_max > 1, eps > 0, lr >= 0");
  return GVE_OK;
}

gve_status check_paper(const gve_ctx* ctx, const gve_paper* p) {
  if (!ctx) return GVE_ERR_INVALID_ARGUMENT;
  const_cast<gve_ctx*>(ctx)->last_error.clear();
  if (!p) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "paper parameter set is NULL");
  if (p->device != ctx->device)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "parameter set and context on different devices");
  return GVE_OK;
}

// Bucket np points into the cell grid: sorted point indices and cell ranges.
gve_status paper_bucket(gve_ctx* ctx, const float* pts, int64_t np, const gve::CellGrid& cg,
                        const uint32_t** sorted, const uint32_t** start) {
  auto& ws = ctx->ws;
  const int64_t ncells = (int64_t)cg.ncx * cg.ncy * cg.ncz;
  if (ncells >= ((int64_t)1 << 31)) return fail(ctx, GVE_ERR_UNSUPPORTED, "too many cells");
  const size_t pb = sizeof(uint32_t) * (size_t)std::max<int64_t>(np, 1);
  for (int b = 0; b < 2; ++b) {
    TRY(ensure(ctx, ws.p_keys[b], pb));
    TRY(ensure(ctx, ws.p_idx[b], pb));
  }
  TRY(ensure(ctx, ws.p_start, sizeof(uint32_t) * (size_t)(ncells + 1)));
  TRY(ensure(ctx, ws.sort_hist, gve::sort_hist_bytes(np)));
  uint32_t* keys[2] = {static_cast<uint32_t*>(ws.p_keys[0].ptr), static_cast<uint32_t*>(ws.p_keys[1].ptr)};
  uint32_t* idx[2] = {static_cast<uint32_t*>(ws.p_idx[0].ptr), static_cast<uint32_t*>(ws.p_idx[1].ptr)};
  TRY_HIP(ctx, gve::paper_cell_keys(pts, np, cg, keys[0], idx[0], ctx->stream));
  int which = 0;
  TRY_HIP(ctx, gve::radix_sort_pairs(keys, idx, np, bits_for(ncells), ws.sort_hist.ptr, &which,
                                     ctx->stream));
  uint32_t* st = static_cast<uint32_t*>(ws.p_start.ptr);
  TRY_HIP(ctx, gve::launch_ranges(keys[which], np, ncells, st, ctx->stream));
  *sorted = idx[which];
  *start = st;
  return GVE_OK;
}

// Sums w a G and w G at np points (the first S get the numerator).
gve_status paper_accumulate(gve_ctx* ctx, const gve_paper* p, const gve::CellGrid& cg, float k,
                            const float* pts, int64_t np, int64_t S, const uint32_t** sorted,
                            const uint32_t** start, double** num, double** den) {
  TRY(paper_bucket(ctx, pts, np, cg, sorted, start));
  TRY(ensure(ctx, ctx->ws.p_acc, sizeof(double) * 2 * (size_t)std::max<int64_t>(np, 1)));
  double* acc = static_cast<double*>(ctx->ws.p_acc.ptr);
  TRY_HIP(ctx, gve::paper_zero(acc, 2 * np, ctx->stream));
  *num = acc;
  *den = acc + np;
  TRY_HIP(ctx, gve::paper_forward(p->theta, p->n, cg, k, S, pts, *sorted, *start, *num, *den,
                                  ctx->stream));
  return GVE_OK;
}

// One objective evaluation at 2S points (samples then partners): losses to
// loss[0..5], gradient (mode 0) or Adam step (mode 1, step t).
gve_status paper_pass(gve_ctx* ctx, gve_paper* p, const float* d_field, const gve_grid& g,
                      const gve_paper_options& o, float lam_sm, const float* pts,
                      const float* vals, int64_t S, int mode, float* d_grad, double* loss) {
  const gve::CellGrid cg = gve::make_cells(g, o.cell);
  const uint32_t *sorted = nullptr, *start = nullptr;
  double *num = nullptr, *den = nullptr;
  TRY_HIP(ctx, gve::paper_zero(loss, 6, ctx->stream));
  TRY(paper_accumulate(ctx, p, cg, o.k, pts, 2 * S, S, &sorted, &start, &num, &den));
  TRY(ensure(ctx, ctx->ws.p_coef, sizeof(float) * 4 * (size_t)S));
  float* coefA = static_cast<float*>(ctx->ws.p_coef.ptr);
  float* coefB = coefA + 2 * S;
  TRY_HIP(ctx, gve::paper_coef(S, o, lam_sm, num, den, vals, coefA, coefB, loss, ctx->stream));
  TRY_HIP(ctx, gve::paper_backward(p->theta, p->m, p->v, p->n, cg, o, mode, p->t, S, pts, sorted,
                                   start, coefA, coefB, d_field, g, d_grad, loss + 3,
                                   ctx->stream));
  return GVE_OK;
}

double paper_total(const gve_paper_options& o, float lam_sm, const double* parts) {
  return parts[0] + o.lam_rho * parts[1] + lam_sm * parts[2] + o.lam_anc * parts[3] +
         o.lam_aniso * parts[4] + o.lam_cap * parts[5];
}

// Class block offsets of the field; returns the class sizes on the host.
gve_status paper_classes(gve_ctx* ctx, const float* d_field, const gve_grid& g,
                         const gve_paper_options& o, const uint32_t** off_hi,
                         const uint32_t** off_mid, uint64_t* n_hi_vox, uint64_t* n_mid_vox) {
  const int64_t M = g.nx * g.ny * g.nz;
  const int64_t nb = gve::paper_class_blocks(M);
  if (M >= ((int64_t)1 << 32)) return fail(ctx, GVE_ERR_UNSUPPORTED, "volume above 2^32 voxels");
  TRY(ensure(ctx, ctx->ws.p_cls, sizeof(uint32_t) * 4 * (size_t)(nb + 1)));
  TRY(ensure(ctx, ctx->ws.scan_tmp, gve::scan_tmp_bytes(nb + 1)));
  uint32_t* base = static_cast<uint32_t*>(ctx->ws.p_cls.ptr);
  uint32_t *c_hi = base, *c_mid = base + (nb + 1), *o_hi = base + 2 * (nb + 1),
           *o_mid = base + 3 * (nb + 1);
  TRY_HIP(ctx, gve::paper_class_counts(d_field, M, o.v_hi, o.v_occ, c_hi, c_mid, ctx->stream));
  TRY_HIP(ctx, gve::scan_exclusive_u32(c_hi, o_hi, nb, ctx->ws.scan_tmp.ptr, ctx->stream));
  TRY_HIP(ctx, gve::scan_exclusive_u32(c_mid, o_mid, nb, ctx->ws.scan_tmp.ptr, ctx->stream));
  uint32_t* hp = static_cast<uint32_t*>(ctx->ws.h_pinned);
  TRY_HIP(ctx, hipMemcpyAsync(hp, o_hi + nb, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(ctx, hipMemcpyAsync(hp + 1, o_mid + nb, sizeof(uint32_t), hipMemcpyDeviceToHost,
                              ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *n_hi_vox = hp[0];
  *n_mid_vox = hp[1];
  *off_hi = o_hi;
  *off_mid = o_mid;
  return GVE_OK;
}

void paper_class_split(const gve_paper_options& o, uint64_t n_hi_vox, uint64_t n_mid_vox,
                       int* n_hi, int* n_mid) {
  const int S = o.samples;
  *n_hi = n_hi_vox ? (int)std::floor((double)o.frac_hi * S + 0.5) : 0;
  *n_mid = n_mid_vox ? (int)std::floor((double)o.frac_mid * S + 0.5) : 0;
}

gve_status paper_points(gve_ctx* ctx, int64_t S, float** pts, float** vals) {
  TRY(ensure(ctx, ctx->ws.p_pts, sizeof(float) * 7 * (size_t)S));
  *pts = static_cast<float*>(ctx->ws.p_pts.ptr);
  *vals = *pts + 6 * S;
  return GVE_OK;
}

}  // namespace

gve_status gve_paper_default_options(gve_paper_options* o) {
  if (!o) return GVE_ERR_INVALID_ARGUMENT;
  o->k = 5.0f;
  o->rho0 = 0.05f;
  o->samples = 3072;
  o->frac_hi = 0.35f;
  o->frac_mid = 0.40f;
  o->v_hi = 0.4f;
  o->v_occ = 0.02f;
  o->lam_rho = 0.1f;
  o->lam_sm_start = 0.1f;
  o->lam_sm_end = 0.01f;
  o->lam_anc = 0.01f;
  o->lam_aniso = 1.0f;
  o->lam_cap = 1.0f;
  o->aniso_max = 3.0f;
  o->ell_lo = std::log(0.25f);
  o->ell_hi = std::log(64.0f);
  o->lr = 8e-3f;
  o->beta1 = 0.9f;
  o->beta2 = 0.999f;
  o->eps = 1e-8f;
  o->cell = 32.0f;
  return GVE_OK;
}

gve_status gve_paper_create(gve_ctx* ctx, int64_t n, gve_paper** out) {
  if (!ctx || !out) return GVE_ERR_INVALID_ARGUMENT;
  ctx->last_error.clear();
  if (n < 1 || n >= ((int64_t)1 << 31))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "primitive count must be in [1, 2^31)");
  TRY(set_device(ctx));
  gve_paper* p = new (std::nothrow) gve_paper();
  if (!p) return GVE_ERR_OUT_OF_MEMORY;
  p->n = n;
  p->device = ctx->device;
  const size_t b = sizeof(float) * kPRows * (size_t)n;
  hipError_t e = hipMalloc(&p->theta, b);
  if (e == hipSuccess) e = hipMalloc(&p->m, b);
  if (e == hipSuccess) e = hipMalloc(&p->v, b);
  if (e == hipSuccess) e = gve::fill_f32(p->theta, kPRows * n, 0.0f, ctx->stream);
  if (e == hipSuccess) e = gve::fill_f32(p->m, kPRows * n, 0.0f, ctx->stream);
  if (e == hipSuccess) e = gve::fill_f32(p->v, kPRows * n, 0.0f, ctx->stream);
  if (e != hipSuccess) {
    gve_paper_destroy(p);
    return from_hip(ctx, e, "gve_paper_create");
  }
  *out = p;
  return GVE_OK;
}

void gve_paper_destroy(gve_paper* p) {
  if (!p) return;
  hipSetDevice(p->device);
  hipDeviceSynchronize();
  if (p->theta) hipFree(p->theta);
  if (p->m) hipFree(p->m);
  if (p->v) hipFree(p->v);
  delete p;
}

gve_status gve_paper_upload(gve_ctx* ctx, gve_paper* p, const float* h_theta) {
  TRY(check_paper(ctx, p));
  if (!h_theta) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "h_theta is NULL");
  TRY(set_device(ctx));
  TRY_HIP(ctx, hipMemcpyAsync(p->theta, h_theta, sizeof(float) * kPRows * (size_t)p->n,
                              hipMemcpyHostToDevice, ctx->stream));
  TRY_HIP(ctx, gve::fill_f32(p->m, kPRows * p->n, 0.0f, ctx->stream));
  TRY_HIP(ctx, gve::fill_f32(p->v, kPRows * p->n, 0.0f, ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  p->t = 0;
  return GVE_OK;
}

gve_status gve_paper_download(gve_ctx* ctx, const gve_paper* p, float* h_theta) {
  TRY(check_paper(ctx, p));
  if (!h_theta) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "h_theta is NULL");
  TRY(set_device(ctx));
  TRY_HIP(ctx, hipMemcpyAsync(h_theta, p->theta, sizeof(float) * kPRows * (size_t)p->n,
                              hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return GVE_OK;
}

gve_status gve_paper_from_params(gve_ctx* ctx, gve_paper* p, const gve_params* src, double kappa,
                                 float w0) {
  TRY(check_paper(ctx, p));
  if (!src || src->n != p->n)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "source params missing or of another size");
  if (!(kappa != 0.0) || !std::isfinite(kappa) || !(w0 > 0.f && w0 < 1.f))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "need kappa != 0 and 0 < w0 < 1");
  TRY(set_device(ctx));
  const int64_t n = p->n;
  std::vector<float> h((size_t)11 * n), out((size_t)kPRows * n);
  TRY_HIP(ctx, hipMemcpyAsync(h.data(), src->theta, sizeof(float) * h.size(), hipMemcpyDeviceToHost,
                              ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  std::copy(h.begin(), h.begin() + 10 * n, out.begin());
  const float logit = std::log(w0 / (1.0f - w0));
  for (int64_t i = 0; i < n; ++i) {
    out[10 * n + i] = (float)(h[10 * n + i] / kappa);
    out[11 * n + i] = logit;
  }
  return gve_paper_upload(ctx, p, out.data());
}

gve_status gve_paper_sample(gve_ctx* ctx, const float* d_field, gve_grid g,
                            const gve_paper_options* o, uint64_t seed, int64_t iter, float* d_pts,
                            float* d_vals) {
  if (!ctx) return GVE_ERR_INVALID_ARGUMENT;
  ctx->last_error.clear();
  TRY(paper_validate(ctx, o));
  if (!d_field || !d_pts || !d_vals || iter < 0)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "field, outputs and iter >= 0 are required");
  TRY(validate_grid(ctx, g));
  TRY(set_device(ctx));
  const uint32_t *oh = nullptr, *om = nullptr;
  uint64_t nh = 0, nm = 0;
  TRY(paper_classes(ctx, d_field, g, *o, &oh, &om, &nh, &nm));
  int n_hi, n_mid;
  paper_class_split(*o, nh, nm, &n_hi, &n_mid);
  TRY_HIP(ctx, gve::paper_sample(d_field, g, oh, om, o->samples, n_hi, n_mid, seed, (uint64_t)iter,
                                 o->v_hi, o->v_occ, d_pts, d_vals, ctx->stream));
  return GVE_OK;
}

gve_status gve_paper_eval(gve_ctx* ctx, const gve_paper* p, gve_grid g, const gve_paper_options* o,
                          const float* d_pts, int64_t npts, float* d_vt, float* d_density) {
  TRY(check_paper(ctx, p));
  TRY(paper_validate(ctx, o));
  if (!d_pts || npts < 1 || npts >= ((int64_t)1 << 31) || (!d_vt && !d_density))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "need points, 1 <= npts < 2^31 and an output");
  TRY(validate_grid(ctx, g));
  TRY(set_device(ctx));
  const uint32_t *sorted = nullptr, *start = nullptr;
  double *num = nullptr, *den = nullptr;
  TRY(paper_accumulate(ctx, p, gve::make_cells(g, o->cell), o->k, d_pts, npts, npts, &sorted,
                       &start, &num, &den));
  TRY_HIP(ctx, gve::paper_density(num, den, npts, o->rho0, d_vt, d_density, ctx->stream));
  return GVE_OK;
}

gve_status gve_paper_loss_grad(gve_ctx* ctx, gve_paper* p, const float* d_field, gve_grid g,
                               const gve_paper_options* o, float lam_sm, const float* d_pts,
                               const float* d_vals, int64_t samples, float* d_grad, double* h_parts,
                               double* h_loss) {
  TRY(check_paper(ctx, p));
  TRY(paper_validate(ctx, o));
  if (!d_field || !d_pts || !d_vals || !d_grad || samples < 1 || samples >= ((int64_t)1 << 30))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "field, points, values, gradient and samples required");
  TRY(validate_grid(ctx, g));
  TRY(set_device(ctx));
  TRY(ensure(ctx, ctx->ws.p_loss, sizeof(double) * 8));
  double* loss = static_cast<double*>(ctx->ws.p_loss.ptr);
  TRY(paper_pass(ctx, p, d_field, g, *o, lam_sm, d_pts, d_vals, samples, 0, d_grad, loss));
  double* hp = static_cast<double*>(ctx->ws.h_pinned);
  TRY_HIP(ctx, hipMemcpyAsync(hp, loss, sizeof(double) * 6, hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h_parts) std::copy(hp, hp + 6, h_parts);
  if (h_loss) *h_loss = paper_total(*o, lam_sm, hp);
  return GVE_OK;
}

gve_status gve_paper_refine(gve_ctx* ctx, gve_paper* p, const float* d_field, gve_grid g,
                            const gve_paper_options* o, uint64_t seed, int32_t iters,
                            int32_t first_iter, int32_t schedule_len, double* h_loss) {
  TRY(check_paper(ctx, p));
  TRY(paper_validate(ctx, o));
  if (!d_field || iters < 0 || first_iter < 0 || schedule_len < 1)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "need a field, iters >= 0, schedule_len >= 1");
  TRY(validate_grid(ctx, g));
  TRY(set_device(ctx));
  if (iters == 0) return GVE_OK;
  const uint32_t *oh = nullptr, *om = nullptr;
  uint64_t nh = 0, nm = 0;
  TRY(paper_classes(ctx, d_field, g, *o, &oh, &om, &nh, &nm));
  int n_hi, n_mid;
  paper_class_split(*o, nh, nm, &n_hi, &n_mid);
  const int64_t S = o->samples;
  TRY(ensure(ctx, ctx->ws.p_loss, sizeof(double) * 6 * (size_t)iters));
  double* loss = static_cast<double*>(ctx->ws.p_loss.ptr);
  float *pts = nullptr, *vals = nullptr;
  TRY(paper_points(ctx, S, &pts, &vals));
  std::vector<float> lam((size_t)iters);
  for (int32_t i = 0; i < iters; ++i) {
    const int32_t it = first_iter + i;
    const double f = schedule_len > 1 ? (double)std::min(it, schedule_len - 1) / (schedule_len - 1)
                                      : 0.0;
    lam[i] = (float)(o->lam_sm_start + (o->lam_sm_end - o->lam_sm_start) * f);
    TRY_HIP(ctx, gve::paper_sample(d_field, g, oh, om, (int)S, n_hi, n_mid, seed, (uint64_t)it,
                                   o->v_hi, o->v_occ, pts, vals, ctx->stream));
    p->t += 1;
    TRY(paper_pass(ctx, p, d_field, g, *o, lam[i], pts, vals, S, 1, nullptr, loss + 6 * i));
  }
  std::vector<double> h((size_t)6 * iters);
  TRY_HIP(ctx, hipMemcpyAsync(h.data(), loss, sizeof(double) * h.size(), hipMemcpyDeviceToHost,
                              ctx->stream));
  TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int32_t i = 0; i < iters; ++i) {
    const double L = paper_total(*o, lam[i], &h[6 * (size_t)i]);
    if (h_loss) h_loss[i] = L;
    if (!std::isfinite(L)) return fail(ctx, GVE_ERR_NUMERIC, "objective is not finite");
  }
  return GVE_OK;
}
