// C ABI of libgve.so: argument validation, device memory, and the order in
// which the binning, field and update kernels are queued on the caller's
// stream.  Declarations and contracts are in include/gve.h.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "common.h"

using gve::Scratch;

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

// Grow-only device buffer.  Synchronises before freeing the old allocation.
gve_status ensure(gve_ctx* ctx, Scratch& s, size_t bytes) {
  if (s.bytes >= bytes && s.ptr) return GVE_OK;
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

// Small device block: [0] loss (double), [1] pair total (u64), [2] clamp
// count (u64), [16 ..] loss-reduction partials.  Zeroed when first allocated.
gve_status ensure_dloss(gve_ctx* ctx) {
  if (ctx->ws.dloss.ptr) return GVE_OK;
  const size_t nd = 16 + gve::loss_reduce_tmp_doubles();
  TRY(ensure(ctx, ctx->ws.dloss, sizeof(double) * nd));
  TRY_HIP(ctx, gve::fill_u64(static_cast<unsigned long long*>(ctx->ws.dloss.ptr), (int64_t)nd,
                             ctx->stream));
  return GVE_OK;
}

gve_status validate_options(const gve_ctx* ctx, const gve_options& o) {
  if (!(o.k > 0.0f) || !std::isfinite(o.k) || o.k > 64.0f)
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "k must be finite, > 0 and <= 64");
  if (!(o.brick == 0 || o.brick == 8 || o.brick == 16))
    return fail(ctx, GVE_ERR_UNSUPPORTED, "brick must be 0 (auto), 8 or 16");
  if (!(o.lr >= 0.0f) || !std::isfinite(o.lr))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "lr must be finite and >= 0");
  if (!(o.beta1 >= 0.0f && o.beta1 < 1.0f) || !(o.beta2 >= 0.0f && o.beta2 < 1.0f))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "beta1, beta2 must lie in [0, 1)");
  if (!(o.eps > 0.0f) || !std::isfinite(o.eps))
    return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "eps must be finite and > 0");
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

int brick_edge(const gve_ctx* ctx) { return ctx->opt.brick == 0 ? 8 : ctx->opt.brick; }

int bits_for(int64_t nbricks) {
  int b = 0;
  while (((int64_t)1 << b) < nbricks) ++b;
  return b;
}

struct Binned {
  gve::BrickGeom bg;
  const uint32_t* gid = nullptr;
  const uint32_t* start = nullptr;
  int64_t npairs = 0;
};

// prep -> scan -> emit -> radix sort -> brick ranges.  Reads the pair count
// back to the host (one small synchronising copy) to size the pair buffers.
gve_status bin(gve_ctx* ctx, const gve_params* p, const gve_grid& g, Binned* out) {
  hipStream_t s = ctx->stream;
  auto& ws = ctx->ws;
  const int64_t n = p->n;
  gve::BrickGeom bg = gve::brick_geometry(g, brick_edge(ctx));
  if (bg.nbricks >= ((int64_t)1 << 31))
    return fail(ctx, GVE_ERR_UNSUPPORTED, "too many bricks for 32-bit brick keys");
  TRY(ensure(ctx, ws.scan_tmp, gve::scan_tmp_bytes(n + 1)));
  TRY(ensure_dloss(ctx));
  unsigned long long* total = reinterpret_cast<unsigned long long*>(ws.dloss.ptr) + 1;
  TRY_HIP(ctx, gve::fill_u64(total, 1, s));
  TRY_HIP(ctx, gve::launch_prep(p->theta, n, g, ctx->opt.k, bg, p->rec, p->count, total, s));
  TRY_HIP(ctx, gve::scan_exclusive_u32(p->count, p->offset, n, ws.scan_tmp.ptr, s));
  TRY_HIP(ctx, hipMemcpyAsync(ws.h_pinned, total, sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s));
  TRY_HIP(ctx, hipStreamSynchronize(s));
  const unsigned long long T = *reinterpret_cast<unsigned long long*>(ws.h_pinned);
  if (T >= 0xFFFFFFF0ull)
    return fail(ctx, GVE_ERR_UNSUPPORTED,
                "more than 2^32 (primitive, brick) pairs; use larger bricks or a smaller k");
  const size_t pair_bytes = sizeof(uint32_t) * (size_t)(T > 0 ? T : 1);
  for (int b = 0; b < 2; ++b) {
    TRY(ensure(ctx, ws.keys[b], pair_bytes));
    TRY(ensure(ctx, ws.vals[b], pair_bytes));
  }
  TRY(ensure(ctx, ws.sort_hist, gve::sort_hist_bytes((int64_t)T)));
  TRY(ensure(ctx, ws.brick_start, sizeof(uint32_t) * (size_t)(bg.nbricks + 1)));
  uint32_t* keys[2] = {static_cast<uint32_t*>(ws.keys[0].ptr), static_cast<uint32_t*>(ws.keys[1].ptr)};
  uint32_t* vals[2] = {static_cast<uint32_t*>(ws.vals[0].ptr), static_cast<uint32_t*>(ws.vals[1].ptr)};
  TRY_HIP(ctx, gve::launch_emit(p->rec, p->offset, n, bg, keys[0], vals[0], s));
  int which = 0;
  TRY_HIP(ctx, gve::radix_sort_pairs(keys, vals, (int64_t)T, bits_for(bg.nbricks), ws.sort_hist.ptr,
                                     &which, s));
  uint32_t* start = static_cast<uint32_t*>(ws.brick_start.ptr);
  TRY_HIP(ctx, gve::launch_ranges(keys[which], (int64_t)T, bg.nbricks, start, s));
  out->bg = bg;
  out->gid = vals[which];
  out->start = start;
  out->npairs = (int64_t)T;
  ctx->stats.n_primitives = n;
  ctx->stats.n_bricks = bg.nbricks;
  ctx->stats.n_overlaps = (int64_t)T;
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

// Fused forward + squared error + backward into p->acc, loss into dloss[0].
gve_status loss_and_sums(gve_ctx* ctx, const gve_params* p, const float* d_field, const gve_grid& g,
                         double* d_loss_out) {
  Binned bn;
  TRY(bin(ctx, p, g, &bn));
  TRY(ensure(ctx, ctx->ws.brick_loss, sizeof(float) * (size_t)bn.bg.nbricks));
  float* bl = static_cast<float*>(ctx->ws.brick_loss.ptr);
  TRY_HIP(ctx, gve::launch_fused(p->rec, bn.gid, bn.start, g, bn.bg, ctx->opt.k, d_field, p->acc,
                                 p->n, bl, ctx->stream));
  double* dl = static_cast<double*>(ctx->ws.dloss.ptr);
  TRY_HIP(ctx, gve::launch_loss_reduce(bl, bn.bg.nbricks, dl + 16, d_loss_out, ctx->stream));
  return GVE_OK;
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
  if (hipGetDevice(&ctx->device) != hipSuccess || hipHostMalloc(&ctx->ws.h_pinned, 256) != hipSuccess) {
    delete ctx;
    return GVE_ERR_DEVICE;
  }
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
                    &ws.grad_tmp};
  for (Scratch* s : all)
    if (s->ptr) hipFree(s->ptr);
  if (ws.h_pinned) hipHostFree(ws.h_pinned);
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
  if (e == hipSuccess) e = hipMalloc(&p->acc, sizeof(float) * 10 * (size_t)n);
  if (e == hipSuccess) e = hipMalloc(&p->rec, sizeof(gve::Record) * (size_t)n);
  if (e == hipSuccess) e = hipMalloc(&p->count, sizeof(uint32_t) * (size_t)n);
  if (e == hipSuccess) e = hipMalloc(&p->offset, sizeof(uint32_t) * (size_t)(n + 1));
  if (e == hipSuccess) e = gve::fill_f32(p->theta, 11 * n, 0.0f, ctx->stream);
  if (e == hipSuccess) e = gve::fill_f32(p->m, 11 * n, 0.0f, ctx->stream);
  if (e == hipSuccess) e = gve::fill_f32(p->v, 11 * n, 0.0f, ctx->stream);
  if (e == hipSuccess) e = gve::fill_f32(p->acc, 10 * n, 0.0f, ctx->stream);
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
  TRY_HIP(ctx, gve::launch_forward(p->rec, bn.gid, bn.start, g, bn.bg, ctx->opt.k, d_out,
                                   ctx->stream));
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
  TRY_HIP(ctx, gve::fill_f32(pm->acc, 10 * p->n, 0.0f, ctx->stream));
  double* dl = static_cast<double*>(ctx->ws.dloss.ptr);
  TRY(loss_and_sums(ctx, p, d_field, g, dl));
  if (d_grad) {
    TRY_HIP(ctx, gve::launch_update(0, pm->theta, pm->m, pm->v, pm->acc, nullptr, d_grad, p->n,
                                    p->t, ctx->opt, nullptr, ctx->stream));
  } else {
    TRY_HIP(ctx, gve::fill_f32(pm->acc, 10 * p->n, 0.0f, ctx->stream));
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

gve_status gve_adam_step(gve_ctx* ctx, gve_params* p, const float* d_grad) {
  TRY(check_ctx_params(ctx, p));
  if (!d_grad) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_grad is NULL");
  TRY(set_device(ctx));
  TRY(ensure_dloss(ctx));
  p->t += 1;
  TRY_HIP(ctx, gve::launch_update(2, p->theta, p->m, p->v, p->acc, d_grad, nullptr, p->n, p->t,
                                  ctx->opt, clamp_counter(ctx), ctx->stream));
  ctx->stats.iterations = p->t;
  return GVE_OK;
}

gve_status gve_refine(gve_ctx* ctx, gve_params* p, const float* d_field, gve_grid g,
                      int32_t iters, double* h_loss_hist) {
  TRY(check_ctx_params(ctx, p));
  if (!d_field) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "d_field is NULL");
  if (iters < 0) return fail(ctx, GVE_ERR_INVALID_ARGUMENT, "iters must be >= 0");
  TRY(validate_grid(ctx, g));
  TRY(set_device(ctx));
  TRY(ensure_dloss(ctx));
  TRY(ensure(ctx, ctx->ws.grad_tmp, sizeof(double) * (size_t)(iters > 0 ? iters : 1)));
  double* hist = static_cast<double*>(ctx->ws.grad_tmp.ptr);
  TRY_HIP(ctx, gve::fill_f32(p->acc, 10 * p->n, 0.0f, ctx->stream));
  for (int32_t it = 0; it < iters; ++it) {
    TRY(loss_and_sums(ctx, p, d_field, g, hist + it));
    p->t += 1;
    TRY_HIP(ctx, gve::launch_update(1, p->theta, p->m, p->v, p->acc, nullptr, nullptr, p->n, p->t,
                                    ctx->opt, clamp_counter(ctx), ctx->stream));
  }
  ctx->stats.iterations = p->t;
  if (iters > 0) {
    TRY_HIP(ctx, hipMemcpyAsync(ctx->ws.h_pinned, clamp_counter(ctx), sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, ctx->stream));
    double last = 0.0;
    if (h_loss_hist) {
      TRY_HIP(ctx, hipMemcpyAsync(h_loss_hist, hist, sizeof(double) * (size_t)iters,
                                  hipMemcpyDeviceToHost, ctx->stream));
    }
    TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->stats.n_clamped = (int64_t) * static_cast<unsigned long long*>(ctx->ws.h_pinned);
    if (h_loss_hist) {
      last = h_loss_hist[iters - 1];
      ctx->stats.last_loss = last;
      for (int32_t it = 0; it < iters; ++it)
        if (!std::isfinite(h_loss_hist[it])) return fail(ctx, GVE_ERR_NUMERIC, "loss is not finite");
    }
  }
  return GVE_OK;
}

gve_status gve_get_stats(const gve_ctx* ctx, gve_stats* out) {
  if (!ctx || !out) return GVE_ERR_INVALID_ARGUMENT;
  *out = ctx->stats;
  return GVE_OK;
}

}  // extern "C"
