/*
 * gve.h -- C ABI of the fixed-budget Gaussian volume encoder (libgve.so).
 *
 * A scalar field on a regular voxel grid is represented by a fixed set of N
 * weighted anisotropic 3-D Gaussians (paper Sec. III-A: the budget N is set
 * before training and never changes).  Primitive i has centre mu_i, a raw
 * quaternion q_i = (w, x, y, z) (scalar first, Hamilton convention, normalised
 * inside every call), log-scales l_i and a scalar weight c_i, and covariance
 * Sigma_i = R(q_i) S_i S_i^T R(q_i)^T with S_i = diag(exp(l_i)).  The encoded
 * field is the truncated weighted sum (Sec. III-C, eq:field, read for an
 * unnormalised sum with one weight per primitive):
 *
 *     Vhat(p) = sum_i c_i exp(-m_i(p)^2 / 2) [m_i(p)^2 < k^2],
 *     m_i(p)^2 = (p - mu_i)^T Sigma_i^{-1} (p - mu_i),
 *
 * with the hard k-sigma cut of Sec. III-C ("squared Mahalanobis distance below"
 * k^2).  Coordinates are voxel-index coordinates (Sec. III-B): voxel (i, j, k)
 * of a grid is the point (x0 + i, y0 + j, z0 + k); field buffers are float32,
 * x fastest: index = i + nx * (j + ny * k).
 *
 * Conventions for every call:
 *  - Return GVE_OK or an error status; no C++ exception crosses the ABI.
 *  - Arguments are validated on the host before any device work is queued; on
 *    a validation error nothing is written.  gve_last_error(ctx) describes the
 *    most recent failure.
 *  - "d_" pointers are device pointers (HIP device memory on the context's
 *    device); "h_" pointers are host pointers.  The caller owns every buffer it
 *    passes and must keep it alive until the stream has executed the work.
 *  - Work is queued on the context's stream.  Calls that write host memory
 *    (h_ outputs) synchronise that stream before returning.  The others queue
 *    their kernels asynchronously, but each binning of the primitives (every
 *    evaluation, loss and gradient) waits for two small device-to-host reads
 *    on the stream (the totals of box and kept (primitive, brick) pairs, from
 *    which the pair buffers are sized), and a call whose grids or brick shape
 *    differ from the previous call's also waits for the upload of its volume
 *    descriptors.  Refinement (gve_refine, gve_batch_refine) waits so only in
 *    its first iteration: later iterations bin into buffers of the first
 *    one's size plus a quarter, with the counts kept on the device, and the
 *    host reads one overflow flag per 64 iterations.  A binning that did not
 *    fit skips its updates; the call then restores the parameters and Adam
 *    state saved at the start of those 64 iterations and redoes them with
 *    buffers sized from the largest totals seen (stats.n_resized counts such
 *    redos).  The result equals that of synchronous binning.
 *  - A context is not thread-safe; use one per host thread.  Contexts own
 *    device scratch that grows as needed and is released by gve_destroy.
 */
#ifndef GVE_H
#define GVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GVE_NPARAM 11 /* mu_x mu_y mu_z q_w q_x q_y q_z l_x l_y l_z c */

typedef enum gve_status {
  GVE_OK = 0,
  GVE_ERR_INVALID_ARGUMENT = 1,
  GVE_ERR_BUDGET_INFEASIBLE = 2, /* Sec. V-B: request cannot be met by distinct seeds */
  GVE_ERR_OUT_OF_MEMORY = 3,
  GVE_ERR_DEVICE = 4,            /* a HIP call or kernel launch failed */
  GVE_ERR_NUMERIC = 5,           /* non-finite loss or parameters */
  GVE_ERR_UNSUPPORTED = 6
} gve_status;

/* Regular voxel grid: nx*ny*nz voxels, voxel (i,j,k) at (x0+i, y0+j, z0+k). */
typedef struct gve_grid {
  int64_t nx, ny, nz;
  int64_t x0, y0, z0;
} gve_grid;

/*
 * Options.  k: truncation radius in standard deviations (> 0; Sec. III-C uses
 * 5).  brick, brick_z: primitives are binned to bricks of brick x brick x
 * brick_z voxels; supported shapes are 8x8x8, 8x8x16, 8x8x32 and 16x16x16
 * (brick_z 0 picks the same as brick).  brick 0 is automatic: the shape and
 * the schedule are chosen per workload (each volume's dimensions and
 * primitive count):
 * the choice made earlier for that workload if any; else, on a call with a
 * target field (gve_loss_grad, gve_refine, gve_batch_loss_grad,
 * gve_batch_refine; not the allocation-free entry point), the fastest of
 * every shape and schedule, timed as gve_autotune does and then kept; else
 * 8x8x32 with the XCD schedule (brick_z and schedule are then not used;
 * stats.bin_brick, bin_brick_z and bin_schedule report the choice).  The
 * shape changes only the summation order, not the result beyond float32
 * rounding.  lr,
 * beta1, beta2, eps: Adam (Sec. III-F cites Kingma and Ba; Table
 * tab:training-config gives lr 8e-3).  ell_min/ell_max: clamp of the
 * log-scales after each Adam step (a guard against collapsing or exploding
 * primitives; pass -inf/+inf to disable).  deterministic: 1 = each
 * (primitive, brick) pair writes its gradient sums to its own slot and the
 * update sums them per primitive in a fixed order, so gradients are bitwise
 * reproducible and no atomics are issued; 0 = each pair's sums are added to
 * the primitive's accumulators with float atomics (default: about 6 % faster
 * end to end, result order-dependent at float32 rounding).
 * schedule: the order in which workgroups take bricks (results are identical
 * under every schedule): GVE_SCHED_INDEX one workgroup per brick in brick
 * order; GVE_SCHED_XCD (default) one workgroup per brick, runs of 256
 * consecutive bricks dealt to the XCDs in turn, so that each XCD's L2 holds
 * the records its bricks share; GVE_SCHED_QUEUE a persistent launch whose
 * workgroups take bricks from a work queue, heaviest first.  gve_autotune
 * measures which is fastest for a workload.
 * brick_waves: waves per brick in the fused kernel (0 or 1: one; 2 or 4 with
 * 8 x 8 columns: the waves share the brick's columns and split its
 * (primitive, brick) pairs, which puts more waves to work when a workload has
 * few bricks; the field's summation order then depends on it, within float32
 * rounding).  Evaluation alone always uses one.
 */
enum { GVE_SCHED_INDEX = 0, GVE_SCHED_XCD = 1, GVE_SCHED_QUEUE = 2 };
typedef struct gve_options {
  float k;
  int32_t brick;
  float lr, beta1, beta2, eps;
  float ell_min, ell_max;
  int32_t brick_z;
  int32_t deterministic;
  int32_t schedule;
  int32_t brick_waves;
} gve_options;

/* Counters of the most recent evaluation / refinement iteration. */
typedef struct gve_stats {
  int64_t n_primitives;   /* N */
  int64_t n_bricks;       /* bricks of the last grid */
  int64_t n_overlaps;     /* T: (primitive, brick) pairs after binning */
  int64_t n_clamped;      /* log-scale entries clamped so far (cumulative) */
  int64_t iterations;     /* Adam steps taken on the last refined params */
  double last_loss;       /* L = sum (Vhat - V)^2 of the last loss evaluation */
  /* Stage timers of the last gve_refine call (HIP events on the context's
   * stream; filled only while timing is enabled, see gve_set_timing). */
  int64_t timed_iterations;
  double ms_bin;          /* prep + scan + emit + sort + ranges */
  double ms_fused;        /* fused forward + squared error + backward kernel */
  double ms_update;       /* loss reduction + chain rule + Adam */
  /* Device scratch the context holds (pair lists, sort buffers, partials,
   * allocation and warm-start work arrays); it grows on demand and is freed
   * by gve_destroy.  Parameter sets are counted separately by the caller
   * (gve_params: 4 [11][n] arrays + a 64-byte record, 16 accumulators and
   * two counts per primitive). */
  int64_t workspace_bytes;
  /* Work of the last counting pass (gve_count_pairs, Sec. III-G): P_in =
   * (primitive, voxel) pairs with m^2 < k^2 inside the grid (the algorithmic
   * work), P_cand = lane-voxel evaluations the brick kernels perform, and the
   * (primitive, brick) pairs whose support meets their brick (one gradient
   * atomic instruction each in the default mode). */
  int64_t n_in_support;
  int64_t n_candidates;
  int64_t n_atomics;
  /* Parameters found non-finite after an Adam step (cumulative); gve_refine
   * returns GVE_ERR_NUMERIC when its steps add to it. */
  int64_t n_nonfinite;
  /* Refinements whose asynchronously sized pair buffers overflowed and that
   * were rolled back and redone with larger buffers (cumulative). */
  int64_t n_resized;
  /* Brick edge, brick depth and schedule of the last binning (with
   * options.brick = 0, the automatic choice). */
  int64_t bin_brick, bin_brick_z, bin_schedule;
  /* Primitives whose quaternion had |q| < 1e-12 at the last binning; they
   * are evaluated with the identity rotation. */
  int64_t n_degenerate_q;
  /* Waves per brick of the last binning's fused kernel (brick_waves). */
  int64_t bin_waves;
} gve_stats;

typedef struct gve_ctx gve_ctx;
typedef struct gve_params gve_params;

/* Fill *opt with k = 3, brick 8 x 8 x 32, lr = 8e-3, beta = (0.9, 0.999),
 * eps = 1e-8, no clamp, atomic gradient sums, the XCD brick schedule.  Returns INVALID_ARGUMENT if
 * opt is NULL. */
gve_status gve_default_options(gve_options* opt);

/* Create a context on the current HIP device.  hip_stream is a hipStream_t
 * borrowed from the caller (NULL = the default stream); it must outlive the
 * context.  opt NULL = defaults.  On success *out owns device scratch. */
gve_status gve_create(gve_ctx** out, const gve_options* opt, void* hip_stream);
gve_status gve_destroy(gve_ctx* ctx);
gve_status gve_set_options(gve_ctx* ctx, const gve_options* opt);
gve_status gve_get_options(const gve_ctx* ctx, gve_options* opt);

/*
 * Primitive sets.  A gve_params holds the N x 11 parameters as a device
 * structure-of-arrays [11][n] (row a = parameter a, in GVE_NPARAM order),
 * the Adam moments of the same shape and the Adam step counter.  n is fixed
 * at creation (the fixed budget of Sec. III-A); n >= 1.
 * upload/download copy the [11][n] float32 host array (and reset / keep the
 * Adam state respectively).  gve_params_device returns the device pointer of
 * the [11][n] parameter array (owned by the params; valid until destroy).
 */
gve_status gve_params_create(gve_ctx* ctx, int64_t n, gve_params** out);
gve_status gve_params_destroy(gve_params* p);
gve_status gve_params_size(const gve_params* p, int64_t* n);
gve_status gve_params_upload(gve_ctx* ctx, gve_params* p, const float* h_soa);
gve_status gve_params_download(gve_ctx* ctx, const gve_params* p, float* h_soa);
gve_status gve_params_copy_from_device(gve_ctx* ctx, gve_params* p, const float* d_soa);
gve_status gve_params_device(gve_params* p, float** d_soa);
/* Zero the Adam moments and step counter. */
gve_status gve_params_reset_adam(gve_ctx* ctx, gve_params* p);
/* Adam state access: d_m, d_v are [11][n] device arrays owned by p; t the step. */
gve_status gve_params_adam_state(gve_params* p, float** d_m, float** d_v, int64_t* t);
gve_status gve_params_set_step(gve_params* p, int64_t t);

/*
 * Truncated field evaluation (Sec. III-C eq:field; Sec. III-G truncation-aware
 * evaluation).  Writes Vhat on every voxel of g into d_out [nz][ny][nx]
 * (caller-owned, nx*ny*nz floats).  Primitives are binned to bricks by their
 * k-sigma bounding boxes; every (primitive, voxel) pair with m^2 < k^2 is
 * summed in float32, in increasing primitive index per voxel, so the result is
 * bitwise reproducible.  Errors: INVALID_ARGUMENT for null pointers or
 * non-positive sizes; DEVICE for HIP failures.
 */
gve_status gve_evaluate(gve_ctx* ctx, const gve_params* p, gve_grid g, float* d_out);

/*
 * Loss and gradient (Sec. III-F value term, as a plain squared norm over
 * every voxel of g).  L = sum_p (Vhat(p) - V(p))^2 with V = d_field [nz][ny][nx]
 * float32.  Writes dL/dtheta as [11][n] float32 into d_grad (caller-owned;
 * may be NULL to skip) with the truncation indicator held fixed, and L into
 * *h_loss if h_loss is not NULL (synchronises).  With options.deterministic
 * the gradient is bitwise reproducible; with float atomics its last bits
 * depend on execution order.
 */
gve_status gve_loss_grad(gve_ctx* ctx, const gve_params* p, const float* d_field, gve_grid g,
                         float* d_grad, double* h_loss);

/*
 * Allocation-free loss and gradient, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and errors as gve_loss_grad, but
 * every work buffer of the call (volume descriptor, pair lists, sort and scan
 * buffers, per-brick losses, deterministic partial sums) is carved from a
 * fixed device array of GVE_STATIC_SCRATCH_BYTES that the library holds on
 * each device from its first gve_create there until the process ends; the
 * call itself allocates and frees nothing.  The gradient accumulators and
 * caches of p (allocated by gve_params_create) are used as by gve_loss_grad.
 * A workload whose buffers do not fit (roughly: 16 bytes per (primitive,
 * brick) pair, 40 more with deterministic sums, plus 4 per primitive and
 * 8 per brick) returns GVE_ERR_UNSUPPORTED with the size it needs, before
 * anything is written to d_grad or *h_loss.  The array is shared by every
 * context on a device and keeps the last call's contents: calls of this
 * entry point that overlap in time on one device (other threads, or other
 * streams that have not finished) race; calls on one stream are ordered.
 */
#define GVE_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
gve_status gve_loss_grad_static(gve_ctx* ctx, const gve_params* p, const float* d_field,
                                gve_grid g, float* d_grad, double* h_loss);

/*
 * Dense reference evaluation (Sec. III-G: the cost of testing every
 * primitive-sample pair is what binning removes).  Same result as
 * gve_evaluate, Vhat on every voxel of g into d_out [nz][ny][nx] (caller-owned
 * device float32), but every (primitive, voxel) pair is evaluated and tested
 * against m^2 < k^2, with no bricks; the time grows as voxels x primitives, so
 * it is meant for small grids (a baseline for the binned path).  Per voxel the
 * sum runs in increasing primitive index.  Errors: INVALID_ARGUMENT for null
 * pointers or bad grids; UNSUPPORTED beyond 65535 * 64 primitives; DEVICE for
 * HIP failures.  Asynchronous.
 */
gve_status gve_dense_evaluate(gve_ctx* ctx, const gve_params* p, gve_grid g, float* d_out);

/*
 * Dense reference loss and gradient: gve_loss_grad's L and dL/dtheta
 * ([11][n] float32 into d_grad, caller-owned device memory, may be NULL) with
 * every (primitive, voxel) pair evaluated.  The gradient sums use float
 * atomics (last bits depend on execution order, whatever
 * options.deterministic says).  The context keeps an [nz][ny][nx] float32
 * residual buffer.  L into *h_loss if not NULL (synchronises).  Errors as
 * gve_dense_evaluate, NUMERIC for a non-finite loss.
 */
gve_status gve_dense_loss_grad(gve_ctx* ctx, const gve_params* p, const float* d_field,
                               gve_grid g, float* d_grad, double* h_loss);

/* Vector-Jacobian product of the truncated field: d_grad [11][n] (device,
 * caller-owned) = sum_p u(p) dVhat(p)/dtheta for an upstream gradient
 * u = d_upstream [nz][ny][nx] (device float32), the truncation indicator held
 * fixed.  With u = 2 (Vhat - V) this is gve_loss_grad's gradient.  It backs
 * automatic differentiation of gve_evaluate.  Asynchronous. */
gve_status gve_vjp(gve_ctx* ctx, const gve_params* p, const float* d_upstream, gve_grid g,
                   float* d_grad);

/* One bias-corrected Adam step on p from the caller's gradient d_grad [11][n]
 * (float32 device), followed by the optional log-scale clamp. */
gve_status gve_adam_step(gve_ctx* ctx, gve_params* p, const float* d_grad);

/*
 * Fixed-budget refinement (Sec. III-F; Table tab:stages row S2): iters rounds
 * of {bin, fused forward + squared-error + backward, chain rule + Adam}
 * against the target d_field on grid g.  If h_loss_hist is not NULL it
 * receives iters doubles, the loss L before each update (synchronises at the
 * end).  iters >= 0.  The primitive count never changes.
 */
gve_status gve_refine(gve_ctx* ctx, gve_params* p, const float* d_field, gve_grid g,
                      int32_t iters, double* h_loss_hist);

/*
 * Structure-aware fixed-budget allocation (Sec. III-E; stage table rows
 * S1a-S1e).  d_field: device float32 [nz][ny][nx], expected in [0, 1] (the
 * preprocessing of Sec. III-B; see gve_normalize).  Draws N_det =
 * floor(0.55 budget + 1/2) detail seeds with probability proportional to
 * |grad V| over the occupied domain V > 0.02 and N_cov = budget - N_det
 * coverage seeds uniformly over it, each draw without replacement (distinct
 * voxels), jitters them off the grid, sets per-group scales from the median
 * nearest-neighbour spacing, orients each primitive along the smallest-
 * eigenvalue axis of its 7^3 structure tensor (elongated with |grad V|,
 * capped at max(dims)/16), and sets weights kappa V(c_i) with kappa the
 * least-squares fit of the allocated field to V.  All steps run on the
 * device; the draws are reproducible from `seed`.  On success *out is a new
 * gve_params of exactly `budget` primitives (detail seeds first, each group in
 * increasing voxel order).  If the field cannot host the budget (Sec. V-B:
 * N_det > #eligible voxels or N_cov > #occupied voxels) returns
 * GVE_ERR_BUDGET_INFEASIBLE, leaves *out untouched and reports the shortfall
 * in info.  info may be NULL.  Synchronises.
 */
typedef struct gve_alloc_info {
  int64_t n_detail, n_coverage;   /* requested split of the budget */
  int64_t n_eligible, n_occupied; /* voxels with V > 0.02 and |grad V| > 0; with V > 0.02 */
  int64_t shortfall;              /* > 0 only for GVE_ERR_BUDGET_INFEASIBLE */
  double s_base_detail, s_base_coverage; /* group scales (voxels) */
  double g99;                     /* 99th percentile of |grad V| over V > 0.02 */
  double kappa;                   /* least-squares weight factor */
} gve_alloc_info;

gve_status gve_allocate(gve_ctx* ctx, const float* d_field, gve_grid g, int64_t budget,
                        uint64_t seed, gve_params** out, gve_alloc_info* info);

/* Min-max normalisation of a device float32 field of n values to [0, 1] in
 * place (Sec. III-B).  A constant field becomes 0.  Asynchronous. */
gve_status gve_normalize(gve_ctx* ctx, float* d_field, int64_t n);

/*
 * Full-precision export (Sec. III-I; Sec. III-J eq:size): a fixed header of
 * GVE_EXPORT_HEADER bytes followed by 48 bytes per primitive: twelve float32
 * (position 3, log-scale 3, quaternion w x y z 4, scalar attribute a, weight
 * w), so S_enc = 48 N + H.  This library's single weight c maps to a = c,
 * w = 1.  The header holds a magic "GVE1", version 1, N, the grid (6 int64),
 * k, the value range [vmin, vmax] of the normalised field (Sec. III-B), and a
 * default 256-entry RGBA float32 transfer-function table (grey ramp, opacity
 * equal to the value; the renderer applies its own, Sec. III-I) at byte 256;
 * the rest of the header is reserved (zero).  The header's size is the H that
 * the compression ratios printed in Sec. V-A/V-B imply (7,000 bytes).
 * gve_export writes exactly gve_export_size(n) bytes into h_buf (host,
 * caller-owned, at least that size).  gve_import creates a gve_params from
 * such a buffer (a*w becomes c) and returns its grid; INVALID_ARGUMENT for
 * a malformed buffer.  Both synchronise.
 */
#define GVE_EXPORT_HEADER 7000
size_t gve_export_size(int64_t n);
gve_status gve_export(gve_ctx* ctx, const gve_params* p, gve_grid g, float vmin, float vmax,
                      void* h_buf, size_t buf_bytes);
gve_status gve_import(gve_ctx* ctx, const void* h_buf, size_t buf_bytes, gve_params** out,
                      gve_grid* g_out);

/*
 * Checkpoint / resume (Sec. III-I: periodic checkpoints hold the full
 * primitive state and accumulated timing, so an interrupted run resumes
 * without repeating allocation).  The buffer holds parameters, both Adam
 * moments, the Adam step and the caller's accumulated seconds; resuming and
 * refining continues exactly as an uninterrupted run (bitwise with
 * deterministic gradients).  Sizes from gve_checkpoint_size(n).
 */
size_t gve_checkpoint_size(int64_t n);
gve_status gve_checkpoint_save(gve_ctx* ctx, const gve_params* p, double elapsed_s, void* h_buf,
                               size_t buf_bytes);
gve_status gve_checkpoint_load(gve_ctx* ctx, const void* h_buf, size_t buf_bytes,
                               gve_params** out, double* elapsed_s);

/* Enable (1) or disable (0) the per-stage HIP-event timers of gve_refine.
 * Timing records events between the stages of every iteration; it does not
 * add synchronisation (the elapsed times are read at the end of the call). */
gve_status gve_set_timing(gve_ctx* ctx, int32_t enable);

/*
 * Measured rates of the units that bound the brick kernels (Sec. III-G's cost
 * is these kernels), from the library's own probe kernels timed with HIP
 * events on the context's stream (median of five launches after a warm-up):
 *   fma_flops_per_s    fp32 FMA issue, eight independent chains per lane,
 *                      2 flops per FMA (non-packed instructions);
 *   exp_per_s          v_exp_f32, eight independent chains per lane;
 *   copy_bytes_per_s   a 1 GiB device copy (0.5 GiB read + 0.5 GiB written);
 *   atomic_instr_per_s float atomic instructions whose ten active lanes add
 *                      into one 64-byte line (the fused kernel's pattern),
 *                      over 2^20 distinct lines.
 * Allocates and frees 1 GiB of device memory; synchronises.  OUT_OF_MEMORY if
 * the buffer cannot be allocated, DEVICE on a launch failure.
 */
typedef struct gve_probe_rates {
  double fma_flops_per_s, exp_per_s, copy_bytes_per_s, atomic_instr_per_s;
} gve_probe_rates;
gve_status gve_probe(gve_ctx* ctx, gve_probe_rates* h_out);

/*
 * Work counters of one truncated evaluation on grid g (Sec. III-G measures the
 * same quantity: the fraction of candidate pairs that contribute).
 * *h_in_support = number of (primitive, voxel) pairs with m^2 < k^2 inside the
 * grid; *h_candidates = lane-voxel evaluations the brick kernels perform.
 * Synchronises.
 */
gve_status gve_count_pairs(gve_ctx* ctx, const gve_params* p, gve_grid g, int64_t* h_in_support,
                           int64_t* h_candidates);

/*
 * Binning inspection (Sec. III-G: primitives are binned by their k-sigma
 * support before evaluation).  Bins p on grid g exactly as gve_evaluate does
 * and reports the (brick key, value) pairs: brick keys are brick ids (x
 * fastest over the grid's bricks of the context's brick shape); values are
 * primitive ids, or with options.deterministic the pairs' emission indices.
 * d_emit_keys / d_emit_vals receive the pairs in emission order (primitive by
 * primitive, in increasing primitive id, each primitive's kept bricks
 * consecutively), d_keys / d_vals the same pairs after the stable sort by
 * brick key, d_brick_start [n_bricks + 1] the first sorted pair of each brick
 * (the last entry = the pair count).  All five are caller-owned device uint32
 * arrays; the pair arrays hold `capacity` entries.  *h_npairs and *h_nbricks
 * (host) receive the counts.  With any of the five pointers NULL only the
 * counts are returned; if the pairs do not fit in `capacity` the counts are
 * returned with INVALID_ARGUMENT and nothing is copied.  Synchronises.
 */
gve_status gve_bin_pairs(gve_ctx* ctx, const gve_params* p, gve_grid g, uint32_t* d_emit_keys,
                         uint32_t* d_emit_vals, uint32_t* d_keys, uint32_t* d_vals,
                         uint32_t* d_brick_start, int64_t capacity, int64_t* h_npairs,
                         int64_t* h_nbricks);

/*
 * Batched volumes: many uneven volumes (bricks of a larger domain, or
 * timesteps) binned together and refined in one launch per stage, every
 * (volume, brick) tile a work item of the same kernels (the work of each
 * volume is exactly that of a separate call).  A batch holds the volumes'
 * grids and one parameter set of sum(counts) primitives: volume i owns the
 * columns [prim_off[i], prim_off[i+1]) of the [11][N] layout and may only be
 * reached by its own primitives.  Fields and outputs are one concatenated
 * device buffer: volume i's voxels (x fastest) start at vox_off[i].  All
 * volumes share the Adam step counter.
 *   gve_batch_create: n_items >= 1 volumes with counts[i] >= 1 primitives
 *     (host arrays); parameters start at zero (set them with
 *     gve_batch_set_item or through gve_batch_params).
 *   gve_batch_params: the batch's parameter set (borrowed: valid until
 *     gve_batch_destroy; do not destroy it).
 *   gve_batch_offsets: prim_off and vox_off, n_items + 1 entries each (host).
 *   gve_batch_set_item: copy src (count[item] primitives) into volume item's
 *     columns and zero their Adam moments.  gve_batch_get_item: the reverse
 *     (dst's Adam state is left as is).  Both asynchronous.
 *   gve_batch_evaluate / gve_batch_loss_grad / gve_batch_refine /
 *   gve_batch_count_pairs: as the single-volume calls, over every volume;
 *   h_loss holds one loss per volume (refine: [iters][n_items]); counts are
 *   totals over the volumes.
 */
typedef struct gve_batch gve_batch;
gve_status gve_batch_create(gve_ctx* ctx, int32_t n_items, const gve_grid* h_grids,
                            const int64_t* h_counts, gve_batch** out);
void gve_batch_destroy(gve_batch* b);
gve_status gve_batch_params(gve_batch* b, gve_params** out);
gve_status gve_batch_offsets(const gve_batch* b, int64_t* h_prim_off, int64_t* h_vox_off);
gve_status gve_batch_set_item(gve_ctx* ctx, gve_batch* b, int32_t item, const gve_params* src);
gve_status gve_batch_get_item(gve_ctx* ctx, const gve_batch* b, int32_t item, gve_params* dst);
gve_status gve_batch_evaluate(gve_ctx* ctx, const gve_batch* b, float* d_out);
gve_status gve_batch_loss_grad(gve_ctx* ctx, const gve_batch* b, const float* d_fields,
                               float* d_grad, double* h_loss);
gve_status gve_batch_refine(gve_ctx* ctx, gve_batch* b, const float* d_fields, int32_t iters,
                            double* h_loss);
gve_status gve_batch_count_pairs(gve_ctx* ctx, const gve_batch* b, int64_t* h_in_support,
                                 int64_t* h_candidates);

/*
 * Autotuner: times the fused pass (binning + fused kernel + loss) under
 * every brick shape and schedule on the caller's workload (b == NULL: the
 * single volume p, d_field, g; otherwise the batch b, d_fields) for `reps`
 * passes each after one warm-up pass, keeps the fastest in the context's
 * options (with options.brick = 0 the options stay automatic and the
 * fastest becomes this workload's automatic choice), and writes one entry
 * per candidate to h_table (up to table_len;
 * *n_written = number written).  Parameters and Adam state are unchanged.
 * Results are cached in the context under a key of (volumes, voxels,
 * primitives, box coverage per voxel at 8x8x8, each rounded to a power of
 * two or half-power); a later call whose workload has the same key applies
 * the cached choice without timing and reports *n_written = 0.  Synchronises.
 */
typedef struct gve_tune_entry {
  int32_t brick, brick_z, schedule;
  float ms;  /* median over the reps */
  int32_t waves;
} gve_tune_entry;
gve_status gve_autotune(gve_ctx* ctx, const gve_params* p, const float* d_field, gve_grid g,
                        const gve_batch* b, int32_t reps, gve_tune_entry* h_table,
                        int32_t table_len, int32_t* n_written);

/*
 * The paper's own training loop (Sec. III-C eq:field, Sec. III-F, Table
 * tab:training-config), beside the sum-of-Gaussians path above.  Primitives
 * carry 12 float32 rows [12][n]: mu (3), raw quaternion w x y z (4),
 * log-scales (3), scalar attribute a, weight logit b (w = sigmoid(b)); the
 * field is Vt(p) = sum w a G / max(sum w G, rho0) with G cut at m^2 >= k^2.
 * Each iteration draws `samples` stratified points (frac_hi from voxels with
 * V > v_hi, frac_mid from v_occ < V <= v_hi, the rest uniform; a class
 * without voxels gives its share to the uniform class), jitters them by
 * U[-1/2, 1/2]^3, gives each a partner jittered by another U[-1/2, 1/2]^3,
 * and minimises
 *   sum_{V>v_occ} (Vt - V)^2 + lam_rho sum_{V>v_occ} (rho - 1)^2
 *   + lam_sm sum (rho(p) - rho(p'))^2 + lam_anc sum_i (a_i - V(mu_i))^2
 *   + lam_aniso sum_i relu(max ell - min ell - ln aniso_max)^2
 *   + lam_cap sum_ij relu(ell - ell_hi)^2 + relu(ell_lo - ell)^2
 * (V at points by trilinear interpolation; V(mu_i) held fixed), lam_sm
 * annealed linearly from lam_sm_start to lam_sm_end over the schedule, with
 * Adam (lr, beta1, beta2, eps).  The paper does not print the lambda values;
 * they are knobs.  `cell` is the edge (voxels) of the grid the sample points
 * are bucketed into.  Random draws use the counter generator of
 * gve_allocate (SplitMix64 of (seed, stream, index), streams 20-26, index
 * iter * samples + s).
 *   gve_paper_create / destroy / upload / download: the parameter set
 *     (upload resets Adam).  gve_paper_from_params: a = c / kappa (the value
 *     at the seed before the allocation's least-squares scale), weight w0.
 *   gve_paper_sample: the points of iteration `iter`: d_pts [2S][3] (samples,
 *     then partners), d_vals [S].
 *   gve_paper_eval: Vt and the density at npts points d_pts [npts][3];
 *     g is the volume the points lie in (for bucketing).
 *   gve_paper_loss_grad: objective (total to *h_loss, the six terms to
 *     h_parts[6]) and gradient [12][n] at the given points (test hook).
 *   gve_paper_refine: `iters` iterations starting at schedule position
 *     `first_iter` of a `schedule_len`-iteration schedule; h_loss[iters]
 *     gets the objective before each update.
 */
typedef struct gve_paper_options {
  float k, rho0;
  int32_t samples;
  float frac_hi, frac_mid, v_hi, v_occ;
  float lam_rho, lam_sm_start, lam_sm_end, lam_anc, lam_aniso, lam_cap;
  float aniso_max, ell_lo, ell_hi;
  float lr, beta1, beta2, eps;
  float cell;
} gve_paper_options;
typedef struct gve_paper gve_paper;
gve_status gve_paper_default_options(gve_paper_options* o);
gve_status gve_paper_create(gve_ctx* ctx, int64_t n, gve_paper** out);
void gve_paper_destroy(gve_paper* p);
gve_status gve_paper_upload(gve_ctx* ctx, gve_paper* p, const float* h_theta);
gve_status gve_paper_download(gve_ctx* ctx, const gve_paper* p, float* h_theta);
gve_status gve_paper_from_params(gve_ctx* ctx, gve_paper* p, const gve_params* src, double kappa,
                                 float w0);
gve_status gve_paper_sample(gve_ctx* ctx, const float* d_field, gve_grid g,
                            const gve_paper_options* o, uint64_t seed, int64_t iter, float* d_pts,
                            float* d_vals);
gve_status gve_paper_eval(gve_ctx* ctx, const gve_paper* p, gve_grid g, const gve_paper_options* o,
                          const float* d_pts, int64_t npts, float* d_vt, float* d_density);
gve_status gve_paper_loss_grad(gve_ctx* ctx, gve_paper* p, const float* d_field, gve_grid g,
                               const gve_paper_options* o, float lam_sm, const float* d_pts,
                               const float* d_vals, int64_t samples, float* d_grad, double* h_parts,
                               double* h_loss);
gve_status gve_paper_refine(gve_ctx* ctx, gve_paper* p, const float* d_field, gve_grid g,
                            const gve_paper_options* o, uint64_t seed, int32_t iters,
                            int32_t first_iter, int32_t schedule_len, double* h_loss);

/*
 * Learned warm start.  The paper has no learned component; this network and
 * its inputs are defined by this library (readings of the shapes it is given):
 * a multilayer perceptron 16 -> 128 -> 128 -> 11 with exact-erf GELU,
 * evaluated and trained with bfloat16 operands on the matrix cores and float32
 * accumulation, float32 master weights and Adam.  Inputs are 16 features per
 * allocated primitive (gve_features), outputs a standardised correction of its
 * 11 parameters.  The flat layout of gve_mlp_export is W1[128][16], b1[128],
 * W2[128][128], b2[128], W3[11][128], b3[11] (GVE_MLP_NWEIGHT floats), then the
 * feature mean[16] and std[16] and target mean[11] and std[11].
 */
#define GVE_MLP_NWEIGHT 20107
#define GVE_MLP_NFLAT (GVE_MLP_NWEIGHT + 54)
typedef struct gve_mlp gve_mlp;

/* He-uniform weights from `seed`, zero biases, identity standardisation. */
gve_status gve_mlp_create(gve_ctx* ctx, uint64_t seed, gve_mlp** out);
gve_status gve_mlp_destroy(gve_mlp* m);
/* Copy the network to / from a host array of GVE_MLP_NFLAT floats (synchronises). */
gve_status gve_mlp_export(gve_ctx* ctx, const gve_mlp* m, float* h_flat);
gve_status gve_mlp_import(gve_ctx* ctx, gve_mlp* m, const float* h_flat);
/* Network on standardised inputs d_X [n][16] -> d_Y [n][11] (device, caller-owned). */
gve_status gve_mlp_forward(gve_ctx* ctx, const gve_mlp* m, const float* d_X, int64_t n, float* d_Y);
/* Mean squared error of the network on standardised (d_X, d_T) and its gradient
 * d_grad [GVE_MLP_NWEIGHT] (device; may be NULL); *h_loss if not NULL. */
gve_status gve_mlp_loss_grad(gve_ctx* ctx, const gve_mlp* m, const float* d_X, const float* d_T,
                             int64_t n, float* d_grad, double* h_loss);
/* Train on raw features d_X [n][16] and raw targets d_T [n][11]: sets the
 * standardisation from the data, then `epochs` passes of Adam (lr) over
 * shuffled mini-batches of `batch` rows (shuffle seeded by `seed`).
 * h_epoch_loss (optional) receives the mean batch loss of every epoch. */
gve_status gve_mlp_train(gve_ctx* ctx, gve_mlp* m, const float* d_X, const float* d_T, int64_t n,
                         int32_t epochs, int32_t batch, float lr, uint64_t seed,
                         double* h_epoch_loss);
/* Features of an allocated primitive set on its field (see gve_allocate:
 * n_detail and g99 come from its gve_alloc_info): log1p of the 7^3
 * structure-tensor eigenvalues / g99^2 at the seed voxel round(mu) (3), the
 * eigenvectors e1, e2, e3 (9), |grad V| / g99 at the seed (1), mean and
 * variance of V over the k-sigma box (2), detail flag (1).  d_X [n][16]. */
gve_status gve_features(gve_ctx* ctx, const gve_params* p, const float* d_field, gve_grid g,
                        int64_t n_detail, double g99, float* d_X);
/* Training targets: refined - allocated parameters [n][11] with the refined
 * quaternion normalised and sign-aligned to the allocated one. */
gve_status gve_targets(gve_ctx* ctx, const gve_params* alloc, const gve_params* refined,
                       float* d_T);
/* Apply the network's correction to an allocated set: theta += alpha * delta
 * for alpha in {1, 1/2, 1/4}; keeps the first alpha whose loss L on d_field is
 * below the unchanged set's, otherwise leaves p unchanged (the plain
 * allocation is the fallback).  *applied = 0 (fallback), 1, 2 or 3 (which
 * alpha); h_losses (optional, 4 doubles) = L before and for each alpha tried
 * (NaN if not tried).  Resets p's Adam state.  Synchronises. */
gve_status gve_warmstart(gve_ctx* ctx, const gve_mlp* m, gve_params* p, const float* d_field,
                         gve_grid g, int64_t n_detail, double g99, int32_t* applied,
                         double* h_losses);

/* Counters of the last call (see gve_stats). */
gve_status gve_get_stats(const gve_ctx* ctx, gve_stats* out);

/* Static description of a status code; never NULL. */
const char* gve_status_string(gve_status s);
/* Message of the last error on ctx ("" if none); valid until the next call. */
const char* gve_last_error(const gve_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* GVE_H */
