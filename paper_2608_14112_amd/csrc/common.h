// Internal declarations shared by the HIP translation units of libgve.so.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "gve.h"

namespace gve {

// Per-primitive record written by the prep kernel and read by the field
// kernels: 16 x 32-bit = 64 bytes, one scalar-load line.  With
// A = -(log2 e / 2) Sigma^{-1}, exp(-m^2/2) = exp2(d^T A d).  Along a voxel
// column (fixed dx, dy) d^T A d is a parabola in dz with its vertex at
// dz = gx dx + gy dy and height qxy(dx, dy) = d_xy^T S d_xy, S the Schur
// complement -(log2 e / 2) (Sigma_xy)^{-1}:
//     d^T A d = qxy - (sz (dz - gx dx - gy dy))^2,  sz = sqrt(-A_zz).
//   mu[3], c, sz, s[3] = (S_xx, 2 S_xy, S_yy), gx, gy,
//   zlo, zhi : inclusive voxel z-index range of the k-sigma support box,
//   sgx = sz gx, sgy = sz gy : the slopes of w = sz t in x and y,
//   cz = exp2(-2 sz^2) : the ratio of consecutive first differences' factors
//        in the backward recurrence, the same in every brick.
// The box's x and y ranges, which only the binning reads, are BoxXY entries
// stored after the n records of a parameter set (record_boxes).
struct alignas(64) Record {
  float mu[3];
  float c;
  float sz;
  float s[3];
  float gx, gy;
  int zlo, zhi;
  float sgx, sgy;
  float cz;
  float spare;
};
static_assert(sizeof(Record) == 64, "record must be 64 bytes");

struct alignas(16) BoxXY {
  int lo[2];
  int hi[2];
};
static_assert(sizeof(BoxXY) == 16, "box must be 16 bytes");

// Bytes of a record array for n primitives: n records, then n boxes.
inline size_t record_bytes(int64_t n) { return (sizeof(Record) + sizeof(BoxXY)) * (size_t)n; }
__host__ __device__ inline BoxXY* record_boxes(Record* rec, int64_t n) {
  return reinterpret_cast<BoxXY*>(rec + n);
}
__host__ __device__ inline const BoxXY* record_boxes(const Record* rec, int64_t n) {
  return reinterpret_cast<const BoxXY*>(rec + n);
}

constexpr float kHalfLog2e = 0.72134752044448170368f;  // log2(e) / 2

// Gradient accumulators: acc[i * kAccStride + a] holds sum a (0..9) of
// primitive i, so the ten float atomics of one (primitive, brick) pair all
// fall in one 64-byte line (entries 10..15 are padding and stay zero).
constexpr int kAccStride = 16;

// One volume of a set that is binned and evaluated together (a single-volume
// call is a set of one).  Primitives [prim0, next prim0) belong to it and
// reach only its bricks [brick0, next brick0); its voxels start at `vox` in
// the concatenated field and output buffers (x fastest within the volume).
struct ItemDesc {
  int64_t nx, ny, nz, x0, y0, z0;  // the volume's grid
  int64_t vox;                     // first voxel in the concatenated buffers
  int32_t nbx, nby, nbz;           // bricks per axis
  uint32_t brick0;                 // first global brick id
  uint32_t prim0;                  // first primitive
  uint32_t pad;
};
static_assert(sizeof(ItemDesc) == 80, "ItemDesc layout");

struct Scratch {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Buffers owned by a context, grown on demand.
struct Workspace {
  Scratch keys[2], vals[2];      // (brick key, primitive id) pairs, ping-pong
  Scratch brick_start;           // uint32 [n_bricks + 1]
  Scratch brick_loss;            // float  [n_bricks]
  Scratch scan_tmp;              // scan partials
  Scratch box_off;               // uint32 [n + 1] scan of box brick counts (culling)
  Scratch owner, slot_gid;       // uint32 [T] primitive of each emission index / sorted pair
                                 // (deterministic sums)
  Scratch sort_hist;             // radix sort histograms
  Scratch dloss;                 // double [4]
  Scratch clamp_count;           // unsigned long long
  Scratch grad_tmp;              // per-iteration loss history of gve_refine
  Scratch alloc;                 // allocation scratch (block counts, indices, states)
  Scratch voxf;                  // float [M] gradient magnitude, then U
  Scratch partials;              // float [T][10] per-(primitive, brick) gradient sums
  Scratch mlp;                   // warm-start network activations and gradients
  Scratch sat;                   // double [2][M] summed-area tables of V and V^2
  Scratch feat;                  // float [n][16] features, then [n][11] network output
  Scratch theta_base;            // float [11][n] parameters before the warm start
  Scratch items;                 // ItemDesc [volumes] of the current binning
  Scratch order_keys[2], order_vals[2];  // heaviest-first brick order (queue schedule)
  Scratch queue;                 // uint32 work counter of the persistent launch
  // the paper's training loop: class block counts / offsets, sample points,
  // their float64 accumulators, gradient coefficients, cell sort, losses
  Scratch p_cls, p_pts, p_acc, p_coef, p_keys[2], p_idx[2], p_start, p_loss;
  Scratch dense;                 // float [M] residual of the dense reference path
  Scratch snap;                  // float [3][11][n] parameters and Adam moments (refinement
                                 // restart point) + counters
  void* h_pinned = nullptr;      // pinned host staging (512 bytes)
};

}  // namespace gve

struct gve_ctx {
  gve_options opt;
  hipStream_t stream = nullptr;
  int device = 0;
  gve::Workspace ws;
  gve_stats stats{};
  std::string last_error;
  bool timing = false;
  std::vector<hipEvent_t> events;  // stage-timer pool, 4 per refinement iteration
  std::vector<gve::ItemDesc> items_host;  // copy of ws.items (what the device holds)
  std::map<std::array<int, 3>, int> resident;  // (brick, depth, waves) -> resident fused workgroups
  std::map<std::array<int, 4>, std::array<int, 4>> tuned;  // autotuner cache
  // Brick shape and schedule in use while options.brick is 0 (automatic):
  // the tuned choice for the current workload once known, else 8 x 8 x 32
  // bricks in XCD chunks.  auto_choice: workload (primitive count, each
  // volume's dimensions and primitive count) -> (brick, brick_z, schedule,
  // waves per brick).
  int auto_bxy = 8, auto_bz = 32, auto_sched = GVE_SCHED_XCD, auto_waves = 1;
  std::map<std::vector<int64_t>, std::array<int, 4>> auto_choice;
  // While set, workspace buffers are carved from this fixed device region
  // (the allocation-free entry point) instead of being allocated.
  char* arena_base = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  // Capacities (box pairs, kept pairs) of the buffers of the asynchronous
  // binning inside refinement (0: not sized yet); valid for the volume
  // descriptors and brick shape they were sized for.
  int64_t box_cap = 0, pair_cap = 0;
  std::vector<gve::ItemDesc> pair_cap_items;
};

struct gve_params {
  int64_t n = 0;
  int device = 0;
  float* theta = nullptr;   // [11][n]
  float* m = nullptr;       // [11][n]
  float* v = nullptr;       // [11][n]
  float* acc = nullptr;     // [n][kAccStride] gradient partial sums (see field kernels)
  gve::Record* rec = nullptr;  // [n]
  uint32_t* count = nullptr;   // [n]   bricks overlapped per primitive
  uint32_t* offset = nullptr;  // [n+1] exclusive scan of count
  int64_t t = 0;               // Adam step
};

namespace gve {

// ---- launch wrappers (each returns hipSuccess or the launch error) ----------

// Device-wide exclusive scan of n uint32 values into out[0..n]; out[n] = total.
// tmp must hold scan_tmp_bytes(n) bytes.
size_t scan_tmp_bytes(int64_t n);
hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, void* tmp,
                              hipStream_t s);

// Stable LSD radix sort of (key, value) uint32 pairs on the low `bits` bits of
// the key.  Ping-pongs between buffers 0 and 1; returns in *which the index of
// the buffer that holds the result.  With dn, the item count is
// min(n, *dn) read on the device (n is then the buffers' capacity).  hist
// must hold sort_hist_bytes(m) bytes for some m >= n (one buffer serves every
// sort of at most m items).
size_t sort_hist_bytes(int64_t n);
hipError_t radix_sort_pairs(uint32_t* keys[2], uint32_t* vals[2], int64_t n, int bits,
                            void* hist, int* which, hipStream_t s, const uint32_t* dn = nullptr);

// Bricks are Bxy x Bxy x Bz voxels: a workgroup's lanes own the Bxy^2 voxel
// columns, each lane Bz voxels of its column.
struct BrickGeom {
  int Bxy, Bz;           // brick edges in voxels
  int64_t nbricks;       // over every volume of the set
  int waves = 1;         // fused kernel: waves per brick splitting its pairs
};


// Host: descriptors of `nitems` volumes with primitive offsets prim_off
// [nitems + 1]; returns the total brick count.
int64_t build_items(const gve_grid* grids, const int64_t* prim_off, int nitems, int Bxy, int Bz,
                    ItemDesc* out);

// Order in which workgroups take bricks.
//   kSchedIndex   : one workgroup per brick, brick = workgroup id;
//   kSchedXcd     : one workgroup per brick, consecutive bricks grouped on one
//                   XCD (workgroups are dealt round-robin over the 8 XCDs, so
//                   each XCD's L2 sees a contiguous run of bricks and of the
//                   primitives they share);
//   kSchedQueue   : persistent workgroups (as many as fit on the chip) take
//                   bricks from a counter in `order`, heaviest first.
enum { kSchedIndex = 0, kSchedXcd = 1, kSchedQueue = 2 };
struct Schedule {
  int kind = kSchedIndex;
  const uint32_t* order = nullptr;  // kSchedQueue: queue position -> brick
  uint32_t* counter = nullptr;      // kSchedQueue: zeroed before the launch
  int persistent_groups = 0;        // kSchedQueue: grid size
};

// Writes rec and count for every primitive and adds the pair total to *total
// (which the caller zeroes first, kTotalSlots + 1 counters).
// The prep kernel adds each block's box brick count to total[block % kTotalSlots]
// (64-bit): spreading the atomics over several addresses keeps them from
// queueing on one; the host sums the slots.  total[kTotalSlots] counts the
// primitives whose quaternion has |q| < 1e-12 (taken as the identity).
constexpr int kTotalSlots = 32;
hipError_t launch_prep(const float* theta, int64_t n, const ItemDesc* items, int nitems, float k,
                       BrickGeom bg, Record* rec, uint32_t* count, unsigned long long* total,
                       hipStream_t s);
// Culling: box_off = exclusive scan of prep's box brick counts; the keys of
// the box bricks a separating plane does not part from the support m^2 < k^2
// go to kept[box_off[i] ..] and their number to count[i].
// With `fits` (launch_fits), a binning whose box pairs exceed the buffers
// keeps nothing (every count 0) instead of writing past them.
hipError_t launch_cull(const Record* rec, int64_t n, const uint32_t* box_off, const ItemDesc* items,
                       int nitems, BrickGeom bg, float k, uint32_t* kept, uint32_t* count,
                       hipStream_t s, const uint32_t* fits = nullptr);
// *fits = (box pair total from prep's slots, or *count when given, <=
// capacity; with count also the previous *fits); *sticky = 1 when it does not
// (cleared by the host only); *need = max(*need, that total); a count that
// does not fit is set to 0.
hipError_t launch_fits(const unsigned long long* slots, uint32_t* count,
                       unsigned long long capacity, uint32_t* fits, uint32_t* sticky,
                       unsigned long long* need, hipStream_t s);
// Pairs at the scanned offsets from the kept keys of launch_cull; values are
// primitive ids, or with `owner` emission indices p (owner[p] = primitive).
// Nothing is written when *fits is 0.
hipError_t launch_emit(const uint32_t* offset, int64_t n, const uint32_t* box_off,
                       const uint32_t* kept, uint32_t* keys, uint32_t* vals, uint32_t* owner,
                       hipStream_t s, const uint32_t* fits = nullptr);
// gid[j] = owner[slot[j]] for j < n (n capped by *dn when given).
hipError_t launch_gather_owner(const uint32_t* owner, const uint32_t* slot, int64_t n,
                               uint32_t* gid, hipStream_t s, const uint32_t* dn = nullptr);
// brick_start[b] = first sorted pair with key >= b; npairs capped by *dn when given.
hipError_t launch_ranges(const uint32_t* sorted_keys, int64_t npairs, int64_t nbricks,
                         uint32_t* brick_start, hipStream_t s, const uint32_t* dn = nullptr);
// Heaviest-first brick order for kSchedQueue: keys = leading zeros of the
// brick's pair count (sorted ascending, stably), vals = brick ids.
hipError_t launch_order_keys(const uint32_t* brick_start, int64_t nbricks, uint32_t* keys,
                             uint32_t* vals, hipStream_t s);

// Brick shapes (Bxy, Bz) the field kernels are compiled for.
bool brick_shape_supported(int bxy, int bz);
// Waves per brick the fused kernels are compiled for with that shape (1; 2
// and 4 for 8 x 8 columns, which then split a brick's pairs).
bool brick_waves_supported(int bxy, int bz, int waves);
// Workgroups of the fused kernel that fit on the device at once.
int fused_resident_groups(int bxy, int bz, int waves, int device);
hipError_t launch_forward(const Record* rec, const uint32_t* pair_gid,
                          const uint32_t* brick_start, const ItemDesc* items, int nitems,
                          BrickGeom bg, float k, float* out, const Schedule& sc, hipStream_t s);
// part == nullptr: float atomics into acc [n][kAccStride].  Otherwise each (primitive,
// brick) pair stores its ten sums to part[pslot[j] * 10 + a], pslot[j] = the
// emission index of sorted pair j (a primitive's emission range is
// [offset[i], offset[i + 1])), which the update sums per primitive in order.
hipError_t launch_fused(const Record* rec, const uint32_t* pair_gid,
                        const uint32_t* brick_start, const ItemDesc* items, int nitems,
                        BrickGeom bg, float k, const float* field, float* acc, int64_t n,
                        float* part, const uint32_t* pslot, float* brick_loss,
                        const Schedule& sc, hipStream_t s, bool vjp = false);
hipError_t launch_count(const Record* rec, const uint32_t* pair_gid, const uint32_t* brick_start,
                        const ItemDesc* items, int nitems, BrickGeom bg, float k,
                        unsigned long long* counts, hipStream_t s);
// Sum of brick_loss in double into *out; part holds loss_reduce_tmp_doubles().
size_t loss_reduce_tmp_doubles();
hipError_t launch_loss_reduce(const float* brick_loss, int64_t nbricks, double* part, double* out,
                              hipStream_t s);
// Per-volume sums of brick_loss in double: out[i] for volume i.
hipError_t launch_item_loss(const float* brick_loss, const ItemDesc* items, int nitems,
                            int64_t nbricks, double* out, hipStream_t s);
hipError_t fill_u32(uint32_t* p, int64_t n, hipStream_t s);

// ---- dense reference path (dense.hip) ---------------------------------------
// Every (primitive, voxel) pair of grid g, no binning.  Forward: field ==
// nullptr writes Vhat to out [M]; otherwise out = 2 (Vhat - field) and
// block_loss [dense_blocks(g)] the per-block sums of (Vhat - field)^2.
// Backward: the ten gradient sums of every primitive from the residual, added
// to acc [n][kAccStride] with float atomics.  Records come from launch_prep.
int64_t dense_blocks(const gve_grid& g);
hipError_t launch_dense_forward(const Record* rec, int64_t n, const gve_grid& g, float k,
                                const float* field, float* out, float* block_loss,
                                hipStream_t s);
hipError_t launch_dense_backward(const Record* rec, int64_t n, const gve_grid& g, float k,
                                 const float* resid, float* acc, hipStream_t s);

// Rate probes (probe.hip): kProbeFma / kProbeExp run `iters` steps of
// probe_chains() independent chains per thread over `blocks` blocks of
// probe_threads() threads, writing one float per thread to buf; kProbeCopy
// copies buf[0, n/2) to buf[n/2, n) (n a multiple of 8); kProbeAtomic adds into
// buf viewed as n / kAccStride 64-byte lines, `iters` instructions per wave.
enum { kProbeFma = 0, kProbeExp = 1, kProbeCopy = 2, kProbeAtomic = 3 };
hipError_t launch_probe(int kind, float* buf, int64_t n, int iters, int blocks, hipStream_t s);
int probe_threads();
int probe_chains();

// Small utility kernels.
hipError_t fill_f32(float* p, int64_t n, float v, hipStream_t s);
hipError_t fill_u64(unsigned long long* p, int64_t n, hipStream_t s);

// ---- allocation (alloc.hip) --------------------------------------------------
size_t alloc_block_count(int64_t M);
hipError_t alloc_grad(const float* f, const gve_grid& g, float* g32, unsigned long long* counts,
                      hipStream_t s);
hipError_t alloc_set_state(unsigned long long* st, unsigned long long prefix,
                           unsigned long long rank, hipStream_t s);
hipError_t alloc_select(int mode, const float* f, const float* g32, const gve_grid& g,
                        uint64_t seed, unsigned long long* st, unsigned long long* hist,
                        uint32_t* less_cnt, uint32_t* tie_cnt, uint32_t* tie_off,
                        uint32_t* take_cnt, uint32_t* out_off, void* scan_tmp, int64_t* out,
                        hipStream_t s);
hipError_t alloc_jitter(const gve_grid& g, const int64_t* det, const int64_t* cov, int64_t n_det,
                        int64_t n, uint64_t seed, float* theta, hipStream_t s);
hipError_t alloc_spacing(const float* theta, int64_t n, int64_t first, int64_t ng, double* best,
                         double* s_base, hipStream_t s);
// J6: 6 n doubles of workspace (the seeds' structure tensors).
hipError_t alloc_assemble(const float* f, const float* g32, const gve_grid& g, const int64_t* det,
                          const int64_t* cov, int64_t n_det, int64_t n, const double* s_base,
                          const unsigned long long* g99_state, uint64_t seed, float* theta,
                          double* J6, hipStream_t s);
size_t alloc_dot_tmp_doubles();
hipError_t alloc_weights(const float* U, const float* f, int64_t M, float* c_row, int64_t n,
                         double* tmp, hipStream_t s);
size_t normalize_tmp_floats();
hipError_t normalize_field(float* f, int64_t M, float* tmp, hipStream_t s);

// ---- the paper's own training loop (paper.hip) -----------------------------------
// Uniform grid of cells (edge h voxels) over a volume, for bucketing sample
// points; points outside are clamped into the border cells.
struct CellGrid {
  float x0, y0, z0, h;
  int ncx, ncy, ncz;
};
CellGrid make_cells(const gve_grid& g, float h);
int64_t paper_class_blocks(int64_t M);
hipError_t paper_class_counts(const float* f, int64_t M, float v_hi, float v_occ, uint32_t* cnt_hi,
                              uint32_t* cnt_mid, hipStream_t s);
hipError_t paper_sample(const float* f, const gve_grid& g, const uint32_t* off_hi,
                        const uint32_t* off_mid, int S, int n_hi, int n_mid, uint64_t seed,
                        uint64_t it, float v_hi, float v_occ, float* pts, float* vals,
                        hipStream_t s);
hipError_t paper_cell_keys(const float* pts, int64_t np, const CellGrid& cg, uint32_t* keys,
                           uint32_t* idx, hipStream_t s);
hipError_t paper_zero(double* p, int64_t n, hipStream_t s);
hipError_t paper_forward(const float* th, int64_t n, const CellGrid& cg, float k, int64_t S,
                         const float* pts, const uint32_t* sorted, const uint32_t* start,
                         double* num, double* den, hipStream_t s);
hipError_t paper_density(const double* num, const double* den, int64_t np, float rho0, float* vt,
                         float* dn, hipStream_t s);
hipError_t paper_coef(int64_t S, const gve_paper_options& o, float lam_sm, const double* num,
                      const double* den, const float* vals, float* coefA, float* coefB,
                      double* loss, hipStream_t s);
hipError_t paper_backward(float* th, float* m, float* v, int64_t n, const CellGrid& cg,
                          const gve_paper_options& o, int mode, int64_t t, int64_t S,
                          const float* pts, const uint32_t* sorted, const uint32_t* start,
                          const float* coefA, const float* coefB, const float* field,
                          const gve_grid& fg, float* grad_out, double* loss, hipStream_t s);

// ---- warm-start network (mlp.hip) --------------------------------------------
hipError_t mlp_gemm(bool ta, bool tb, int epi, int M, int N, int K, const float* A, int lda,
                    const float* B, int ldb, float* C, int ldc, const float* bias, float* C2,
                    float* split_tmp, size_t split_tmp_floats, hipStream_t s);
hipError_t mlp_gelu_back(float* dH, const float* Z, int64_t n, hipStream_t s);
hipError_t mlp_colsum(const float* X, int rows, int cols, float* out, hipStream_t s);
hipError_t mlp_mse_grad(const float* Y, const float* T, int64_t n, float scale, float* dY,
                        double* part, double* acc_out, double acc_scale, hipStream_t s);
hipError_t mlp_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1,
                    float b2, float eps, int64_t t, hipStream_t s);
hipError_t mlp_colstats(const float* X, int64_t rows, int cols, float* mean, float* stdv,
                        hipStream_t s);
hipError_t mlp_standardize(const float* X, const uint32_t* perm, int64_t rows, int cols,
                           const float* mean, const float* stdv, float* out, hipStream_t s);
hipError_t mlp_perm_keys(uint32_t* keys, uint32_t* vals, int64_t n, uint64_t seed, uint64_t epoch,
                         hipStream_t s);
hipError_t mlp_sat(const float* f, const gve_grid& g, double* s1, double* s2, hipStream_t s);
// J6: 6 n doubles of workspace (the structure tensors at the centres).
hipError_t mlp_features(const float* f, const float* theta, int64_t n, int64_t n_detail,
                        const gve_grid& g, double g99, float k, const double* s1, const double* s2,
                        double* J6, float* X, hipStream_t s);
hipError_t mlp_targets(const float* ta, const float* tr, int64_t n, float* T, hipStream_t s);
hipError_t mlp_apply_delta(float* theta, const float* base, const float* Y, int64_t n,
                           const float* tmean, const float* tstd, float alpha, hipStream_t s);

// mode 0: chain rule -> grad_out ([11][n]); mode 1: chain rule + Adam;
// mode 2: Adam from grad_in.  In modes 1 and 2 clamp_count[0] counts the
// log-scale entries clamped and clamp_count[1] the parameters left non-finite.  In modes 0 and 1 the ten sums come from acc
// (zeroed after use) or, when part is given, from the primitive's partials
// part[offset[i] .. offset[i+1]) summed in order.
// With `fits` (launch_fits of this iteration's binning) the update does
// nothing when the binning did not fit its buffers.
hipError_t launch_update(int mode, float* theta, float* m, float* v, float* acc,
                         const float* part, const uint32_t* offset, const float* grad_in,
                         float* grad_out, int64_t n, int64_t t, const gve_options& opt,
                         unsigned long long* clamp_count, hipStream_t s,
                         const uint32_t* fits = nullptr);

}  // namespace gve
