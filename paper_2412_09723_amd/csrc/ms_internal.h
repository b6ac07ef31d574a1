// Internal definitions shared by the HIP translation units of libmacsplat.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "macsplat.h"

namespace ms {

// ---------------------------------------------------------------- constants
// sqrt(log2(e)/2): Mahalanobis factors are scaled so that q = d^2 log2(e)/2
// and the splat weight is o * 2^-q.
constexpr double kKappa = 0x1.b2da4e9808a53p-1;
// 4.5 log2(e): q at the 3-sigma footprint d^2 = 9.
constexpr double kQ9 = 0x1.9f7f051d0f35ep+2;
constexpr double kLog2e = 0x1.71547652b82fep+0;
constexpr double kLn2 = 0x1.62e42fefa39efp-1;
constexpr double kBoxSigmas = 3.01171875;     // 3 (1 + 2^-8)
constexpr double kDilation = 0.3;             // px^2 low-pass added to Sigma'
constexpr double kGuard = 0.65;               // 1.3 x half field of view
constexpr double kCentreLimit = 4194304.0;    // 2^22 px
constexpr double kSigma2Limit = 4194304.0;    // 2^22 px^2
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;

// Record of one visible Gaussian, 16 x 32-bit words (64 bytes), stored in
// depth-rank order. Layout documented in macsplat.h (ms_record_layout).
enum RecWord {
  R_UI = 0, R_VI = 1, R_UF = 2, R_VF = 3, R_A = 4, R_B = 5, R_C = 6, R_QCUT = 7,
  R_LO2 = 8, R_Z = 9, R_CR = 10, R_CG = 11, R_CB = 12, R_BX = 13, R_BY = 14, R_IDX = 15
};

constexpr int kGradFields = 10;   // per-rank screen-space adjoint accumulators
// 0 E = sum dL/dalpha * alpha~ (unclamped), 1 P1 = sum t1 e, 2 P2 = sum t2 e,
// 3 P1x = sum t1 e dx, 4 P1y = sum t1 e dy, 5 P2y = sum t2 e dy,
// 6-8 sum G_rgb alpha T, 9 sum G_depth alpha T.

// Device counters (uint64).
// C_ERROR: bounded waits that gave up (0 in every correct run).
enum Counter { C_VISIBLE = 0, C_PAIRS = 1, C_OVERFLOW = 2, C_ERROR = 5, C_COUNT = 8 };

// Work counters, added to once per wavefront by the compositing kernels:
// W_COMPOSITED: composited (pixel, Gaussian) pairs of the last forward;
// W_STAGED: bin-list entries walked by the forward, summed over wavefronts;
// W_REDUCED: packed list entries walked by the backward, summed over wavefronts.
// Thousands of wavefronts adding to one address serialise at the memory side
// and back up the vector memory pipeline of every CU, so each counter is
// spread over kWorkSlots 64-byte lines (slot = wavefront index mod
// kWorkSlots) and summed when the statistics are read.
enum WorkCounter { W_COMPOSITED = 0, W_STAGED = 1, W_REDUCED = 2 };
constexpr int kWorkSlots = 256;
constexpr int kWorkStride = 8;     // uint64 per slot
constexpr int kWorkBase = 32;      // uint64 offset of slot 0 from the counters array
constexpr size_t kCounterBytes = 8 * (size_t)(kWorkBase + kWorkSlots * kWorkStride);

__device__ inline void work_add(uint64_t* counters, int slot, int which, uint64_t v) {
  atomicAdd((unsigned long long*)&counters[kWorkBase + (slot & (kWorkSlots - 1)) * kWorkStride + which],
            (unsigned long long)v);
}

// ------------------------------------------------------------------ batches
// A batch renders several jobs (a map, a camera, its images) through one
// launch sequence. Job j's Gaussians take the virtual indices [g0, g0 + n)
// (g0 a multiple of kAdjSlots, so each projection block and each adjoint
// block belongs to one job), its
// compositing tiles the global tile ids [tile0, tile0 + tiles), its bins
// [bin0, bin0 + bins) and its pixels [pix0, pix0 + W*H) of the per-pixel
// arrays. The depth sort and the pair sort run once over all jobs: restricted
// to one job's Gaussians, the global (depth, index) order is that job's own
// order, and every bin belongs to one job. A single render is a batch of one.
constexpr int kMaxJobs = 12;
constexpr int kAdjSlots = 1024;   // Gaussian slots per projection-adjoint block (four per thread)
struct JobDesc {
  const float *means, *scales, *quats, *opacity, *colors;   // map, SoA [k][n]
  const float* viewmat;                                      // [12]
  float *rgb, *depth, *sil;                                  // forward outputs
  const float *g_rgb, *g_depth, *g_sil;                      // backward upstream
  float *gm, *gs, *gq, *go, *gc, *gview, *gtwist;            // backward outputs
  int64_t n, g0, pix0;
  int W, H;
  float fx, fy, cx, cy;
  int tile0, tiles, tx;      // compositing tiles
  int bin0, bins, bx;        // bins
  int block0, blocks;        // projection blocks of 256 Gaussians (block0 a multiple of kAdjSlots / 256)
  uint32_t flags;            // MS_FLAG_POSE_GRAD_ONLY / MS_FLAG_NO_POSE_GRAD for this job, kJobL1Upstream
  float l1s[3];              // kJobL1Upstream: the L1 gradient's scale of the rgb, depth, silhouette planes
};
struct JobTable {
  int njobs, pad;
  JobDesc job[kMaxJobs];
};

// Job flag (internal): the backward's upstream gradient is the L1 loss
// gradient scale * sign(pred - target), formed per pixel from the rendered
// images (rgb, depth, sil: the prediction) and the target planes, which then
// sit in g_rgb, g_depth, g_sil.
constexpr uint32_t kJobL1Upstream = 1u << 30;

// Global-address-space view of a device pointer read from a job table in
// memory. The compiler cannot tell where such a pointer points and would
// access it with flat instructions, which also count against the LDS wait
// counter, so every LDS wait would wait for them as well.
template <class T>
__device__ inline __attribute__((address_space(1))) T* global_ptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Gradient of scale * |d| with sign(0) = 0.
__host__ __device__ inline float l1_sign(float d, float sc) { return d > 0.f ? sc : (d < 0.f ? -sc : 0.f); }

// The upstream gradient of pixel `pix` of job J (P = W H).
__device__ inline void load_upstream(const JobDesc& J, int64_t pix, int64_t P, float& G0, float& G1, float& G2,
                                     float& GD, float& GS) {
  const auto g_rgb = global_ptr(J.g_rgb);
  const auto g_depth = global_ptr(J.g_depth);
  const auto g_sil = global_ptr(J.g_sil);
  if (J.flags & kJobL1Upstream) {
    const auto rgb = global_ptr(J.rgb);
    G0 = l1_sign(rgb[pix] - g_rgb[pix], J.l1s[0]);
    G1 = l1_sign(rgb[P + pix] - g_rgb[P + pix], J.l1s[0]);
    G2 = l1_sign(rgb[2 * P + pix] - g_rgb[2 * P + pix], J.l1s[0]);
    GD = l1_sign(global_ptr(J.depth)[pix] - g_depth[pix], J.l1s[1]);
    GS = l1_sign(global_ptr(J.sil)[pix] - g_sil[pix], J.l1s[2]);
  } else {
    G0 = g_rgb[pix];
    G1 = g_rgb[P + pix];
    G2 = g_rgb[2 * P + pix];
    GD = g_depth[pix];
    GS = g_sil[pix];
  }
}

// Job owning global tile `t` (tile ranges ascend with the job index).
__device__ inline int job_of_tile(const JobDesc* __restrict__ jobs, int njobs, int t) {
  int j = 0;
  for (int k = 1; k < njobs; k++)
    if (t >= jobs[k].tile0) j = k;
  return j;
}

// Job owning projection block `b`.
__device__ inline int job_of_block(const JobDesc* __restrict__ jobs, int njobs, int b) {
  int j = 0;
  for (int k = 1; k < njobs; k++)
    if (b >= jobs[k].block0) j = k;
  return j;
}

// ------------------------------------------------------------ workspace plan
// Two binning paths produce the same per-bin lists, ordered by (depth key,
// Gaussian index):
//  * per-bin sort (by_index, used when all jobs together have at most
//    kFastBins bins): pairs are counted per (unit of Gaussians, bin), placed
//    by one scan, emitted in index order and sorted by depth key inside each
//    bin; list entries are virtual Gaussian indices into the index-order
//    records rec_i, and the backward accumulators are indexed the same way;
//  * global depth sort (otherwise): the visible Gaussians are sorted by depth
//    once, pairs are emitted in rank order and sorted by bin; list entries
//    are depth ranks into the rank-order records rec.
constexpr int kFastBins = 1024;
constexpr int64_t kUnitEntries = 131072;   // bound on unit groups x bins for the single-block scan
constexpr int kUnitThreads = 256;          // binning unit: 4 waves, each `unit_rounds` rounds of 64 Gaussians
constexpr int kGroupUnits = 8;             // units per group (the scan works on group totals)

struct Plan {
  int64_t n, cap;                   // n: virtual Gaussian slots (all jobs, padded)
  int njobs;
  int tile, tiles;                  // compositing tile edge, tiles of all jobs
  int bin, bins, bshift;            // binning tiles: bin = tile << bshift; bins of all jobs
  int64_t pixels;                   // pixels of all jobs
  bool by_index;                    // per-bin sort path (see above)
  int unit_rounds, units, groups;   // per-bin path: rounds per wave of a unit, units, unit groups
  int scan_blocks_n;     // blocks of the length-n scans
  int pose_blocks;
  int rank_bits;         // bits of a depth rank (n - 1)
  bool packed;           // pairs stored as one word: tile << rank_bits | rank
  // byte offsets
  // control region (zeroed by one fill at every forward): counters, sort
  // tickets, digit histograms, look-back words, unit-group pair counts, bin
  // ranges
  size_t counters, tickets, digit_hist, lookback, gcnt, trange, ctrl_end;
  size_t jobs;           // device JobTable
  size_t key, rec_i, g2d, pose_part, tfinal, last, pkey, pval, pkey2, pval2;
  // persistent compositing: tile queue, its claim counters, per-wave list depths of the forward
  size_t order, qctr, wcost;
  // per-bin path
  size_t gbin, ucnt, uvis;
  // global depth sort path
  size_t vis_pos, ntiles, rank_of, ckey, cval, ckey2, cval2, rec, cnt, cnt_off, scan_part;
  size_t total;
};

// Records addressed by list entries (and rows of the backward accumulators).
inline size_t rec_slots(const Plan& p) { return p.by_index ? p.rec_i : p.rec; }

// Bin footprint of a visible Gaussian on the per-bin path (uint2): x = its
// first (lowest) global bin, y = (ntx - 1) | (nty - 1) << 10 | (bx - 1) << 20
// with ntx x nty bins covered and bx bins per row of its job (all <= 1024 as
// the path has at most kFastBins bins); x = 0xFFFFFFFF when culled.
constexpr uint32_t kNoBin = 0xFFFFFFFFu;

// Per-job layout (offsets of every job's slots) for options `tile`, `bin`.
bool layout_jobs(int njobs, JobTable& t, int tile, int bin, int64_t& n_virtual, int& tiles, int& bins,
                 int64_t& pixels);
// Workspace plan of a batch; lays the jobs out in `t` (their slot offsets).
bool make_plan(JobTable& t, int tile, int bin, int64_t cap, Plan& p);
// Plan of a single render (a batch of one job of n Gaussians at W x H).
bool make_plan(int64_t n, int W, int H, int tile, int bin, int64_t cap, Plan& p);

// Mask extracting the depth rank from a sorted pair word.
inline uint32_t rank_mask(const Plan& p) { return p.packed ? ((1u << p.rank_bits) - 1u) : 0xFFFFFFFFu; }

// Number of LSD passes (<= 8 bits each) for keys of `bits` significant bits.
inline int sort_passes(int bits) { return (bits + 7) / 8; }
// Significant bits of a tile id.
inline int tile_bits(int tiles) {
  int b = 0;
  while ((1 << b) < tiles) b++;
  return b;
}

// ---------------------------------------------------------------- launchers
// Every launcher enqueues on `st` and returns the launch status. The job
// table lives in the workspace (written by launch_setup).
// Writes the job table into the workspace and zeroes `count` words at `zero`.
hipError_t launch_setup(const JobTable& t, const Plan& p, char* ws, uint32_t* zero, int64_t count, hipStream_t st);
// The projection also writes the job table and zeroes `zcount` words at `zero`.
hipError_t launch_project_fwd(const Plan& p, float near_z, const JobTable& t, uint32_t* zero, int64_t zcount,
                              char* ws, hipStream_t st);
hipError_t launch_bin(const Plan& p, char* ws, hipStream_t st);
hipError_t launch_composite_fwd(const Plan& p, int wave_batch, uint32_t flags, char* ws, hipStream_t st);
// The MFMA backward (MS_FLAG_MFMA_BWD) also writes the job table `t` into the
// workspace; the other backward kernels read it from there.
hipError_t launch_composite_bwd(const Plan& p, int wave_batch, uint32_t flags, const JobTable& t, char* ws,
                                hipStream_t st);
hipError_t launch_project_bwd(const Plan& p, bool any_pose, char* ws, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* dst, uint32_t value, int64_t count, hipStream_t st);
// The L1 loss gradient of the rgb (3P), depth (P) and silhouette (P) planes
// in one launch.
hipError_t launch_l1_grad(const float* const pred[3], const float* const target[3], float* const grad[3], int64_t P,
                          const float scale[3], float* loss, hipStream_t st);
hipError_t launch_zero_scalar(float* p, hipStream_t st);
// SSIM term of the mapping loss over `C` planes of W x H (the kernel in
// ssim.hip): grad = (accumulate ? grad : 0) + d/dpred [weight (1 - mean S)],
// and *loss += weight (1 - mean S) when loss is not null. w: the 11 window
// weights; dS = -weight / (C W H).
struct SsimArgs {
  const float* pred;       // x [C][H][W]
  const float* target;     // y
  float* grad;             // dL/dx
  float* loss;
  int C, W, H, accumulate;
  float weight, dS;        // SSIM weight; dL/dS = -weight / (C W H)
  float w[11];             // window taps
  // pair form (Eq. 7 for two rendered views): grad_y != NULL
  float* grad_y;           // dL/dy
  float sl1;               // L1 scale of the channels: w_l1 / (C W H)
  const float *dx, *dy;    // depth planes [H][W]
  float *gdx, *gdy;        // their gradients
  float sgeom;             // w_geom / (W H)
};
hipError_t launch_ssim_grad(const SsimArgs& a, hipStream_t st);
// Map pruning (prune.hip): scratch bytes for n Gaussians, and the three
// launches writing the survivors into `out` (row stride *kept) and *kept.
// Stage timing of the profiler attached to the calling thread (no-ops when
// none is attached or the stage is not selected).
int prof_begin(int stage, hipStream_t st);
void prof_end(int slot, hipStream_t st);
struct StageScope {
  int slot;
  hipStream_t st;
  StageScope(int stage, hipStream_t s) : slot(prof_begin(stage, s)), st(s) {}
  ~StageScope() { prof_end(slot, st); }
};

size_t prune_workspace_bytes(int64_t n);
// One workgroup: bcount[b] (nblocks counts) becomes the exclusive offset of
// block b, *total the sum.
hipError_t launch_block_offsets(uint32_t* bcount, int64_t nblocks, int64_t* total, hipStream_t st);

// Generalized-ICP workspace plan (gicp.hip): byte offsets of its regions.
struct GicpPlan {
  int64_t nbuckets, max_src, max_tgt, nblocks;
  double cell;
  size_t bcount, fillpos, bstart, bsum, total, entries, corr, cslot, rec, eslot, partial, out, bytes;
};
GicpPlan gicp_plan(int64_t max_src, int64_t max_tgt, float d_max);
hipError_t gicp_build(const GicpPlan& p, const float* mu, int64_t n, const int32_t* idx, int64_t m, char* ws,
                      hipStream_t st);
// cslot: device int32 [n] receiving each source's grid entry (or -1), or null
hipError_t gicp_correspond(const GicpPlan& p, const float* src, int64_t n, const float* T, float d_max,
                           int32_t* corr, int32_t* cslot, char* ws, hipStream_t st);
hipError_t gicp_normal(const GicpPlan& p, const ms_map& src, const ms_map& tgt, const float* T, const int32_t* corr,
                       float eps, char* ws, hipStream_t st);
// The grid entries' target records from `tgt` (once per alignment), and the
// normal equations over the entries the last correspondence search left in
// the workspace (bit for bit those of gicp_normal with its map indices).
hipError_t gicp_records(const GicpPlan& p, const ms_map& tgt, char* ws, hipStream_t st);
hipError_t gicp_normal_records(const GicpPlan& p, const ms_map& src, const float* T, float eps, char* ws,
                               hipStream_t st);
hipError_t gicp_solve(const GicpPlan& p, int64_t n_src, float* T, double* out, double* hist, char* ws, hipStream_t st,
                      bool update);

struct SelectArgs {
  const float* means;      // [3][n]
  int64_t n;
  const float* viewmat;    // device [12]
  double fx, fy, cx, cy, near, dmax2, xmin, xmax, ymin, ymax;
};
size_t select_workspace_bytes(int64_t n);
hipError_t launch_select(const SelectArgs& a, int32_t* idx, int64_t* count, void* ws, hipStream_t st);
constexpr int64_t kPruneNoAllocMaxN = int64_t(1) << 26;   // largest map of ms_prune_noalloc
hipError_t prune_scratch(uint32_t** out);
hipError_t launch_prune(const ms_map& in, const ms_map& out, float tau_o, float tau_s, float tau_e, int64_t* kept,
                        void* ws, hipStream_t st);
hipError_t launch_pose_adam(float* viewmat, const float* g, float* state, float lr, float b1, float b2, float eps,
                            hipStream_t st);

template <typename T>
__host__ __device__ inline T* at(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

}  // namespace ms
