// Host side of the C ABI: argument validation, workspace planning and the
// launch sequence of the forward and backward passes. Allocates nothing;
// every launch goes to the caller's stream.
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ms_internal.h"

namespace ms {

namespace {

thread_local std::string g_last_error;

int32_t fail(ms_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int32_t fail(ms_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return (int32_t)s;
}

int32_t hip_fail(hipError_t e, const char* where) {
  return fail(MS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

bool valid_options(const ms_options* o) {
  return o && (o->tile == 8 || o->tile == 16 || o->tile == 32) &&
         (o->wave_batch == 32 || o->wave_batch == 64 || o->wave_batch == 128) && std::isfinite(o->near_z) &&
         o->near_z > 0.f;
}

int32_t check_common(const ms_intrinsics* intr, const ms_options* opts, int64_t n, int64_t cap) {
  if (!intr || !opts) return fail(MS_ERR_INVALID_ARG, "null intrinsics or options");
  if (intr->width < 1 || intr->width > 16384 || intr->height < 1 || intr->height > 16384)
    return fail(MS_ERR_INVALID_ARG, "image size %dx%d outside [1, 16384]", intr->width, intr->height);
  if (!(std::isfinite(intr->fx) && std::isfinite(intr->fy) && std::isfinite(intr->cx) && std::isfinite(intr->cy)) ||
      !(intr->fx > 0.f) || !(intr->fy > 0.f))
    return fail(MS_ERR_INVALID_ARG, "intrinsics must be finite with fx, fy > 0");
  if (opts->tile != 8 && opts->tile != 16 && opts->tile != 32)
    return fail(MS_ERR_UNSUPPORTED, "tile %d not in {8, 16, 32}", opts->tile);
  if (opts->wave_batch != 32 && opts->wave_batch != 64 && opts->wave_batch != 128)
    return fail(MS_ERR_UNSUPPORTED, "wave_batch %d not in {32, 64, 128}", opts->wave_batch);
  if (!valid_options(opts)) return fail(MS_ERR_INVALID_ARG, "near_z must be finite and > 0");
  if (opts->bin_tile != 0) {
    const int b = opts->bin_tile;
    if (b < opts->tile || b > 256 || (b & (b - 1)) != 0)
      return fail(MS_ERR_UNSUPPORTED, "bin_tile %d must be 0 or a power of two in [tile, 256]", b);
  }
  if (n < 0 || n > (int64_t)0x7FFFFFFF) return fail(MS_ERR_INVALID_ARG, "n = %lld outside [0, 2^31)", (long long)n);
  if (cap < 0 || cap > ((int64_t)1 << 31))
    return fail(MS_ERR_INVALID_ARG, "pair capacity %lld outside [0, 2^31]", (long long)cap);
  return MS_OK;
}

int32_t check_map(const ms_map* map) {
  if (!map) return fail(MS_ERR_INVALID_ARG, "null map");
  if (map->n > 0 && (!map->means || !map->scales || !map->quats || !map->opacity || !map->colors))
    return fail(MS_ERR_INVALID_ARG, "null map array");
  return MS_OK;
}

int32_t check_ws(const void* ws, size_t ws_bytes, const Plan& p) {
  if (!ws) return fail(MS_ERR_WORKSPACE, "null workspace");
  if (((uintptr_t)ws & 255u) != 0) return fail(MS_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < p.total)
    return fail(MS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, p.total);
  return MS_OK;
}


}  // namespace

}  // namespace ms

struct ms_profiler {
  uint32_t mask = 0;
  int cap = 0;
  int used = 0;
  std::vector<hipEvent_t> ev;   // 2 * cap
  std::vector<int> stage;       // cap
};

namespace ms {
namespace {

thread_local ms_profiler* g_prof = nullptr;

using StageTimer = StageScope;

}  // namespace

// Records the start event of a stage on `st` when the attached profiler
// selects it; returns the event slot, or -1 (also when the record fails:
// the stage then goes untimed).
int prof_begin(int stage, hipStream_t st) {
  ms_profiler* p = g_prof;
  if (!p || !(p->mask & (1u << stage)) || p->used >= p->cap) return -1;
  const int slot = p->used;
  if (hipEventRecord(p->ev[2 * slot], st) != hipSuccess) return -1;
  p->stage[slot] = stage;
  p->used++;
  return slot;
}

// A slot whose end event could not be recorded is dropped from the totals.
void prof_end(int slot, hipStream_t st) {
  if (slot >= 0 && g_prof && hipEventRecord(g_prof->ev[2 * slot + 1], st) != hipSuccess) g_prof->stage[slot] = -1;
}

bool layout_jobs(int njobs, JobTable& t, int tile, int bin, int64_t& n_virtual, int& tiles, int& bins,
                 int64_t& pixels) {
  t.njobs = njobs;
  int64_t g = 0, pix = 0;
  int tl = 0, bn = 0;
  for (int j = 0; j < njobs; j++) {
    JobDesc& J = t.job[j];
    J.g0 = g;
    J.block0 = (int)(g / 256);
    J.blocks = (int)((J.n + 255) / 256);
    g += (J.n + kAdjSlots - 1) / kAdjSlots * kAdjSlots;
    J.tx = (J.W + tile - 1) / tile;
    J.tile0 = tl;
    J.tiles = J.tx * ((J.H + tile - 1) / tile);
    tl += J.tiles;
    J.bx = (J.W + bin - 1) / bin;
    J.bin0 = bn;
    J.bins = J.bx * ((J.H + bin - 1) / bin);
    bn += J.bins;
    J.pix0 = pix;
    pix += (int64_t)J.W * J.H;
  }
  n_virtual = g;
  tiles = tl;
  bins = bn;
  pixels = pix;
  return true;
}

bool make_plan(int64_t n, int W, int H, int tile, int bin, int64_t cap, Plan& p) {
  JobTable t;
  std::memset(&t, 0, sizeof(t));
  t.job[0].n = n;
  t.job[0].W = W;
  t.job[0].H = H;
  t.njobs = 1;
  return make_plan(t, tile, bin, cap, p);
}

bool make_plan(JobTable& t, int tile, int bin, int64_t cap, Plan& p) {
  std::memset(&p, 0, sizeof(p));
  p.tile = tile;
  p.bin = bin > 0 ? bin : tile;
  p.bshift = 0;
  while ((tile << p.bshift) < p.bin) p.bshift++;
  int64_t n = 0;
  layout_jobs(t.njobs, t, tile, p.bin, n, p.tiles, p.bins, p.pixels);
  p.njobs = t.njobs;
  p.n = n;
  p.cap = cap;
  const int64_t nn = n > 0 ? n : 1;
  const int64_t cc = cap > 0 ? cap : 1;
  p.scan_blocks_n = (int)((nn + 2047) / 2048);
  p.pose_blocks = (int)((nn + kAdjSlots - 1) / kAdjSlots);
  p.rank_bits = 1;
  while (p.rank_bits < 31 && ((int64_t)1 << p.rank_bits) < nn) p.rank_bits++;
  // per-bin path: units of kUnitThreads * R Gaussians, R a power of two in
  // [2, 64] chosen so that unit groups x bins stays within the scan's bound
  if (p.bins <= kFastBins) {
    for (int r = 2; r <= 64; r *= 2) {
      const int64_t units = (nn + (int64_t)kUnitThreads * r - 1) / ((int64_t)kUnitThreads * r);
      const int64_t groups = (units + kGroupUnits - 1) / kGroupUnits;
      if (groups * p.bins <= kUnitEntries) {
        p.by_index = true;
        p.unit_rounds = r;
        p.units = (int)units;
        p.groups = (int)groups;
        break;
      }
    }
  }
  p.packed = !p.by_index && p.rank_bits + tile_bits(p.bins) <= 32;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += align_up(bytes);
    return r;
  };
  p.counters = take(kCounterBytes);
  if (!p.by_index) {
    p.tickets = take(4 * 8);                       // 2 sorts x 4 passes
    p.digit_hist = take(4 * 256 * 8);              // 2 sorts x 4 passes x 256 digits
    const int64_t os_tile = 2048;
    const int64_t tiles_v = (nn + os_tile - 1) / os_tile, tiles_p = (cc + os_tile - 1) / os_tile;
    p.lookback = take(8 * 256 * (size_t)(tiles_v > tiles_p ? tiles_v : tiles_p));
  } else {
    p.gcnt = take(4 * (size_t)p.groups * p.bins);
  }
  p.trange = take(8 * (size_t)p.bins);
  p.ctrl_end = o;
  p.key = take(4 * nn);
  p.rec_i = take(64 * nn);
  if (p.by_index) {
    p.gbin = take(8 * nn);
    p.ucnt = take(4 * (size_t)p.units * (kUnitThreads / 64) * p.bins);   // per wave
    p.uvis = take(4 * (size_t)p.units);
  } else {
    p.vis_pos = take(4 * nn);
    p.ntiles = take(4 * nn);
    p.rank_of = take(4 * nn);
    p.ckey = take(4 * nn);
    p.cval = take(4 * nn);
    p.ckey2 = take(4 * nn);
    p.cval2 = take(4 * nn);
    p.rec = take(64 * nn);
    p.cnt = take(4 * nn);
    p.cnt_off = take(8 * nn);
    p.scan_part = take(8 * (size_t)(p.scan_blocks_n + 1));
  }
  p.pkey = take(4 * cc);
  p.pval = p.packed ? p.pkey : take(4 * cc);
  p.pkey2 = take(4 * cc);
  p.pval2 = p.packed ? p.pkey2 : take(4 * cc);
  p.tfinal = take(4 * (size_t)p.pixels);
  p.last = take(4 * (size_t)p.pixels);
  p.order = take(4 * (size_t)p.tiles);
  p.qctr = take(512);   // eight claim counters on lines of their own
  p.wcost = take(4 * (size_t)p.tiles * (size_t)((tile / 8) * (tile / 8)));
  p.g2d = take(4 * (size_t)kGradFields * nn);
  p.pose_part = take(8 * 12 * (size_t)p.pose_blocks);
  p.jobs = take(sizeof(JobTable));
  p.total = o;
  return true;
}

}  // namespace ms

using namespace ms;

extern "C" {

int32_t ms_abi_version(void) { return MS_ABI_VERSION; }

const char* ms_status_string(int32_t s) {
  switch (s) {
    case MS_OK: return "ok";
    case MS_ERR_INVALID_ARG: return "invalid argument";
    case MS_ERR_CAPACITY: return "pair capacity exceeded";
    case MS_ERR_WORKSPACE: return "workspace too small or misaligned";
    case MS_ERR_HIP: return "HIP runtime error";
    case MS_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
  }
}

const char* ms_last_error(void) { return g_last_error.c_str(); }

size_t ms_workspace_bytes(int64_t n, const ms_intrinsics* intr, const ms_options* opts, int64_t pair_capacity) {
  if (check_common(intr, opts, n, pair_capacity) != MS_OK) return 0;
  Plan p;
  make_plan(n, intr->width, intr->height, opts->tile, opts->bin_tile, pair_capacity, p);
  return p.total;
}

}  // extern "C"

namespace ms {
namespace {

JobDesc job_from_map(const ms_map& map, const float* viewmat, const ms_intrinsics& intr) {
  JobDesc J;
  std::memset(&J, 0, sizeof(J));
  J.means = map.means;
  J.scales = map.scales;
  J.quats = map.quats;
  J.opacity = map.opacity;
  J.colors = map.colors;
  J.viewmat = viewmat;
  J.n = map.n;
  J.W = intr.width;
  J.H = intr.height;
  J.fx = intr.fx;
  J.fy = intr.fy;
  J.cx = intr.cx;
  J.cy = intr.cy;
  return J;
}

// The forward launch sequence over a job table (outputs set in the table).
int32_t run_forward(JobTable& t, const ms_options* opts, void* workspace, size_t ws_bytes, int64_t cap,
                    hipStream_t st) {
  Plan p;
  make_plan(t, opts->tile, opts->bin_tile, cap, p);
  int32_t s = check_ws(workspace, ws_bytes, p);
  if (s != MS_OK) return s;
  char* ws = (char*)workspace;
  // the projection writes the job table and zeroes the control region; with
  // no Gaussians a separate launch does both
  uint32_t* ctrl = at<uint32_t>(ws, p.counters);
  const int64_t ctrl_words = (int64_t)((p.ctrl_end - p.counters) / 4);
  hipError_t e = hipSuccess;
  if (p.n == 0) {
    e = launch_setup(t, p, ws, ctrl, ctrl_words, st);
    if (e != hipSuccess) return hip_fail(e, "counters");
  }
  {
    StageTimer tm(MS_STAGE_PROJECT, st);
    e = launch_project_fwd(p, opts->near_z, t, ctrl, ctrl_words, ws, st);
  }
  if (e != hipSuccess) return hip_fail(e, "project");
  {
    StageTimer tm(MS_STAGE_BIN, st);
    e = launch_bin(p, ws, st);
  }
  if (e != hipSuccess) return hip_fail(e, "bin");
  {
    StageTimer tm(MS_STAGE_COMPOSITE, st);
    e = launch_composite_fwd(p, opts->wave_batch, opts->flags, ws, st);
  }
  if (e != hipSuccess) return hip_fail(e, "composite");
  return MS_OK;
}

// The backward launch sequence over a job table (upstream and gradient
// pointers and per-job flags set in the table).
int32_t run_backward(JobTable& t, const ms_options* opts, void* workspace, size_t ws_bytes, int64_t cap,
                     hipStream_t st) {
  Plan p;
  make_plan(t, opts->tile, opts->bin_tile, cap, p);
  int32_t s = check_ws(workspace, ws_bytes, p);
  if (s != MS_OK) return s;
  char* ws = (char*)workspace;
  bool any_pose = false;
  for (int j = 0; j < t.njobs; j++) any_pose |= !(t.job[j].flags & MS_FLAG_NO_POSE_GRAD);
  // the global depth-sort path zeroes its accumulator rows here; on the
  // per-bin path the rows of the visible Gaussians are zeroed by the
  // projection and again by the projection adjoint after use, and the MFMA
  // backward writes the job table itself
  hipError_t e = hipSuccess;
  if (!(p.by_index && (opts->flags & MS_FLAG_MFMA_BWD) && p.tiles > 0)) {
    e = launch_setup(t, p, ws, at<uint32_t>(ws, p.g2d), p.by_index ? 0 : (int64_t)kGradFields * p.n, st);
    if (e != hipSuccess) return hip_fail(e, "job table");
  }
  {
    StageTimer tm(MS_STAGE_COMPOSITE_BWD, st);
    e = launch_composite_bwd(p, opts->wave_batch, opts->flags, t, ws, st);
  }
  if (e != hipSuccess) return hip_fail(e, "composite backward");
  {
    StageTimer tm(MS_STAGE_PROJECT_BWD, st);
    e = launch_project_bwd(p, any_pose, ws, st);
  }
  if (e != hipSuccess) return hip_fail(e, "project backward");
  return MS_OK;
}

int32_t check_backward_job(const ms_map& map, const ms_images* grad_out, const ms_grads* grads, uint32_t flags) {
  if (!grad_out || !grad_out->rgb || !grad_out->depth || !grad_out->silhouette)
    return fail(MS_ERR_INVALID_ARG, "null upstream gradient image");
  if (!grads) return fail(MS_ERR_INVALID_ARG, "null gradients");
  const bool map_g = !(flags & MS_FLAG_POSE_GRAD_ONLY);
  const bool pose_g = !(flags & MS_FLAG_NO_POSE_GRAD);
  if (map_g && map.n > 0 && (!grads->means || !grads->scales || !grads->quats || !grads->opacity || !grads->colors))
    return fail(MS_ERR_INVALID_ARG, "null map gradient array");
  if (pose_g && (!grads->viewmat || !grads->twist)) return fail(MS_ERR_INVALID_ARG, "null pose gradient");
  return MS_OK;
}

void set_backward_job(JobDesc& J, const ms_images& grad_out, const ms_grads& g, uint32_t flags) {
  J.g_rgb = grad_out.rgb;
  J.g_depth = grad_out.depth;
  J.g_sil = grad_out.silhouette;
  J.gm = g.means;
  J.gs = g.scales;
  J.gq = g.quats;
  J.go = g.opacity;
  J.gc = g.colors;
  J.gview = g.viewmat;
  J.gtwist = g.twist;
  J.flags = flags & (MS_FLAG_POSE_GRAD_ONLY | MS_FLAG_NO_POSE_GRAD | MS_FLAG_ACCUMULATE_MAP_GRADS);
}

constexpr uint32_t kPoseFlags = MS_FLAG_POSE_GRAD_ONLY | MS_FLAG_NO_POSE_GRAD;

// Validates a batch and fills the job table (images of the forward, or
// upstream and gradients of the backward).
int32_t batch_table(int32_t njobs, const ms_job* jobs, const ms_options* opts, int64_t cap, bool backward,
                    JobTable& t) {
  if (njobs < 1 || njobs > kMaxJobs) return fail(MS_ERR_INVALID_ARG, "njobs %d outside [1, %d]", njobs, kMaxJobs);
  if (!jobs) return fail(MS_ERR_INVALID_ARG, "null job array");
  std::memset(&t, 0, sizeof(t));
  t.njobs = njobs;
  for (int j = 0; j < njobs; j++) {
    const ms_job& b = jobs[j];
    int32_t s = check_map(&b.map);
    if (s == MS_OK) s = check_common(&b.intr, opts, b.map.n, cap);
    if (s != MS_OK) return s;
    if (!b.viewmat) return fail(MS_ERR_INVALID_ARG, "job %d: null viewmat", j);
    t.job[j] = job_from_map(b.map, b.viewmat, b.intr);
    if (backward) {
      const uint32_t flags = b.flags | (opts->flags & kPoseFlags);
      s = check_backward_job(b.map, &b.grad_out, &b.grads, flags);
      if (s != MS_OK) return s;
      set_backward_job(t.job[j], b.grad_out, b.grads, flags);
    } else {
      if (!b.out.rgb || !b.out.depth || !b.out.silhouette)
        return fail(MS_ERR_INVALID_ARG, "job %d: null output image", j);
      t.job[j].rgb = b.out.rgb;
      t.job[j].depth = b.out.depth;
      t.job[j].sil = b.out.silhouette;
    }
  }
  if (backward) {
    // map gradient arrays written by more than one job must be accumulated
    // by all of them (plain writes of one job would race with the others)
    for (int j = 0; j < njobs; j++) {
      const JobDesc& A = t.job[j];
      if ((A.flags & MS_FLAG_POSE_GRAD_ONLY) || A.n == 0) continue;
      for (int k = j + 1; k < njobs; k++) {
        const JobDesc& B = t.job[k];
        if ((B.flags & MS_FLAG_POSE_GRAD_ONLY) || B.n == 0) continue;
        const float* a[5] = {A.gm, A.gs, A.gq, A.go, A.gc};
        const float* b[5] = {B.gm, B.gs, B.gq, B.go, B.gc};
        bool shared = false;
        for (int u = 0; u < 5; u++)
          for (int v = 0; v < 5; v++) shared |= a[u] == b[v];
        if (shared && !((A.flags & B.flags) & MS_FLAG_ACCUMULATE_MAP_GRADS))
          return fail(MS_ERR_INVALID_ARG, "jobs %d and %d share a map gradient array without MS_FLAG_ACCUMULATE_MAP_GRADS",
                      j, k);
        if (shared && A.n != B.n)
          return fail(MS_ERR_INVALID_ARG, "jobs %d and %d share map gradient arrays but not the map size", j, k);
      }
    }
  }
  int64_t total = 0;
  for (int j = 0; j < njobs; j++) total += (jobs[j].map.n + kAdjSlots - 1) / kAdjSlots * kAdjSlots;
  if (total > (int64_t)0x7FFFFFFF) return fail(MS_ERR_INVALID_ARG, "batch of %lld Gaussian slots", (long long)total);
  return MS_OK;
}

}  // namespace
}  // namespace ms

extern "C" {

int32_t ms_forward(const ms_map* map, const float* viewmat, const ms_intrinsics* intr, const ms_options* opts,
                   void* workspace, size_t ws_bytes, int64_t pair_capacity, const ms_images* out, void* stream) {
  int32_t s = check_map(map);
  if (s != MS_OK) return s;
  s = check_common(intr, opts, map->n, pair_capacity);
  if (s != MS_OK) return s;
  if (!viewmat) return fail(MS_ERR_INVALID_ARG, "null viewmat");
  if (!out || !out->rgb || !out->depth || !out->silhouette) return fail(MS_ERR_INVALID_ARG, "null output image");
  JobTable t;
  std::memset(&t, 0, sizeof(t));
  t.njobs = 1;
  t.job[0] = job_from_map(*map, viewmat, *intr);
  t.job[0].rgb = out->rgb;
  t.job[0].depth = out->depth;
  t.job[0].sil = out->silhouette;
  return run_forward(t, opts, workspace, ws_bytes, pair_capacity, (hipStream_t)stream);
}

int32_t ms_backward(const ms_map* map, const float* viewmat, const ms_intrinsics* intr, const ms_options* opts,
                    void* workspace, size_t ws_bytes, int64_t pair_capacity, const ms_images* grad_out,
                    const ms_grads* grads, void* stream) {
  int32_t s = check_map(map);
  if (s != MS_OK) return s;
  s = check_common(intr, opts, map->n, pair_capacity);
  if (s != MS_OK) return s;
  if (!viewmat) return fail(MS_ERR_INVALID_ARG, "null viewmat");
  s = check_backward_job(*map, grad_out, grads, opts->flags);
  if (s != MS_OK) return s;
  JobTable t;
  std::memset(&t, 0, sizeof(t));
  t.njobs = 1;
  t.job[0] = job_from_map(*map, viewmat, *intr);
  set_backward_job(t.job[0], *grad_out, *grads, opts->flags);
  return run_backward(t, opts, workspace, ws_bytes, pair_capacity, (hipStream_t)stream);
}

int32_t ms_backward_l1(const ms_map* map, const float* viewmat, const ms_intrinsics* intr, const ms_options* opts,
                       void* workspace, size_t ws_bytes, int64_t pair_capacity, const ms_images* pred,
                       const ms_images* target, float w_rgb, float w_depth, float w_sil, const ms_grads* grads,
                       void* stream) {
  int32_t s = check_map(map);
  if (s != MS_OK) return s;
  s = check_common(intr, opts, map->n, pair_capacity);
  if (s != MS_OK) return s;
  if (!viewmat) return fail(MS_ERR_INVALID_ARG, "null viewmat");
  if (!pred || !pred->rgb || !pred->depth || !pred->silhouette)
    return fail(MS_ERR_INVALID_ARG, "null rendered image");
  if (!std::isfinite(w_rgb) || !std::isfinite(w_depth) || !std::isfinite(w_sil))
    return fail(MS_ERR_INVALID_ARG, "non-finite loss weight");
  s = check_backward_job(*map, target, grads, opts->flags);   // target in the upstream's place
  if (s != MS_OK) return s;
  JobTable t;
  std::memset(&t, 0, sizeof(t));
  t.njobs = 1;
  t.job[0] = job_from_map(*map, viewmat, *intr);
  set_backward_job(t.job[0], *target, *grads, opts->flags);
  JobDesc& J = t.job[0];
  J.rgb = pred->rgb;
  J.depth = pred->depth;
  J.sil = pred->silhouette;
  // the scales of ms_l1_loss_grad, so that both paths form the same upstream
  const int64_t P = (int64_t)intr->width * intr->height;
  J.l1s[0] = w_rgb / (3.0f * (float)P);
  J.l1s[1] = w_depth / (float)P;
  J.l1s[2] = w_sil / (float)P;
  J.flags |= kJobL1Upstream;
  return run_backward(t, opts, workspace, ws_bytes, pair_capacity, (hipStream_t)stream);
}

size_t ms_batch_workspace_bytes(int32_t njobs, const ms_job* jobs, const ms_options* opts, int64_t pair_capacity) {
  if (!opts) return 0;
  if (njobs < 1 || njobs > kMaxJobs || !jobs) return 0;
  JobTable t;
  std::memset(&t, 0, sizeof(t));
  t.njobs = njobs;
  for (int j = 0; j < njobs; j++) {
    if (check_common(&jobs[j].intr, opts, jobs[j].map.n, pair_capacity) != MS_OK) return 0;
    t.job[j] = job_from_map(jobs[j].map, jobs[j].viewmat, jobs[j].intr);
  }
  Plan p;
  make_plan(t, opts->tile, opts->bin_tile, pair_capacity, p);
  return p.total;
}

int32_t ms_forward_batch(int32_t njobs, const ms_job* jobs, const ms_options* opts, void* workspace, size_t ws_bytes,
                         int64_t pair_capacity, void* stream) {
  JobTable t;
  int32_t s = batch_table(njobs, jobs, opts, pair_capacity, false, t);
  if (s != MS_OK) return s;
  return run_forward(t, opts, workspace, ws_bytes, pair_capacity, (hipStream_t)stream);
}

int32_t ms_backward_batch(int32_t njobs, const ms_job* jobs, const ms_options* opts, void* workspace,
                          size_t ws_bytes, int64_t pair_capacity, void* stream) {
  JobTable t;
  int32_t s = batch_table(njobs, jobs, opts, pair_capacity, true, t);
  if (s != MS_OK) return s;
  return run_backward(t, opts, workspace, ws_bytes, pair_capacity, (hipStream_t)stream);
}

}  // extern "C"

namespace ms {
namespace {

int32_t read_stats(const void* workspace, size_t ws_bytes, const Plan& p, int64_t out[7], hipStream_t st) {
  int32_t s = check_ws(workspace, ws_bytes, p);
  if (s != MS_OK) return s;
  std::vector<uint64_t> c(kCounterBytes / 8);
  hipError_t e = hipMemcpyAsync(c.data(), (const char*)workspace + p.counters, kCounterBytes, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "read stats");
  uint64_t w[3] = {0, 0, 0};
  for (int slot = 0; slot < kWorkSlots; slot++)
    for (int k = 0; k < 3; k++) w[k] += c[kWorkBase + slot * kWorkStride + k];
  out[0] = (int64_t)c[C_VISIBLE];
  out[1] = (int64_t)c[C_PAIRS];
  out[2] = (int64_t)c[C_OVERFLOW];
  out[3] = p.bins;
  out[4] = (int64_t)w[W_COMPOSITED];
  out[5] = (int64_t)w[W_STAGED];
  out[6] = (int64_t)w[W_REDUCED];
  if (c[C_ERROR]) return fail(MS_ERR_HIP, "a bounded device wait gave up %llu time(s)", (unsigned long long)c[C_ERROR]);
  return MS_OK;
}

}  // namespace
}  // namespace ms

extern "C" {

int32_t ms_read_stats(const void* workspace, size_t ws_bytes, int64_t n, const ms_intrinsics* intr,
                      const ms_options* opts, int64_t pair_capacity, int64_t out[7], void* stream) {
  int32_t s = check_common(intr, opts, n, pair_capacity);
  if (s != MS_OK) return s;
  if (!out) return fail(MS_ERR_INVALID_ARG, "null output");
  Plan p;
  make_plan(n, intr->width, intr->height, opts->tile, opts->bin_tile, pair_capacity, p);
  return read_stats(workspace, ws_bytes, p, out, (hipStream_t)stream);
}

int32_t ms_batch_read_stats(int32_t njobs, const ms_job* jobs, const ms_options* opts, const void* workspace,
                            size_t ws_bytes, int64_t pair_capacity, int64_t out[7], void* stream) {
  if (!out) return fail(MS_ERR_INVALID_ARG, "null output");
  if (!opts || njobs < 1 || njobs > kMaxJobs || !jobs) return fail(MS_ERR_INVALID_ARG, "bad batch");
  JobTable t;
  std::memset(&t, 0, sizeof(t));
  t.njobs = njobs;
  for (int j = 0; j < njobs; j++) {
    int32_t s = check_common(&jobs[j].intr, opts, jobs[j].map.n, pair_capacity);
    if (s != MS_OK) return s;
    t.job[j] = job_from_map(jobs[j].map, jobs[j].viewmat, jobs[j].intr);
  }
  Plan p;
  make_plan(t, opts->tile, opts->bin_tile, pair_capacity, p);
  return read_stats(workspace, ws_bytes, p, out, (hipStream_t)stream);
}

int32_t ms_state_view_get(void* workspace, size_t ws_bytes, int64_t n, const ms_intrinsics* intr,
                          const ms_options* opts, int64_t pair_capacity, ms_state_view* v) {
  int32_t s = check_common(intr, opts, n, pair_capacity);
  if (s != MS_OK) return s;
  if (!v) return fail(MS_ERR_INVALID_ARG, "null view");
  Plan p;
  make_plan(n, intr->width, intr->height, opts->tile, opts->bin_tile, pair_capacity, p);
  s = check_ws(workspace, ws_bytes, p);
  if (s != MS_OK) return s;
  char* ws = (char*)workspace;
  v->depth_key = at<uint32_t>(ws, p.key);
  v->sorted_index = p.by_index ? nullptr : at<uint32_t>(ws, p.cval);
  v->rank_of = p.by_index ? nullptr : at<int32_t>(ws, p.rank_of);
  v->pair_tile = p.by_index ? nullptr : at<uint32_t>(ws, p.pkey);
  v->pair_rank = at<uint32_t>(ws, p.pval);
  v->tile_range = at<uint32_t>(ws, p.trange);
  v->records = at<float>(ws, rec_slots(p));
  v->list_kind = p.by_index ? 1 : 0;
  v->tfinal = at<float>(ws, p.tfinal);
  v->last = at<uint32_t>(ws, p.last);
  v->counters = at<uint64_t>(ws, p.counters);
  v->grad2d = at<float>(ws, p.g2d);
  v->pair_rank_bits = p.packed ? p.rank_bits : 0;
  v->tile_order = at<uint32_t>(ws, p.order);
  v->tile_cost = at<uint32_t>(ws, p.wcost);
  v->tiles = p.tiles;
  v->tile_waves = (p.tile / 8) * (p.tile / 8);
  return MS_OK;
}

int32_t ms_l1_loss_grad(const ms_images* pred, const ms_images* target, const ms_intrinsics* intr, float w_rgb,
                        float w_depth, float w_sil, const ms_images* grad, float* loss, void* stream) {
  if (!pred || !target || !grad || !intr) return fail(MS_ERR_INVALID_ARG, "null argument");
  if (!pred->rgb || !pred->depth || !pred->silhouette || !target->rgb || !target->depth || !target->silhouette ||
      !grad->rgb || !grad->depth || !grad->silhouette)
    return fail(MS_ERR_INVALID_ARG, "null image");
  if (intr->width < 1 || intr->width > 16384 || intr->height < 1 || intr->height > 16384)
    return fail(MS_ERR_INVALID_ARG, "image size %dx%d outside [1, 16384]", intr->width, intr->height);
  if (!std::isfinite(w_rgb) || !std::isfinite(w_depth) || !std::isfinite(w_sil))
    return fail(MS_ERR_INVALID_ARG, "non-finite loss weight");
  hipStream_t st = (hipStream_t)stream;
  const int64_t P = (int64_t)intr->width * intr->height;
  hipError_t e = hipSuccess;
  if (loss) e = launch_zero_scalar(loss, st);
  if (e == hipSuccess) {
    const float* pr[3] = {pred->rgb, pred->depth, pred->silhouette};
    const float* tg[3] = {target->rgb, target->depth, target->silhouette};
    float* gr[3] = {grad->rgb, grad->depth, grad->silhouette};
    const float sc[3] = {w_rgb / (3.0f * (float)P), w_depth / (float)P, w_sil / (float)P};
    StageTimer tm(MS_STAGE_LOSS, st);
    e = launch_l1_grad(pr, tg, gr, P, sc, loss, st);
  }
  if (e != hipSuccess) return hip_fail(e, "l1 loss");
  return MS_OK;
}

namespace {
void ssim_window(float out[11]);
bool means_overlap(const void* a, size_t abytes, const void* b, size_t bbytes);
}  // namespace

int32_t ms_ssim_loss_grad(const float* pred, const float* target, int32_t channels, int32_t width, int32_t height,
                          float weight, float* grad, int32_t accumulate, float* loss, void* stream) {
  if (!pred || !target || !grad) return fail(MS_ERR_INVALID_ARG, "null argument");
  if (channels < 1 || channels > 16) return fail(MS_ERR_INVALID_ARG, "channels = %d outside [1, 16]", channels);
  if (width < 1 || width > 16384 || height < 1 || height > 16384)
    return fail(MS_ERR_INVALID_ARG, "image size %dx%d outside [1, 16384]", width, height);
  if (!std::isfinite(weight)) return fail(MS_ERR_INVALID_ARG, "non-finite loss weight");
  if (accumulate != 0 && accumulate != 1) return fail(MS_ERR_INVALID_ARG, "accumulate must be 0 or 1");
  {
    // every workgroup reads a halo of neighbouring pixels: a gradient written
    // over an input would race with those reads
    const size_t bytes = (size_t)channels * (size_t)width * (size_t)height * sizeof(float);
    const uintptr_t g0 = (uintptr_t)grad, g1 = g0 + bytes;
    const uintptr_t p0 = (uintptr_t)pred, t0 = (uintptr_t)target;
    if ((g0 < p0 + bytes && p0 < g1) || (g0 < t0 + bytes && t0 < g1))
      return fail(MS_ERR_INVALID_ARG, "grad overlaps pred or target");
  }
  hipStream_t st = (hipStream_t)stream;
  SsimArgs a;
  std::memset(&a, 0, sizeof(a));
  a.pred = pred;
  a.target = target;
  a.grad = grad;
  a.loss = loss;
  a.C = channels;
  a.W = width;
  a.H = height;
  a.accumulate = accumulate;
  a.weight = weight;
  a.dS = (float)(-(double)weight / ((double)channels * (double)width * (double)height));
  ssim_window(a.w);
  hipError_t e = hipSuccess;
  StageTimer tm(MS_STAGE_LOSS, st);
  if (loss && !accumulate) e = launch_zero_scalar(loss, st);
  if (e == hipSuccess) e = launch_ssim_grad(a, st);
  if (e != hipSuccess) return hip_fail(e, "ssim loss");
  return MS_OK;
}

int32_t ms_pair_loss_grad(const float* rgb_i, const float* rgb_j, const float* depth_i, const float* depth_j,
                          int32_t width, int32_t height, float w_l1, float w_ssim, float w_geom, float* g_rgb_i,
                          float* g_rgb_j, float* g_depth_i, float* g_depth_j, int32_t accumulate, float* loss,
                          void* stream) {
  if (!rgb_i || !rgb_j || !depth_i || !depth_j || !g_rgb_i || !g_rgb_j || !g_depth_i || !g_depth_j)
    return fail(MS_ERR_INVALID_ARG, "null argument");
  if (width < 1 || width > 16384 || height < 1 || height > 16384)
    return fail(MS_ERR_INVALID_ARG, "image size %dx%d outside [1, 16384]", width, height);
  if (!std::isfinite(w_l1) || !std::isfinite(w_ssim) || !std::isfinite(w_geom))
    return fail(MS_ERR_INVALID_ARG, "non-finite loss weight");
  if (accumulate != 0 && accumulate != 1) return fail(MS_ERR_INVALID_ARG, "accumulate must be 0 or 1");
  const size_t P = (size_t)width * (size_t)height;
  const void* ins[4] = {rgb_i, rgb_j, depth_i, depth_j};
  const size_t inb[4] = {3 * P * 4, 3 * P * 4, P * 4, P * 4};
  const void* outs[4] = {g_rgb_i, g_rgb_j, g_depth_i, g_depth_j};
  for (int o = 0; o < 4; o++) {
    for (int i = 0; i < 4; i++)   // the window reads neighbouring pixels of every input
      if (means_overlap(outs[o], inb[o], ins[i], inb[i])) return fail(MS_ERR_INVALID_ARG, "gradient overlaps an input");
    for (int q = o + 1; q < 4; q++)
      if (means_overlap(outs[o], inb[o], outs[q], inb[q])) return fail(MS_ERR_INVALID_ARG, "gradients overlap");
  }
  hipStream_t st = (hipStream_t)stream;
  SsimArgs a;
  std::memset(&a, 0, sizeof(a));
  a.pred = rgb_i;
  a.target = rgb_j;
  a.grad = g_rgb_i;
  a.grad_y = g_rgb_j;
  a.loss = loss;
  a.C = 3;
  a.W = width;
  a.H = height;
  a.accumulate = accumulate;
  a.weight = w_ssim;
  a.dS = (float)(-(double)w_ssim / (3.0 * (double)P));
  a.sl1 = (float)((double)w_l1 / (3.0 * (double)P));
  a.dx = depth_i;
  a.dy = depth_j;
  a.gdx = g_depth_i;
  a.gdy = g_depth_j;
  a.sgeom = (float)((double)w_geom / (double)P);
  ssim_window(a.w);
  hipError_t e = hipSuccess;
  StageTimer tm(MS_STAGE_LOSS, st);
  if (loss && !accumulate) e = launch_zero_scalar(loss, st);
  if (e == hipSuccess) e = launch_ssim_grad(a, st);
  if (e != hipSuccess) return hip_fail(e, "pair loss");
  return MS_OK;
}

size_t ms_prune_workspace_bytes(int64_t n) { return n < 0 ? 0 : prune_workspace_bytes(n); }

namespace {
// Gaussian window of the SSIM statistics, standard deviation 1.5 px,
// normalised in binary64.
void ssim_window(float out[11]) {
  double wsum = 0.0, w[11];
  for (int k = 0; k < 11; k++) {
    const double d = k - 5;
    w[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    wsum += w[k];
  }
  for (int k = 0; k < 11; k++) out[k] = (float)(w[k] / wsum);
}

bool means_overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + bbytes && b0 < a0 + abytes;
}

// Host checks shared by ms_prune and ms_prune_noalloc.
int32_t check_prune(const ms_map* in, float tau_o, float tau_s, float tau_e, const ms_map* out, const int64_t* kept) {
  int32_t s = check_map(in);
  if (s != MS_OK) return s;
  if (in->n < 0) return fail(MS_ERR_INVALID_ARG, "n = %lld < 0", (long long)in->n);
  if (!out || !kept) return fail(MS_ERR_INVALID_ARG, "null output");
  if (in->n > 0 && (!out->means || !out->scales || !out->quats || !out->opacity || !out->colors))
    return fail(MS_ERR_INVALID_ARG, "null output array");
  if (out->n < in->n) return fail(MS_ERR_INVALID_ARG, "output capacity %lld < n = %lld", (long long)out->n, (long long)in->n);
  const float* ia[5] = {in->means, in->scales, in->quats, in->opacity, in->colors};
  const float* oa[5] = {out->means, out->scales, out->quats, out->opacity, out->colors};
  for (int u = 0; u < 5 && in->n > 0; u++)
    for (int v = 0; v < 5; v++)
      if (ia[u] == oa[v]) return fail(MS_ERR_INVALID_ARG, "output array aliases an input array");
  if (!std::isfinite(tau_o) || !std::isfinite(tau_s) || !std::isfinite(tau_e) || tau_e < 0.f)
    return fail(MS_ERR_INVALID_ARG, "thresholds must be finite and tau_e >= 0");
  return MS_OK;
}
}  // namespace

int32_t ms_prune(const ms_map* in, float tau_o, float tau_s, float tau_e, const ms_map* out, int64_t* kept,
                 void* workspace, size_t ws_bytes, void* stream) {
  int32_t s = check_prune(in, tau_o, tau_s, tau_e, out, kept);
  if (s != MS_OK) return s;
  if (!workspace) return fail(MS_ERR_WORKSPACE, "null workspace");
  if (ws_bytes < prune_workspace_bytes(in->n)) return fail(MS_ERR_WORKSPACE, "workspace too small");
  hipError_t e = launch_prune(*in, *out, tau_o, tau_s, tau_e, kept, workspace, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "prune");
  return MS_OK;
}

int32_t ms_prune_noalloc(const ms_map* in, float tau_o, float tau_s, float tau_e, const ms_map* out, int64_t* kept,
                         void* stream) {
  int32_t s = check_prune(in, tau_o, tau_s, tau_e, out, kept);
  if (s != MS_OK) return s;
  if (in->n > kPruneNoAllocMaxN)
    return fail(MS_ERR_INVALID_ARG, "n = %lld exceeds the %lld Gaussians of the static scratch", (long long)in->n,
                (long long)kPruneNoAllocMaxN);
  hipStream_t st = (hipStream_t)stream;
  if (st) {   // the scratch is the current device's copy: the stream must run there
    int cur = 0;
    hipDevice_t sdev = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess) e = hipStreamGetDevice(st, &sdev);
    if (e != hipSuccess) return hip_fail(e, "prune (device of the stream)");
    if ((int)sdev != cur) return fail(MS_ERR_INVALID_ARG, "stream on device %d, current device %d", (int)sdev, cur);
  }
  uint32_t* ws = nullptr;
  hipError_t e = prune_scratch(&ws);
  if (e != hipSuccess) return hip_fail(e, "prune scratch address");
  e = launch_prune(*in, *out, tau_o, tau_s, tau_e, kept, ws, st);
  if (e != hipSuccess) return hip_fail(e, "prune");
  return MS_OK;
}

size_t ms_select_workspace_bytes(int64_t n) { return n < 0 ? 0 : select_workspace_bytes(n); }

int32_t ms_select_candidates(const float* means, int64_t n, const float* viewmat, const ms_intrinsics* intr,
                             float near_z, float max_dist, float margin, int32_t* indices, int64_t* count,
                             void* workspace, size_t ws_bytes, void* stream) {
  if (n < 0 || n > INT32_MAX) return fail(MS_ERR_INVALID_ARG, "n = %lld outside [0, 2^31 - 1]", (long long)n);
  if ((n > 0 && (!means || !indices)) || !viewmat || !intr || !count) return fail(MS_ERR_INVALID_ARG, "null argument");
  if (intr->width < 1 || intr->width > 16384 || intr->height < 1 || intr->height > 16384)
    return fail(MS_ERR_INVALID_ARG, "image size %dx%d outside [1, 16384]", intr->width, intr->height);
  if (!std::isfinite(intr->fx) || !std::isfinite(intr->fy) || !std::isfinite(intr->cx) || !std::isfinite(intr->cy) ||
      !(intr->fx > 0.f) || !(intr->fy > 0.f))
    return fail(MS_ERR_INVALID_ARG, "intrinsics must be finite with fx, fy > 0");
  if (!std::isfinite(near_z) || !(near_z > 0.f)) return fail(MS_ERR_INVALID_ARG, "near_z must be finite and > 0");
  if (!std::isfinite(max_dist) || max_dist < 0.f) return fail(MS_ERR_INVALID_ARG, "max_dist must be finite and >= 0");
  if (!std::isfinite(margin) || margin < 0.f) return fail(MS_ERR_INVALID_ARG, "margin must be finite and >= 0");
  if (n > 0 && (means_overlap(indices, (size_t)n * sizeof(int32_t), means, (size_t)n * 3 * sizeof(float))))
    return fail(MS_ERR_INVALID_ARG, "indices overlap the means");
  if (!workspace) return fail(MS_ERR_WORKSPACE, "null workspace");
  if (ws_bytes < select_workspace_bytes(n)) return fail(MS_ERR_WORKSPACE, "workspace too small");
  SelectArgs a;
  a.means = means;
  a.n = n;
  a.viewmat = viewmat;
  a.fx = (double)intr->fx;
  a.fy = (double)intr->fy;
  a.cx = (double)intr->cx;
  a.cy = (double)intr->cy;
  a.near = (double)near_z;
  a.dmax2 = (double)max_dist * (double)max_dist;
  a.xmin = -(double)margin;
  a.xmax = (double)(intr->width - 1) + (double)margin;
  a.ymin = -(double)margin;
  a.ymax = (double)(intr->height - 1) + (double)margin;
  hipError_t e = launch_select(a, indices, count, workspace, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "candidate selection");
  return MS_OK;
}

namespace {
int32_t check_gicp_cfg(const ms_gicp_config* c) {
  if (!c) return fail(MS_ERR_INVALID_ARG, "null configuration");
  if (c->max_src < 0 || c->max_tgt < 0 || c->max_src > INT32_MAX || c->max_tgt > INT32_MAX)
    return fail(MS_ERR_INVALID_ARG, "counts outside [0, 2^31 - 1]");
  if (!std::isfinite(c->d_max) || !(c->d_max > 0.f)) return fail(MS_ERR_INVALID_ARG, "d_max must be finite and > 0");
  if (!std::isfinite(c->eps) || c->eps < 0.f) return fail(MS_ERR_INVALID_ARG, "eps must be finite and >= 0");
  return MS_OK;
}

// A map of means with optional (scales, quats); opacity and colors unused.
int32_t check_gicp_map(const ms_map* m, int64_t limit, const char* what) {
  if (!m) return fail(MS_ERR_INVALID_ARG, "null %s map", what);
  if (m->n < 0 || m->n > limit)
    return fail(MS_ERR_INVALID_ARG, "%s count %lld outside [0, %lld]", what, (long long)m->n, (long long)limit);
  if (m->n > 0 && !m->means) return fail(MS_ERR_INVALID_ARG, "null %s means", what);
  if ((m->scales == nullptr) != (m->quats == nullptr))
    return fail(MS_ERR_INVALID_ARG, "%s scales and quats must both be given or both be NULL", what);
  return MS_OK;
}

int32_t check_gicp_ws(const GicpPlan& p, void* ws, size_t ws_bytes) {
  if (!ws) return fail(MS_ERR_WORKSPACE, "null workspace");
  if (((uintptr_t)ws & 255) != 0) return fail(MS_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < p.bytes) return fail(MS_ERR_WORKSPACE, "workspace too small");
  return MS_OK;
}
}  // namespace

size_t ms_gicp_workspace_bytes(const ms_gicp_config* cfg) {
  if (!cfg || cfg->max_src < 0 || cfg->max_tgt < 0 || !(cfg->d_max > 0.f)) return 0;
  return gicp_plan(cfg->max_src, cfg->max_tgt, cfg->d_max).bytes;
}

int32_t ms_gicp_build(const ms_gicp_config* cfg, const ms_map* tgt, const int32_t* tgt_idx, int64_t m,
                      void* workspace, size_t ws_bytes, void* stream) {
  int32_t s = check_gicp_cfg(cfg);
  if (s == MS_OK) s = check_gicp_map(tgt, INT32_MAX, "target");
  if (s != MS_OK) return s;
  if (m < 0 || m > cfg->max_tgt) return fail(MS_ERR_INVALID_ARG, "m = %lld outside [0, max_tgt]", (long long)m);
  if (!tgt_idx && m != tgt->n) return fail(MS_ERR_INVALID_ARG, "without an index list m must equal the map's n");
  if (tgt_idx && m > 0 && tgt->n == 0) return fail(MS_ERR_INVALID_ARG, "indices into an empty map");
  const GicpPlan p = gicp_plan(cfg->max_src, cfg->max_tgt, cfg->d_max);
  s = check_gicp_ws(p, workspace, ws_bytes);
  if (s != MS_OK) return s;
  StageTimer tm(MS_STAGE_GICP, (hipStream_t)stream);
  hipError_t e = gicp_build(p, tgt->means, tgt->n, tgt_idx, m, (char*)workspace, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "alignment grid");
  return MS_OK;
}

int32_t ms_gicp_correspond(const ms_gicp_config* cfg, const ms_map* src, const float* T, int32_t* corr,
                           void* workspace, size_t ws_bytes, void* stream) {
  int32_t s = check_gicp_cfg(cfg);
  if (s == MS_OK) s = check_gicp_map(src, cfg->max_src, "source");
  if (s != MS_OK) return s;
  if (!T || (src->n > 0 && !corr)) return fail(MS_ERR_INVALID_ARG, "null pose or correspondence array");
  const GicpPlan p = gicp_plan(cfg->max_src, cfg->max_tgt, cfg->d_max);
  s = check_gicp_ws(p, workspace, ws_bytes);
  if (s != MS_OK) return s;
  StageTimer tm(MS_STAGE_GICP, (hipStream_t)stream);
  hipError_t e = gicp_correspond(p, src->means, src->n, T, cfg->d_max, corr, nullptr, (char*)workspace,
                                 (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "correspondences");
  return MS_OK;
}

int32_t ms_gicp_normal_equations(const ms_gicp_config* cfg, const ms_map* src, const ms_map* tgt, const float* T,
                                 const int32_t* corr, double* out, void* workspace, size_t ws_bytes, void* stream) {
  int32_t s = check_gicp_cfg(cfg);
  if (s == MS_OK) s = check_gicp_map(src, cfg->max_src, "source");
  if (s == MS_OK) s = check_gicp_map(tgt, INT32_MAX, "target");
  if (s != MS_OK) return s;
  if (!T || !out || (src->n > 0 && !corr)) return fail(MS_ERR_INVALID_ARG, "null pose, output or correspondences");
  const GicpPlan p = gicp_plan(cfg->max_src, cfg->max_tgt, cfg->d_max);
  s = check_gicp_ws(p, workspace, ws_bytes);
  if (s != MS_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  StageTimer tm(MS_STAGE_GICP, st);
  hipError_t e = gicp_normal(p, *src, *tgt, T, corr, cfg->eps, (char*)workspace, st);
  if (e == hipSuccess) e = gicp_solve(p, src->n, nullptr, out, nullptr, (char*)workspace, st, false);
  if (e != hipSuccess) return hip_fail(e, "normal equations");
  return MS_OK;
}

int32_t ms_gicp_align(const ms_gicp_config* cfg, const ms_map* src, const ms_map* tgt, float* T, int32_t iters,
                      int32_t* corr, double* hist, void* workspace, size_t ws_bytes, void* stream) {
  int32_t s = check_gicp_cfg(cfg);
  if (s == MS_OK) s = check_gicp_map(src, cfg->max_src, "source");
  if (s == MS_OK) s = check_gicp_map(tgt, INT32_MAX, "target");
  if (s != MS_OK) return s;
  if (!T) return fail(MS_ERR_INVALID_ARG, "null pose");
  if (iters < 0 || iters > 1000) return fail(MS_ERR_INVALID_ARG, "iters = %d outside [0, 1000]", iters);
  const GicpPlan p = gicp_plan(cfg->max_src, cfg->max_tgt, cfg->d_max);
  s = check_gicp_ws(p, workspace, ws_bytes);
  if (s != MS_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  int32_t* c = corr ? corr : at<int32_t>(ws, p.corr);
  StageTimer tm(MS_STAGE_GICP, st);
  // the targets' covariances and means, gathered once for all iterations
  if (iters > 0) {
    const hipError_t e = gicp_records(p, *tgt, ws, st);
    if (e != hipSuccess) return hip_fail(e, "target records");
  }
  for (int it = 0; it < iters; it++) {
    hipError_t e = gicp_correspond(p, src->means, src->n, T, cfg->d_max, c, at<int32_t>(ws, p.cslot), ws, st);
    if (e == hipSuccess) e = gicp_normal_records(p, *src, T, cfg->eps, ws, st);
    if (e == hipSuccess)
      e = gicp_solve(p, src->n, T, at<double>(ws, p.out), hist ? hist + 29 * (int64_t)it : nullptr, ws, st, true);
    if (e != hipSuccess) return hip_fail(e, "alignment iteration");
  }
  return MS_OK;
}

int32_t ms_pose_adam_step(float* viewmat, const float* twist_grad, float* state, float lr, float beta1, float beta2,
                          float eps, void* stream) {
  if (!viewmat || !twist_grad || !state) return fail(MS_ERR_INVALID_ARG, "null argument");
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(MS_ERR_INVALID_ARG, "Adam hyper-parameters out of range");
  StageTimer tm(MS_STAGE_POSE_STEP, (hipStream_t)stream);
  hipError_t e = launch_pose_adam(viewmat, twist_grad, state, lr, beta1, beta2, eps, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "pose step");
  return MS_OK;
}

int32_t ms_profiler_create(uint32_t stage_mask, int32_t capacity, ms_profiler** out) {
  if (!out || capacity < 1 || capacity > (1 << 20)) return fail(MS_ERR_INVALID_ARG, "bad profiler arguments");
  ms_profiler* p = new ms_profiler();
  p->mask = stage_mask;
  p->cap = capacity;
  p->ev.resize(2 * (size_t)capacity);
  p->stage.resize(capacity);
  for (auto& e : p->ev) {
    // timing-only events: no system-scope fence when they complete, which
    // would otherwise write back and invalidate caches between the stages
    hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    if (r != hipSuccess) {
      e = nullptr;
      ms_profiler_destroy(p);
      return hip_fail(r, "hipEventCreate");
    }
  }
  *out = p;
  return MS_OK;
}

int32_t ms_profiler_destroy(ms_profiler* p) {
  if (!p) return MS_OK;
  if (g_prof == p) g_prof = nullptr;
  for (auto& e : p->ev)
    if (e) (void)hipEventDestroy(e);   // nothing to do about a failure while tearing down
  delete p;
  return MS_OK;
}

int32_t ms_profiler_attach(ms_profiler* p) {
  g_prof = p;
  return MS_OK;
}

int32_t ms_profiler_read(ms_profiler* p, double total_ms[MS_STAGE_COUNT], int64_t launches[MS_STAGE_COUNT]) {
  if (!p || !total_ms || !launches) return fail(MS_ERR_INVALID_ARG, "null argument");
  for (int s = 0; s < MS_STAGE_COUNT; s++) {
    total_ms[s] = 0.0;
    launches[s] = 0;
  }
  for (int i = 0; i < p->used; i++) {
    if (p->stage[i] < 0) continue;   // its end event was never recorded
    hipError_t e = hipEventSynchronize(p->ev[2 * i + 1]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e, "profiler read");
    total_ms[p->stage[i]] += ms;
    launches[p->stage[i]] += 1;
  }
  p->used = 0;
  return MS_OK;
}

}  // extern "C"
