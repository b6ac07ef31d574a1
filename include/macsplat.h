/*
 * macsplat.h -- C ABI of the MI355X differentiable RGB-D Gaussian rasterizer.
 *
 * What it computes (MAC-Ego3D, arXiv 2412.09723):
 *   * Sec. 3.3, Eq. 2: a map of 3D Gaussians (mean, covariance, opacity,
 *     colour) rendered into an image by front-to-back alpha compositing,
 *     I(p) = sum_i c_i f_i(p) prod_{j<i} (1 - f_j(p)).
 *   * Sec. 3.5, Eq. 7: depth maps rendered the same way from the Gaussians;
 *     the silhouette (accumulated opacity) 1 - prod_j (1 - f_j(p)).
 *   * Sec. 3.4 "Optimization" and Sec. 3.5 "Optimization": gradients of a
 *     loss on those images with respect to the map and the camera pose.
 *   * Sec. 3.1: the pose is an element of SE(3); here the world-to-camera
 *     transform [R|t].
 *   * App. C.1: Gaussians carry per-axis scales; the covariance is
 *     Sigma = Rq diag(s)^2 Rq^T with Rq the rotation of a quaternion.
 *
 * The paper does not define the projection f_i. This library uses EWA
 * local-affine splatting: Sigma' = J R Sigma R^T J^T + 0.3 I (pixels^2), J the
 * perspective Jacobian with the normalised image coordinate clamped to 1.3x
 * the half field of view; f_i(p) = min(0.99, o_i exp(-d^2/2)), d^2 the
 * Mahalanobis distance of p under Sigma'; a Gaussian counts at p only if
 * d^2 <= 9 and o_i exp(-d^2/2) >= 1/255; compositing stops before the
 * Gaussian that would take the transmittance below 1e-4; depth is
 * sum z alpha T with z the camera-frame depth of the mean; background 0;
 * pixel (x, y) is sampled at integer coordinates (x, y).
 *
 * Discrete structure (pinned recipe). Visibility, pixel boxes, depth keys,
 * per-tile lists and per-pixel acceptance are integer outcomes of
 * floating-point tests. They are defined by this evaluation order, which any
 * conforming implementation reproduces bit for bit:
 *   Projection, IEEE binary64, round to nearest, no fused multiply-add,
 *   sums left to right as written; float inputs widened exactly.
 *     p_i = ((R_i0 m_0 + R_i1 m_1) + R_i2 m_2) + t_i
 *     culled unless p_2 > near, p finite, o, s and the colour finite;
 *     n2 = ((w w + x x) + y y) + z z, culled unless 0 < n2 < inf;
 *     r = 1/sqrt(n2); (w,x,y,z) *= r; Rq from the products xx, yy, zz, xy,
 *       xz, yz, wx, wy, wz as Rq00 = 1 - 2(yy+zz), Rq01 = 2(xy-wz),
 *       Rq02 = 2(xz+wy), Rq10 = 2(xy+wz), Rq11 = 1 - 2(xx+zz),
 *       Rq12 = 2(yz-wx), Rq20 = 2(xz-wy), Rq21 = 2(yz+wx), Rq22 = 1 - 2(xx+yy);
 *     M_ij = Rq_ij s_j;  W_ij = (R_i0 M_0j + R_i1 M_1j) + R_i2 M_2j;
 *     rz = 1/p_2; xn = p_0 rz; yn = p_1 rz; limx = (0.65 W)/fx;
 *       limy = (0.65 H)/fy; xc = min(max(xn, -limx), limx), yc likewise;
 *     j00 = fx rz; j02 = -((fx xc) rz); j11 = fy rz; j12 = -((fy yc) rz);
 *     V0k = j00 W_0k + j02 W_2k;  V1k = j11 W_1k + j12 W_2k;
 *     S00 = ((V00 V00 + V01 V01) + V02 V02) + 0.3;
 *     S01 = (V00 V10 + V01 V11) + V02 V12;
 *     S11 = ((V10 V10 + V11 V11) + V12 V12) + 0.3;
 *     culled unless S00 <= 2^22, S11 <= 2^22, S01 finite;
 *     u = fx xn + cx; v = fy yn + cy; culled unless |u|, |v| <= 2^22;
 *     rx = ceil(3.01171875 sqrt(S00)); ry = ceil(3.01171875 sqrt(S11));
 *     box: xlo = ceil(u - rx), xhi = floor(u + rx), ylo, yhi likewise;
 *       culled unless xlo <= W-1, xhi >= 0, ylo <= H-1, yhi >= 0;
 *       then clamped to the image;
 *     det = S00 S11 - S01 S01, culled unless det > 0;
 *     z32 = (float)p_2, culled unless finite; depth key = bits(z32);
 *     sd = sqrt(det); s1 = sqrt(S11); l11 = s1/sd; l12 = -S01/(sd s1);
 *       l22 = 1/s1; a = (float)(K l11), b = (float)(K l12),
 *       c = (float)(K l22) with K = sqrt(log2(e)/2) = 0x1.b2da4e9808a53p-1;
 *     ui = floor(u), uf = (float)(u - ui), vi, vf likewise;
 *     qcut = (float)min(Q9, L2(255 o)) (-inf when 255 o <= 0), where
 *       Q9 = 4.5 log2(e) = 0x1.9f7f051d0f35ep+2 and L2 is the pinned log2:
 *       m, e = frexp(x); m = 2m, e = e-1; if m > 1.4142135623730951 then
 *       m = m/2, e = e+1; y = (m-1)/(m+1); P = 1/23; for k = 10..0:
 *       P = P y^2 + 1/(2k+1); L2 = e + (2 y P) log2(e).
 *   Per-pixel acceptance, IEEE binary32, fma fused:
 *     dx = (float)(x - ui) - uf; dy = (float)(y - vi) - vf;
 *     t1 = fma(a, dx, b dy); t2 = c dy; q = fma(t1, t1, t2 t2);
 *     accepted iff q <= qcut.  (q approximates d^2 log2(e)/2; the 2^-8 box
 *     margin guarantees that no pixel outside the box is ever accepted.)
 *   Order: a pixel visits accepted Gaussians by ascending (depth key, index).
 *   Tile lists for bin tile size B: Gaussian i is in tile (tx, ty) iff
 *     xlo/B <= tx <= xhi/B and ylo/B <= ty <= yhi/B (integer division),
 *     each list ordered by (depth key, index).
 * Continuous values (alpha, transmittance, colours, depth, gradients) are
 * binary32 on the device.
 *
 * Conventions. Camera x right, y down, z forward. viewmat is the row-major
 * 3x4 world-to-camera matrix [R|t]. Arrays are structure-of-arrays float32:
 * means [3][n], scales [3][n] (standard deviations in metres), quats [4][n]
 * (w, x, y, z; any non-zero norm, normalised inside), opacity [n] (already in
 * (0,1); 0 is accepted and composites nowhere), colors [3][n] (RGB). Images are planar: rgb [3][H][W], depth and
 * silhouette [H][W].
 *
 * Memory and streams. Every array pointer is a DEVICE pointer unless stated
 * otherwise, allocated and owned by the caller. The library allocates no
 * device memory: scratch state lives in a caller-provided workspace of
 * ms_workspace_bytes() bytes (256-byte aligned). All work is enqueued on the
 * given HIP stream (hipStream_t passed as void*; NULL = default stream);
 * calls are stream-ordered and return before the device finishes, except
 * those documented as synchronising.
 *
 * Errors. Functions return an ms_status and never throw. Host-side argument
 * checks are synchronous. A (Gaussian, tile) pair count above the capacity is
 * detected on the device: the job's images are then filled with NaN, nothing
 * is truncated silently, and the condition is reported by ms_read_stats() and
 * by the next ms_backward() on that workspace (MS_ERR_CAPACITY).
 */
#ifndef MACSPLAT_H
#define MACSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MS_ABI_VERSION 5

typedef enum {
  MS_OK = 0,
  MS_ERR_INVALID_ARG = 1,   /* null pointer, bad size, bad option */
  MS_ERR_CAPACITY = 2,      /* more (Gaussian, tile) pairs than the workspace holds */
  MS_ERR_WORKSPACE = 3,     /* workspace too small or misaligned */
  MS_ERR_HIP = 4,           /* a HIP runtime call failed; see ms_last_error() */
  MS_ERR_UNSUPPORTED = 5    /* option value outside the supported set */
} ms_status;

/* Pinhole intrinsics, pixels. width, height in [1, 16384]. */
typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
} ms_intrinsics;

/* Flags of ms_options.flags. */
#define MS_FLAG_POSE_GRAD_ONLY 1u   /* backward: only the pose gradient (map gradients untouched) */
#define MS_FLAG_NO_POSE_GRAD 2u     /* backward: skip the pose gradient (viewmat/twist untouched) */
#define MS_FLAG_SCALAR_FWD 4u       /* forward compositing reads each Gaussian's record with wave-uniform
                                       scalar loads instead of staging wave_batch records through LDS */
#define MS_FLAG_SCALAR_BWD 8u       /* the same for backward compositing */
#define MS_FLAG_ACCUMULATE_MAP_GRADS 32u /* backward (per job): add this job's map gradients into grads
                                           instead of writing them; the caller zeroes the arrays first.
                                           Jobs of one batch that share a map (several views of one map)
                                           then sum into one set of arrays. Float atomics: the summation
                                           order, and so the last bits, vary from run to run. */
#define MS_FLAG_MFMA_BWD 16u        /* backward compositing with the per-Gaussian reduction over each 8x8
                                       sub-block done as a matrix-core product in binary32 (fp32
                                       operands and accumulation, v_mfma_f32_16x16x4_f32) */
#define MS_FLAG_BWD_BF16X3 64u      /* with MS_FLAG_MFMA_BWD: form that product from bf16 high/low parts
                                       (hi*hi + hi*lo + lo*hi, about 16 significant bits per term,
                                       fp32 accumulation; v_mfma_f32_16x16x32_bf16). Faster, less
                                       precise; not the default */
#define MS_FLAG_TILE_QUEUE 128u     /* compositing (the LDS-staged forward and the MFMA backward) as a
                                       persistent launch: as many workgroups as the device holds at once
                                       take tiles from a queue sorted by expected work, longest first (the
                                       bin's list length for the forward, the forward's per-sub-block list
                                       depth for the backward). Same results as the one-workgroup-per-tile
                                       grid up to float summation order. The scalar-record kernels and the
                                       LDS backward ignore it */
#define MS_FLAG_XCD_QUEUES 256u     /* with MS_FLAG_TILE_QUEUE: eight queues, one per XCD, dealt the
                                       sorted tiles round-robin; a workgroup drains its own XCD's queue
                                       first, then the others in turn */

/* Launch options. tile: edge in pixels of the screen tile one compositing
 * workgroup owns, 8 | 16 | 32. bin_tile: edge of the tiles whose
 * (Gaussian, tile) lists are built and sorted, 0 (same as tile) or a multiple
 * of tile in {8, ..., 256}; each compositing workgroup walks the list of the
 * bin tile containing it. wave_batch: Gaussians staged per wavefront per
 * step, 32 | 64 | 128. near_z: near plane in metres, > 0 (0.2 is the
 * documented default). */
typedef struct {
  int32_t tile;
  int32_t wave_batch;
  float near_z;
  uint32_t flags;
  int32_t bin_tile;
} ms_options;

/* A Gaussian map (device pointers, float32 SoA, see Conventions). n >= 0. */
typedef struct {
  int64_t n;
  const float *means, *scales, *quats, *opacity, *colors;
} ms_map;

/* Rendered images or their upstream gradients (device pointers). */
typedef struct {
  float *rgb;          /* [3][H][W] */
  float *depth;        /* [H][W] */
  float *silhouette;   /* [H][W] */
} ms_images;

/* Gradients (device pointers), same shapes as ms_map; written, not
 * accumulated: entries of culled Gaussians are set to zero. viewmat: [12]
 * dL/d[R|t] row-major. twist: [6] dL/dxi for the left perturbation
 * exp(xi^) [R|t], xi = (rho, phi), rho the translation part. Pointers the
 * flags exclude may be NULL. */
typedef struct {
  float *means, *scales, *quats, *opacity, *colors;
  float *viewmat, *twist;
} ms_grads;

/* ABI version (MS_ABI_VERSION). */
int32_t ms_abi_version(void);

/* Static description of a status code. Never NULL. */
const char* ms_status_string(int32_t status);

/* Detail of the last non-OK status returned on the calling thread. */
const char* ms_last_error(void);

/* Workspace size in bytes for a job of n Gaussians at the given intrinsics
 * and options holding up to pair_capacity (Gaussian, tile) pairs. Returns 0
 * for invalid arguments. The same (n, intrinsics, tile, pair_capacity) must
 * be passed to ms_forward and the matching ms_backward. */
size_t ms_workspace_bytes(int64_t n, const ms_intrinsics* intr, const ms_options* opts, int64_t pair_capacity);

/* Forward render (Eq. 2 and its depth/silhouette analogues).
 * map: Gaussian map; viewmat: device float[12]; intr, opts: host structs;
 * workspace: device buffer of ws_bytes >= ms_workspace_bytes(...), 256-byte
 * aligned, reused by the matching ms_backward (its forward state lives
 * there); out: device images written in full.
 * Enqueued on `stream`; returns before completion. */
int32_t ms_forward(const ms_map* map, const float* viewmat, const ms_intrinsics* intr, const ms_options* opts,
                   void* workspace, size_t ws_bytes, int64_t pair_capacity, const ms_images* out, void* stream);

/* Backward pass of the last ms_forward on this workspace (same map, viewmat,
 * intrinsics, options and capacity). grad_out: upstream gradients dL/d(rgb,
 * depth, silhouette) (device); grads: written (see ms_grads). Transmittance is
 * recomputed per pixel from the forward's per-pixel final transmittance and
 * last-composited index; no per-Gaussian per-pixel state is stored.
 * Returns MS_ERR_CAPACITY when the forward overflowed (checked on the host
 * only if a previous ms_read_stats() saw it; otherwise the device skips the
 * work and the gradients are NaN). Enqueued on `stream`. */
int32_t ms_backward(const ms_map* map, const float* viewmat, const ms_intrinsics* intr, const ms_options* opts,
                    void* workspace, size_t ws_bytes, int64_t pair_capacity, const ms_images* grad_out,
                    const ms_grads* grads, void* stream);

/* ms_backward for the L1 loss of Eq. 7's L1 terms as a per-agent tracking
 * loss, w_rgb mean|rgb - rgb*| + w_depth mean|D - D*| + w_sil mean|S - S*|,
 * with its upstream gradient formed per pixel inside the compositing
 * backward (sign(0) = 0) instead of read from gradient planes: the same
 * result, bit for bit, as ms_l1_loss_grad followed by ms_backward, without
 * the planes' round trip through memory. pred: the images the last
 * ms_forward on this workspace wrote; target: the observed images (device,
 * same layout). Other arguments, errors and stream behaviour as
 * ms_backward. */
int32_t ms_backward_l1(const ms_map* map, const float* viewmat, const ms_intrinsics* intr, const ms_options* opts,
                       void* workspace, size_t ws_bytes, int64_t pair_capacity, const ms_images* pred,
                       const ms_images* target, float w_rgb, float w_depth, float w_sil, const ms_grads* grads,
                       void* stream);

/* Counters of the last forward (and backward) on a workspace, copied to
 * host memory out[7]: visible Gaussians, (Gaussian, bin tile) pairs,
 * pair-capacity overflow flag (0/1), bin tiles, composited (pixel, Gaussian)
 * pairs, bin-list entries walked by the forward wavefronts, packed
 * (wavefront, Gaussian) entries walked by the backward(s) since the forward.
 * Arguments as for ms_forward. SYNCHRONISES the stream. Returns MS_ERR_HIP
 * when a bounded device wait gave up. */
int32_t ms_read_stats(const void* workspace, size_t ws_bytes, int64_t n, const ms_intrinsics* intr,
                      const ms_options* opts, int64_t pair_capacity, int64_t out[7], void* stream);

/* ------------------------------------------------------------- batches
 * Several jobs -- one map, one camera, one set of images each, e.g. the
 * tracking or mapping iterations of different agents (Sec. 3.6: agents run
 * their intra-agent processes independently and in parallel; inter-agent
 * optimisation batches its rendering) -- rendered through ONE launch
 * sequence: one projection launch over all jobs' Gaussians, one depth sort,
 * one pair sort, one compositing launch over all jobs' tiles, one backward.
 * Each job's result is the result of rendering it alone (the per-job
 * lists, and so every decision, are the same).
 * Every job shares `opts` (tile, wave_batch, bin_tile, near_z, kernel
 * flags); intrinsics and sizes may differ. At most MS_MAX_BATCH jobs. */
#define MS_MAX_BATCH 12

typedef struct {
  ms_map map;
  const float* viewmat;     /* device [12] */
  ms_intrinsics intr;
  ms_images out;            /* forward: written in full */
  ms_images grad_out;       /* backward: upstream gradients */
  ms_grads grads;           /* backward: written as by ms_backward */
  uint32_t flags;           /* backward: MS_FLAG_POSE_GRAD_ONLY / MS_FLAG_NO_POSE_GRAD for this job
                               (ORed with those of opts) */
} ms_job;

/* Workspace bytes for a batch (0 on invalid arguments). */
size_t ms_batch_workspace_bytes(int32_t njobs, const ms_job* jobs, const ms_options* opts, int64_t pair_capacity);

/* Forward of every job of `jobs` (host array of njobs) into one workspace;
 * pair_capacity bounds the (Gaussian, bin) pairs of all jobs together.
 * Errors as ms_forward; an overflow NaN-fills every job's images. */
int32_t ms_forward_batch(int32_t njobs, const ms_job* jobs, const ms_options* opts, void* workspace, size_t ws_bytes,
                         int64_t pair_capacity, void* stream);

/* Backward of the last ms_forward_batch on this workspace (same jobs, in
 * the same order, with the same maps, cameras, options and capacity). */
int32_t ms_backward_batch(int32_t njobs, const ms_job* jobs, const ms_options* opts, void* workspace,
                          size_t ws_bytes, int64_t pair_capacity, void* stream);

/* ms_read_stats for a batch workspace (counters summed over the jobs). */
int32_t ms_batch_read_stats(int32_t njobs, const ms_job* jobs, const ms_options* opts, const void* workspace,
                            size_t ws_bytes, int64_t pair_capacity, int64_t out[7], void* stream);

/* Device views of the forward state inside a workspace, for inspection and
 * testing (pointers into `workspace`, valid while it is not reused).
 *
 * Every bin list holds its Gaussians ordered by (depth key, Gaussian index).
 * Two layouts exist, chosen by the workspace plan:
 *  list_kind 1 (at most 1024 bins over all jobs): list entries are Gaussian
 *    indices, `records` holds one record per Gaussian in index order, and
 *    sorted_index, rank_of and pair_tile are NULL;
 *  list_kind 0 (more bins): list entries are depth ranks, `records` holds one
 *    record per visible Gaussian in depth-rank order, sorted_index and
 *    rank_of give the permutation. */
typedef struct {
  uint32_t* depth_key;      /* [n] binary32 depth bits, 0xFFFFFFFF when culled */
  uint32_t* sorted_index;   /* kind 0: [n] Gaussian index of depth rank r (first n_visible valid) */
  int32_t* rank_of;         /* kind 0: [n] depth rank of Gaussian i, -1 when culled */
  uint32_t* pair_tile;      /* kind 0: [pair_capacity] bin id of each sorted pair (packed: the pair word) */
  uint32_t* pair_rank;      /* [pair_capacity] list entry of each sorted pair (kind 0 packed: the pair word) */
  uint32_t* tile_range;     /* [bins][2] start, end of each bin's list in pair_rank */
  float* records;           /* [n][16] records, see ms_record_layout (kind 1: index order; 0: rank order) */
  float* tfinal;            /* [H][W] final transmittance */
  uint32_t* last;           /* [H][W] last composited position (+1) in the pixel's bin list */
  uint64_t* counters;       /* [8] visible, pairs, overflow, ... */
  float* grad2d;            /* [n][10] screen-space gradient accumulators, one row per list entry value
                               (kind 1: zero outside a backward pass) */
  int32_t pair_rank_bits;   /* 0: separate arrays; > 0: each pair is one word tile << bits | rank */
  int32_t list_kind;
  uint32_t* tile_order;     /* [tiles] compositing tiles in the order of the last persistent launch's
                               queue (MS_FLAG_TILE_QUEUE), longest expected work first */
  uint32_t* tile_cost;      /* [tiles][tile_waves] per 8x8 sub-block of each compositing tile (row-major
                               in the tile): the deepest list position + 1 any of its pixels composited
                               in the last LDS-staged forward, 0 for none */
  int32_t tiles;            /* compositing tiles (tile edge opts->tile) */
  int32_t tile_waves;       /* (tile / 8)^2 */
} ms_state_view;

/* Record layout (16 x 32-bit words per visible Gaussian):
 * 0 floor(u), 1 floor(v) (integer-valued floats), 2 uf, 3 vf, 4 a, 5 b, 6 c, 7 qcut,
 * 8 log2(opacity), 9 z32, 10-12 colour, 13 xlo | xhi << 16, 14 ylo | yhi << 16,
 * 15 Gaussian index (uint32). */
int32_t ms_state_view_get(void* workspace, size_t ws_bytes, int64_t n, const ms_intrinsics* intr,
                          const ms_options* opts, int64_t pair_capacity, ms_state_view* view);

/* ------------------------------------------------------------ tracking helpers
 * Gradient of the L1 loss  w_rgb mean|rgb - rgb*| + w_depth mean|D - D*| +
 * w_sil mean|S - S*|  (the L1 terms of Eq. 7 used as a per-agent tracking
 * loss; means over 3HW entries for RGB and HW for depth and silhouette).
 * pred, target, grad: device images of intr's size; grad is written (sign(0) =
 * 0). loss: device float receiving the loss value, or NULL. Enqueued on
 * `stream`. */
int32_t ms_l1_loss_grad(const ms_images* pred, const ms_images* target, const ms_intrinsics* intr, float w_rgb,
                        float w_depth, float w_sil, const ms_images* grad, float* loss, void* stream);

/* SSIM term of the mapping objective (Eq. 7), with the SSIM formula of the
 * evaluation-metrics appendix computed from local statistics under an 11x11
 * Gaussian window (standard deviation 1.5 px, weights summing to 1; zero
 * outside the image), C1 = 0.01^2, C2 = 0.03^2 for intensities on [0, 1]:
 *   loss = weight * (1 - mean SSIM(pred, target)) over all channels and pixels,
 * and its gradient with respect to pred (target is fixed).
 * pred, target, grad: device float [channels][height][width], planar, caller-
 * owned; grad must not overlap pred or target. accumulate = 0 overwrites
 * grad and *loss, 1 adds to them (so the term can join an L1 gradient).
 * loss: device float, or NULL. channels in [1, 16], sizes in [1, 16384];
 * otherwise MS_ERR_INVALID_ARG and nothing is enqueued. Enqueued on `stream`. */
int32_t ms_ssim_loss_grad(const float* pred, const float* target, int32_t channels, int32_t width, int32_t height,
                          float weight, float* grad, int32_t accumulate, float* loss, void* stream);

/* The loss of Eq. 7 for one pair (i, j) of rendered views (the images of
 * two agents' maps, or two maps, rendered at one pose), with the readings
 * of the SSIM term above (the term is w_ssim (1 - SSIM)):
 *   L = w_l1 mean|I_i - I_j| + w_ssim (1 - mean SSIM(I_i, I_j))
 *       + w_geom mean|D_i - D_j|,
 * means over 3 W H colour values and W H depths, sign(0) = 0, and its
 * gradient with respect to all four rendered images (the paper's weights
 * are 0.8, 0.2 and 0.1). One launch: the SSIM window sums of both images
 * give dL/dI_i and dL/dI_j (SSIM is symmetric in its two images), the L1
 * terms join them in the same pass, and further workgroups take the depth
 * planes. rgb_*: device float [3][H][W]; depth_*: [H][W]; g_*: gradients of
 * the same shapes, overlapping no input and each other; accumulate = 0
 * overwrites them and *loss, 1 adds to them. loss: device float or NULL.
 * Errors: MS_ERR_INVALID_ARG (null or overlapping arrays, sizes outside
 * [1, 16384], non-finite weights); nothing is enqueued then. Enqueued on
 * `stream`. */
int32_t ms_pair_loss_grad(const float* rgb_i, const float* rgb_j, const float* depth_i, const float* depth_j,
                          int32_t width, int32_t height, float w_l1, float w_ssim, float w_geom, float* g_rgb_i,
                          float* g_rgb_j, float* g_depth_i, float* g_depth_j, int32_t accumulate, float* loss,
                          void* stream);

/* ----------------------------------------------------------------- map upkeep
 * Map pruning (App. C.1, Algorithm 1). A Gaussian is removed when its opacity
 * is below tau_o (0.005 in the paper), or, when tau_s > 0, when its largest
 * scale exceeds tau_s (0.25) or exceeds tau_e (10) times the sum of its other
 * two scales; tau_s <= 0 runs the opacity test alone. The comparisons are
 * strict and taken in binary32: the largest scale is the first of s0, s1, s2
 * that no later one exceeds, the other two are added in index order.
 * in: the map (device, planar [k][n]). out: device arrays with room for
 * k x out->n floats each, out->n >= in->n, aliasing no input array; the
 * survivors are written in their original order as planar [k][kept] (row
 * stride kept). kept: device int64 receiving the survivor count. workspace:
 * device scratch of ms_prune_workspace_bytes(n) bytes. Errors:
 * MS_ERR_INVALID_ARG (null or aliased arrays, capacity, non-finite
 * thresholds, tau_e < 0), MS_ERR_WORKSPACE; nothing is enqueued then.
 * Enqueued on `stream`. */
size_t ms_prune_workspace_bytes(int64_t n);
int32_t ms_prune(const ms_map* in, float tau_o, float tau_s, float tau_e, const ms_map* out, int64_t* kept,
                 void* workspace, size_t ws_bytes, void* stream);

/* ms_prune for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same computation and results, with the scratch in a static device
 * array of the library instead of a workspace. Maps of at most
 * MS_PRUNE_NOALLOC_MAX_N Gaussians (2^26); larger n returns
 * MS_ERR_INVALID_ARG and enqueues nothing. The array (256 KB) is held on
 * each GPU the library runs on until the process ends; its device address
 * is looked up on the first call on a device (the current device, which
 * must be the device of `stream`, else MS_ERR_INVALID_ARG). It allocates
 * nothing (no hipMalloc, hipFree or allocating library call). Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams, or from different threads) race and must be ordered by
 * the caller. Other arguments and errors as ms_prune. */
#define MS_PRUNE_NOALLOC_MAX_N (1LL << 26)
int32_t ms_prune_noalloc(const ms_map* in, float tau_o, float tau_s, float tau_e, const ms_map* out, int64_t* kept,
                         void* stream);

/* Candidate selection (Sec. 3.4, "1) Selection"): the Gaussians of a local
 * map within the camera's field of view and within max_dist of its pose,
 * which the intra-agent association and alignment then work on. Gaussian i
 * is a candidate when its mean, in camera coordinates p = R mu + t, lies
 * beyond the near plane (p_z > near_z), within max_dist of the camera centre
 * (|p| <= max_dist) and projects onto the image widened by `margin` pixels
 * (-margin <= u <= W - 1 + margin, likewise v, pixels sampled at integer
 * coordinates). The decisions are taken in binary64 from the binary32
 * inputs in this order, with no fused operations:
 *   p_k = ((R_k0 mu_0 + R_k1 mu_1) + R_k2 mu_2) + t_k,
 *   d2 = (p_0 p_0 + p_1 p_1) + p_2 p_2 <= max_dist^2,
 *   rz = 1 / p_z, u = fx (p_x rz) + cx, v = fy (p_y rz) + cy;
 * a non-finite mean is never a candidate.
 * means: device [3][n] float; viewmat: device float[12] world-to-camera
 * [R|t]; intr: host struct. indices: device int32 with room for n entries,
 * receiving the candidates' indices in ascending (map) order; count: device
 * int64 receiving their number. workspace: device scratch of
 * ms_select_workspace_bytes(n) bytes. n in [0, 2^31 - 1]. Errors:
 * MS_ERR_INVALID_ARG (null or overlapping arrays, sizes, non-finite or
 * negative near_z, max_dist, margin, fx, fy <= 0), MS_ERR_WORKSPACE;
 * nothing is enqueued then. Enqueued on `stream`. */
size_t ms_select_workspace_bytes(int64_t n);
int32_t ms_select_candidates(const float* means, int64_t n, const float* viewmat, const ms_intrinsics* intr,
                             float near_z, float max_dist, float margin, int32_t* indices, int64_t* count,
                             void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- alignment
 * Generalized-ICP alignment (Sec. 3.4 "3) Alignment", Eqs. 3-4; Sec. 3.5
 * "3) Alignment", Eq. 6). A rigid transform T = [R|t] (device float[12],
 * row-major, binary32) takes source Gaussians x_k (observed points, or
 * another map's Gaussians) onto target Gaussians y_l (the map, or the
 * candidates of ms_select_candidates), minimising
 *   E(T) = sum_(k,l) r^T (R S_k R^T + S_l + eps I)^-1 r,   r = T x_k - y_l,
 * with S = R_q diag(s^2) R_q^T from a Gaussian's scales and quaternion (zero
 * for a map without scales: points, which gives Eq. 4's Mahalanobis
 * distance under the map covariance). Eq. 6 as printed adds S_k unrotated;
 * here it is rotated by T (Generalized-ICP's form).
 * Correspondences: each source takes the nearest target mean within d_max
 * (the paper's point-selection distance, 0.02 m), inclusive, ties to the
 * smaller target index, decided in binary32 in this order without fused
 * operations: y_i = ((R_i0 x_0 + R_i1 x_1) + R_i2 x_2) + t_i;
 * d = y - mu; d2 = (d_0 d_0 + d_1 d_1) + d_2 d_2 <= fl(d_max d_max).
 * An iteration: correspondences at T, the Gauss-Newton normal equations in
 * binary64 (J = [I | -[T x]_x] for the left twist xi = (rho, phi),
 * H = sum J^T M J, g = sum J^T M r with M = (R S_k R^T + S_l + eps I)^-1 at
 * T), xi = -(H + lam I)^-1 g with lam = 1e-12 trace(H) / 6, and
 * T <- exp(xi^) T stored in binary32; with fewer than 6 correspondences T
 * stays. Sums are returned as 29 doubles: H's upper triangle row by row
 * (21), g (6), the cost E, the number of correspondences.
 * The target grid is built once (ms_gicp_build) and serves every call
 * after it on the same workspace. Maps: device [3][n] means; scales [3][n]
 * and quats [4][n] both given or both NULL (points); opacity and colors are
 * not read. Coordinates must be finite to take part (others are skipped)
 * and below 1e6 m in magnitude. Every call is enqueued on `stream`; errors
 * (MS_ERR_INVALID_ARG: null or inconsistent arrays, sizes above the
 * configuration, non-finite or non-positive d_max, negative eps;
 * MS_ERR_WORKSPACE) enqueue nothing. */
typedef struct {
  int64_t max_src, max_tgt;   /* largest source and target counts the workspace serves */
  float d_max;                /* correspondence distance, metres, > 0 */
  float eps;                  /* covariance regularisation, m^2, >= 0 (1e-6 suggested) */
} ms_gicp_config;

size_t ms_gicp_workspace_bytes(const ms_gicp_config* cfg);
/* Hashed grid of the target means: all of `tgt` (tgt_idx NULL, m = tgt->n)
 * or its m Gaussians listed in tgt_idx (device int32, e.g. the candidates of
 * ms_select_candidates). m <= cfg->max_tgt. */
int32_t ms_gicp_build(const ms_gicp_config* cfg, const ms_map* tgt, const int32_t* tgt_idx, int64_t m,
                      void* workspace, size_t ws_bytes, void* stream);
/* Correspondences at T: corr (device int32 [src->n]) receives each source's
 * target map index, or -1. */
int32_t ms_gicp_correspond(const ms_gicp_config* cfg, const ms_map* src, const float* T, int32_t* corr,
                           void* workspace, size_t ws_bytes, void* stream);
/* Normal equations at T for the correspondences corr (device int32
 * [src->n], target map indices or -1): out, device double[29]. */
int32_t ms_gicp_normal_equations(const ms_gicp_config* cfg, const ms_map* src, const ms_map* tgt, const float* T,
                                 const int32_t* corr, double* out, void* workspace, size_t ws_bytes, void* stream);
/* `iters` iterations from T, updating T in place on the device (no host
 * synchronisation). corr: device int32 [src->n] receiving the last
 * iteration's correspondences, or NULL. hist: device double[iters][29]
 * receiving each iteration's sums, or NULL. */
int32_t ms_gicp_align(const ms_gicp_config* cfg, const ms_map* src, const ms_map* tgt, float* T, int32_t iters,
                      int32_t* corr, double* hist, void* workspace, size_t ws_bytes, void* stream);

/* One Adam step on the pose's left twist (Sec. 3.1: poses in SE(3)).
 * viewmat: device float[12] [R|t], updated in place to exp(-step^) [R|t]
 * with step = lr * mhat / (sqrt(vhat) + eps); twist_grad: device float[6]
 * (rho, phi) as written by ms_backward; state: device float[13] (m[6], v[6],
 * step count), zero-initialised by the caller before the first step.
 * Enqueued on `stream`. */
int32_t ms_pose_adam_step(float* viewmat, const float* twist_grad, float* state, float lr, float beta1, float beta2,
                          float eps, void* stream);

/* ------------------------------------------------------------------ profiling
 * Optional per-stage timing with HIP events on the caller's stream. A
 * profiler attached to the calling thread makes ms_forward / ms_backward
 * record an event pair around every stage selected by stage_mask (bit s for
 * stage s). Events are created once by ms_profiler_create (no device memory);
 * at most `capacity` pairs are kept until ms_profiler_read, which waits for
 * them, returns the summed milliseconds and launch counts per stage, and
 * resets the profiler. */
enum {
  MS_STAGE_PROJECT = 0,        /* projection forward */
  MS_STAGE_BIN = 1,            /* compaction, depth sort, pair emission, tile sort, ranges */
  MS_STAGE_COMPOSITE = 2,      /* compositing forward */
  MS_STAGE_COMPOSITE_BWD = 3,  /* compositing backward (includes zeroing its accumulators) */
  MS_STAGE_PROJECT_BWD = 4,    /* projection backward and pose reduction */
  /* single kernels inside the stages above (timed within them) */
  MS_STAGE_BIN_COUNT = 5,      /* per-bin path: pair counts per unit and bin, and their scan */
  MS_STAGE_BIN_EMIT = 6,       /* per-bin path: pair emission into each bin's segment */
  MS_STAGE_BIN_SORT = 7,       /* per-bin path: each bin's stable depth sort */
  MS_STAGE_POSE = 8,           /* deterministic fold of the pose partials */
  /* helpers, timed in their own calls */
  MS_STAGE_LOSS = 9,           /* ms_l1_loss_grad, ms_ssim_loss_grad */
  MS_STAGE_POSE_STEP = 10,     /* ms_pose_adam_step */
  MS_STAGE_GICP = 11,          /* ms_gicp_* */
  MS_STAGE_COUNT = 12
};
typedef struct ms_profiler ms_profiler;
int32_t ms_profiler_create(uint32_t stage_mask, int32_t capacity, ms_profiler** out);
int32_t ms_profiler_destroy(ms_profiler* prof);
int32_t ms_profiler_attach(ms_profiler* prof);   /* NULL detaches */
int32_t ms_profiler_read(ms_profiler* prof, double total_ms[MS_STAGE_COUNT], int64_t launches[MS_STAGE_COUNT]);

#ifdef __cplusplus
}
#endif

#endif /* MACSPLAT_H */
