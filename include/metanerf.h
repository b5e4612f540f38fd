/*
 * metanerf.h -- C ABI of the MI355X (gfx950) posed-body volume renderer.
 *
 * Paper: "Envisioning a Next Generation Extended Reality Conferencing System
 * with Efficient Photorealistic Human Rendering" (arXiv 2306.16541).
 * The library renders a posed human body (Sec. 4, Fig. 2): rays are sampled
 * inside the body's bounding box (Sec. 4.4), each sample is warped from the
 * observed pose to the canonical pose by inverse linear blend skinning
 * (Sec. 4.2, Eq. 7-9), the canonical radiance field c, sigma = MLP(enc(x))
 * is queried (Sec. 4.4, Eq. 13) and the samples are alpha-composited front
 * to back (Sec. 2.1, Eq. 3) with the likelihood augmentation of Sec. 4.4.
 * It also trains that field (Sec. 5.2: squared-error loss of Eq. 14, Adam)
 * and serves many users' frames (Sec. 3, multi-user conferencing).
 *
 * Conventions for every entry point:
 *   - Every call returns mnr_status; MNR_OK == 0.  Nothing throws across
 *     the ABI.  On failure mnr_last_error() (thread-local) holds the reason.
 *   - Arguments are validated on the host before anything is launched; an
 *     invalid call launches nothing and changes no output.
 *   - "dev" pointers are device memory on the current HIP device, owned by
 *     the caller; "host" pointers are read during the call only.  The
 *     library keeps no device memory outside a server object.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *     asynchronously; a HIP launch error is reported as MNR_E_HIP.
 *   - All rendering entry points are reentrant on distinct streams.
 *     Training entry points write gradients/parameters and must be
 *     serialised by the caller.
 */
#ifndef METANERF_H
#define METANERF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MNR_MAX_BONES 32
#define MNR_MAX_LEVELS 16
#define MNR_MAX_LAYERS 5
#define MNR_MAX_SPP 1024
/* Bytes of the optional device workspace of the render entry points: eight
 * per-XCD work-queue counters (zeroed by the library on the call's stream
 * before use).  With a workspace, waves pull work dynamically and balance
 * the very uneven per-ray cost; without one (NULL) work is split
 * statically.  Concurrent calls need distinct workspaces. */
#define MNR_WORKSPACE_BYTES 64

typedef enum {
  MNR_OK = 0,
  MNR_E_INVALID = -1,     /* null pointer, NaN/inf pose, bad option */
  MNR_E_SHAPE = -2,       /* unsupported size or layer widths */
  MNR_E_DTYPE = -3,       /* unsupported dtype combination */
  MNR_E_OOM = -4,         /* request exceeds a memory budget */
  MNR_E_HIP = -5,         /* HIP runtime error (text in mnr_last_error) */
  MNR_E_BUSY = -6,        /* server has no free slot right now */
  MNR_E_UNSUPPORTED = -7  /* valid but not implemented configuration */
} mnr_status;

typedef enum { MNR_F32 = 0, MNR_F16 = 1, MNR_BF16 = 2 } mnr_dtype;
typedef enum { MNR_ENC_GRID = 0, MNR_ENC_FREQ = 1 } mnr_encoding;

/* Canonical radiance field (Sec. 4.4, Eq. 13): a multiresolution grid
 * encoding (Mueller et al. 2022, cited in Sec. 2.3) followed by a bias-free
 * MLP with ReLU hidden layers; outputs rgb = sigmoid(o[0:3]), sigma =
 * ReLU(o[3]).
 *   table: dev [n_levels][2^log2_T][n_feat], dtype table_dtype (F32 or F16).
 *     Level l has resolution level_res[l]; it is stored densely (vertex
 *     (x,y,z) at row x + (N+1)(y + (N+1)z)) when (N+1)^3 <= 2^log2_T, else
 *     at row ((x*1) ^ (y*2654435761) ^ (z*805459861)) mod 2^log2_T (uint32).
 *     The encoding of point x is taken at u = clamp((x - box_min) /
 *     (box_max - box_min), 0, 1), p = u*N, cell min(floor(p), N-1).
 *   w[k]: dev row-major [width[k+1]][width[k]], dtype mlp_dtype (F32 or BF16).
 *   dense_packed (optional, NULL = unused): a copy of the dense levels
 *     written by mnr_field_pack in which the four x-y corners of every
 *     cell are adjacent, so that a dense level's sample takes two (F16) or
 *     four (F32) 16-byte loads instead of eight row gathers.  The renderer
 *     reads it instead of `table` for dense levels when present (bitwise
 *     identical results); re-pack after changing `table` (mnr_train_step
 *     does so itself).
 * Supported: n_feat = 2, n_levels * n_feat = width[0] = 32, hidden widths
 * 64, width[n_layers] = 4, 2 <= n_layers <= 4, log2_T <= 24.
 *
 * encoding = MNR_ENC_FREQ selects the paper's own field instead (Sec. 4.4,
 * Eq. 13, Fig. 9): c, sigma = MLP_nerf(gamma(x)) with the positional
 * encoding gamma(x) = [x, sin(2^k pi x_c), cos(2^k pi x_c) for k = 0..9,
 * c = 0..2, one zero] (64 values: x, then per band the three sines and the
 * three cosines) and a skip of gamma into the fourth layer:
 *   h1 = ReLU(W1 gamma), h2 = ReLU(W2 h1), h3 = ReLU(W3 h2),
 *   h4 = ReLU(W4 [h3; gamma]), o = W5 h4  (c = sigmoid(o[0:3]), sigma = ReLU(o[3])).
 * Then n_layers = 5, width = {64, 64, 64, 64, 64, 4} (w[3] is [64][128]:
 * h3 and gamma), mlp_dtype = MNR_BF16 (BF16 MFMA, FP32 accumulation); the
 * grid fields (n_levels .. table, dense_packed) are ignored.  It trains:
 * mnr_render_backward and mnr_train_step run its adjoint (split, through
 * the adjoint workspace, which it requires); the server serves it. */
typedef struct {
  int32_t n_levels, n_feat, log2_T;
  int32_t level_res[MNR_MAX_LEVELS];
  float box_min[3], box_max[3];
  mnr_dtype table_dtype;
  const void* table;
  int32_t n_layers;
  int32_t width[MNR_MAX_LAYERS + 1];
  mnr_dtype mlp_dtype;
  const void* w[MNR_MAX_LAYERS];
  const void* dense_packed;
  int32_t encoding;
} mnr_field;

/* Size in bytes of the packed copy of the dense levels: for every dense
 * level in level order, [z in 0..N][y in 0..N-1][x in 0..N-1] groups of the
 * rows of vertices (x,y,z), (x+1,y,z), (x,y+1,z), (x+1,y+1,z) (n_feat
 * values each, table_dtype), N = level_res[l].  0 when no level is dense or
 * the field is invalid. */
uint64_t mnr_field_packed_bytes(const mnr_field* field);
/* Write field->dense_packed (dev, mnr_field_packed_bytes bytes, 16-byte
 * aligned, caller-owned) from field->table on `stream`. */
mnr_status mnr_field_pack(const mnr_field* field, void* stream);

/* Canonical blend-weight volume W^c (Sec. 4.2, Eq. 9-10): dev float
 * [n_bones + 1][res^3], voxel (x,y,z) at x + res*(y + res*z), channel
 * n_bones = background.  Vertex-aligned over [box_min, box_max]; trilinear
 * samples treat vertices outside the volume as zero.
 * packed (optional, NULL = unused): a copy of the bone channels written by
 * mnr_motion_pack in which the four x-y corners of every trilinear cell are
 * adjacent, so that one bone's sample takes two 16-byte loads instead of
 * eight 4-byte gathers.  The renderer reads it instead of `weights` when
 * present (bitwise identical results); the caller re-packs after changing
 * `weights` (mnr_train_step does so itself). */
typedef struct {
  int32_t n_bones, res;
  float box_min[3], box_max[3];
  const float* weights;
  const float* packed;
  /* Residual non-rigid motion (Sec. 4.3, Eq. 11-12), optional: res_w[0] ==
   * NULL turns it off.  Otherwise dev BF16 row-major weights
   *   res_w[0] W1 [64][32], res_w[1] W2 [64][64], res_w[2] W3 [64][64],
   *   res_w[3] W4 [64][96], res_w[4] W5 [3][64], res_w[5] W_omega [64][3 n_bones]
   * of  h1 = ReLU(W1 g + W_omega Omega), h2 = ReLU(W2 h1), h3 = ReLU(W3 h2),
   *     h4 = ReLU(W4 [h3; g]) (skip connection at the 4th layer), x_res = W5 h4,
   * where Omega is the observed pose's joint angles (joint-major): the
   * axis angles, or with a refiner adjustment (mnr_pose.delta) the
   * axis-angle of R(delta_j) R(axis_angle_j), angle in [0, pi], and
   *   g = [x, for k = 0..3: w_k sin(2^k pi x_c), w_k cos(2^k pi x_c) (c = 0..2),
   *        five zeros],  w_k = (1 - cos(pi clamp(res_alpha - k, 0, 1))) / 2
   * (a truncated Hann window over the frequency bands; res_alpha = 4 opens
   * all of them), x = x_skel.  The field is then queried at x_skel + x_res.
   * Runs on BF16 MFMA with FP32 accumulation, so it needs mlp_dtype ==
   * MNR_BF16.  It trains (mnr_render_backward's grad_res, mnr_train_step's
   * res_* state; gradients reach W1..W5 and W_omega, not Omega); the server
   * serves it, conditioned on each request's pose. */
  const void* res_w[6];
  float res_alpha;
} mnr_motion;

/* Size in bytes of the packed copy: n_bones * res * (res+1)^2 * 16
 * (layout [bone][z][y+1][x+1] of float4 {W(x,y,z), W(x+1,y,z), W(x,y+1,z),
 * W(x+1,y+1,z)}, zero for vertices outside the volume, x, y in [-1, res-1]).
 * 0 for invalid sizes. */
uint64_t mnr_motion_packed_bytes(int32_t res, int32_t n_bones);
/* Write motion->packed (dev, mnr_motion_packed_bytes bytes, caller-owned)
 * from motion->weights on `stream`.  MNR_E_INVALID for a NULL or misaligned
 * (16 B) packed pointer or bad sizes. */
mnr_status mnr_motion_pack(const mnr_motion* motion, void* stream);

/* Body pose (Sec. 4.1-4.2): host arrays.  parent[j] < j (root: -1), rest
 * joints [n][3] in the canonical (rest) pose, axis-angle [n][3] of the
 * estimated pose.  delta (optional, NULL = none): the pose refiner's
 * adjustments [n][3] (Sec. 4.1, Eq. 5-6); the observed pose theta^o then
 * rotates joint j by R(delta_j) R(axis_angle_j).  Bone transforms G_j
 * (Eq. 8) are computed from it by forward kinematics in double precision on
 * the host.  (The residual motion network is conditioned on axis_angle and
 * is rejected with MNR_E_UNSUPPORTED together with delta.) */
typedef struct {
  int32_t n_joints;
  const int32_t* parent;
  const float* rest_joints;
  const float* axis_angle;
  const float* delta;
} mnr_pose;

/* Pinhole camera, x_cam = R_wc * X + T (R_wc row-major); pixel (u, v) =
 * (id % W, id / W) shoots through its centre (u + 0.5, v + 0.5).  box_min /
 * box_max bound the body in observation space: samples are taken only inside
 * it (Sec. 4.4). */
typedef struct {
  float fx, fy, cx, cy;
  float R_wc[9];
  float T[3];
  float box_min[3], box_max[3];
} mnr_camera;

/* Render options.  ert_tau: early ray termination.  A ray stops once its
 * transmittance is below ert_tau: checked after every sample for full
 * frames, after every 64-sample chunk for ray lists (0 disables it).  The
 * colour then differs from the full sum by at most ert_tau * (1 + |bg|).
 * stratified = 0 samples stratum midpoints; 1 draws the jitter xi of sample
 * i of ray b from SplitMix64: output n = b*spp + i of the stream seeded with
 * `seed`, xi = (out >> 40) * 2^-24. */
typedef struct {
  float ert_tau;
  float bg[3];
  int32_t stratified;
  uint64_t seed;
} mnr_opts;

const char* mnr_status_str(mnr_status s);
const char* mnr_last_error(void);
const char* mnr_version(void);

/* Forward kinematics (Sec. 4.2, Eq. 8): host-only, double precision,
 * rounded to float.  G_out: host [n_joints][3][4] = [R_j | t_j] with
 * G_j(x) = R_j x + t_j mapping an observed point to the canonical pose
 * (the inverse of bone j's skinning transform). */
mnr_status mnr_fk_bones(const mnr_pose* pose, float* G_out);

/* Adjoint of mnr_fk_bones (host, double precision, exact derivatives by
 * forward-mode dual numbers): given grad_G (host [n][3][4], dL/dG), writes
 * dL/d(delta) to grad_delta and dL/d(axis_angle) to grad_axis_angle (host
 * [n][3] each; either may be NULL).  mnr_render_backward's grad_bones is
 * the device-side source of grad_G. */
mnr_status mnr_fk_backward(const mnr_pose* pose, const float* grad_G, float* grad_delta, float* grad_axis_angle);

/* Pose refiner MLP_theta (Sec. 4.1, Eq. 5): delta = W_L ReLU(... ReLU(W_1
 * Omega)), Omega = the pose's axis angles flattened (3 n values), no
 * biases.  Host weights w[k] row-major [width[k+1]][width[k]], width[0] =
 * width[n_layers] = 3 n_joints, hidden widths <= 1024, 1 <= n_layers <= 4.
 * Evaluated on the host in double precision: it runs once per frame. */
typedef struct {
  int32_t n_layers;
  int32_t width[MNR_MAX_LAYERS + 1];
  const float* w[MNR_MAX_LAYERS];
} mnr_refiner;

/* delta (host [n][3]) = MLP_theta(omega), omega host [n][3]. */
mnr_status mnr_refiner_apply(const mnr_refiner* refiner, int32_t n_joints, const float* omega, float* delta);
/* Accumulate dL/dw[k] into grad_w[k] (host, same shapes as w) given
 * grad_delta = dL/d(delta) (host [n][3]). */
mnr_status mnr_refiner_backward(const mnr_refiner* refiner, int32_t n_joints, const float* omega,
                                const float* grad_delta, float* const* grad_w);
/* Adam (Sec. 5.2: beta1 = 0.9, beta2 = 0.99) on the refiner's host weights,
 * one call per optimiser step.  w[k] must be the writable buffers that
 * refiner->w[k] points to; grad_w[k], m[k], v[k] have the same shapes (host
 * float, caller-owned, m and v zero before step 1).  step is 1-based (bias
 * correction).  Updates w, m, v in place, computing in double precision,
 * and clears grad_w for the next accumulation. */
mnr_status mnr_refiner_adam(const mnr_refiner* refiner, int32_t n_joints, float* const* w, float* const* grad_w,
                            float* const* m, float* const* v, int32_t step, float lr, float beta1, float beta2,
                            float eps);

/* Render rays (Sec. 4, Fig. 2; Eq. 3, 7-9, 13).  pixel_ids: dev int32
 * [n_rays] pixel indices of an H x W image, or NULL for the full frame in
 * row-major order (then n_rays must equal H*W).  Ids outside [0, H*W)
 * render as misses.  out_rgba: dev float [n_rays][4] = (r, g, b, opacity);
 * rays that miss the box get (bg, 0).
 * t_chunks (optional, dev float [n_rays][ceil(spp/64) + 1]): the state the
 * adjoint needs -- transmittance at the start of each 64-sample chunk the
 * ray reached (-1 for chunks it never reached), then the number of samples
 * it processed.  A ray that misses the box (or a listed id outside the
 * image) gets -1 in every chunk entry and 0 processed samples; the adjoint
 * skips it.  n_evaluated (optional, dev uint64, accumulated with atomics)
 * counts the samples actually evaluated. */
mnr_status mnr_render(const mnr_field* field, const mnr_motion* motion, const mnr_pose* pose,
                      const mnr_camera* cam, int32_t H, int32_t W, int32_t spp,
                      const mnr_opts* opts, const int32_t* pixel_ids, int32_t n_rays,
                      float* out_rgba, float* t_chunks, unsigned long long* n_evaluated,
                      void* workspace, void* stream);

/* mnr_render for callers that cannot allocate device memory or pass a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, results and errors as
 * mnr_render with a workspace, minus the workspace: the work-queue counters
 * live in a library-owned device array of MNR_NOALLOC_SCRATCH_BYTES that
 * each GPU holds from the first call on it until the process ends.  The
 * call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); it clears the counters with a fill kernel on `stream` before
 * the render.  The counters' size does not depend on the frame or ray
 * count, so every size mnr_render accepts is accepted here.  All calls on
 * one GPU share the array: calls that overlap in time on one GPU (distinct
 * streams, or host threads without ordering) race on it and must be
 * serialised by the caller; calls in one stream are ordered. */
#define MNR_NOALLOC_SCRATCH_BYTES 64
mnr_status mnr_render_noalloc(const mnr_field* field, const mnr_motion* motion, const mnr_pose* pose,
                              const mnr_camera* cam, int32_t H, int32_t W, int32_t spp,
                              const mnr_opts* opts, const int32_t* pixel_ids, int32_t n_rays,
                              float* out_rgba, float* t_chunks, unsigned long long* n_evaluated,
                              void* stream);

/* Adjoint of mnr_render (hand-written; recomputes per-sample activations
 * instead of storing them).  Given t_chunks written by mnr_render with the
 * same arguments and dL/d(rgba) grad_rgba (dev [n_rays][4]), ACCUMULATES
 * into
 *   grad_table   dev float [n_levels][2^log2_T][n_feat]
 *   grad_w[k]    dev float [width[k+1]][width[k]]
 *   grad_weights dev float [n_bones + 1][res^3]   (dL/dW^c)
 *   grad_bones   dev float [n_bones][3][4]         (dL/dG_j of Eq. 8; optional,
 *                NULL skips it): through the warp's points G_j x and its
 *                blend weights, per wave summed before one atomic per entry;
 *                mnr_fk_backward carries it on to the pose.
 * Gradients are those of the forward actually computed (early termination
 * included).  Summation order of the atomics is not deterministic.
 * Frequency-encoded field (encoding = MNR_ENC_FREQ): grad_table is unused
 * (may be NULL) and grad_w[0..4] are W1..W5 (grad_w[3] [64][128]); the
 * adjoint runs split: the forward pass again with its four hidden
 * activations saved (BF16) and the compositing adjoint, then the skip
 * MLP's adjoint on BF16 MFMA from the saved activations (weight gradients
 * and dL/dx_final through gamma's derivative), then the skinning adjoint;
 * it needs adjoint_ws.
 * grad_res (NULL unless motion->res_w[0] != NULL): dev float pointers for
 * the residual motion network's gradients, W1..W5 and W_omega (shapes as
 * motion->res_w), accumulated.  The adjoint then runs split: the warp and
 * residual network forward, the field's adjoint at x_final, the residual
 * network's adjoint (Sec. 4.3, Eq. 11-12, on BF16 MFMA) and the skinning
 * adjoint at x_skel, passing per-sample values through the workspace.
 * adjoint_ws (dev, 256-byte aligned, adjoint_ws_bytes >=
 * mnr_adjoint_ws_bytes(field, motion, n_rays, spp); contents are scratch):
 *   - the table and blend-weight gradients leave the adjoint as (key,
 *     value) records that are binned by slice and summed in LDS in 64-bit
 *     fixed point, instead of global float atomics (the same sum in
 *     another order): every hashed level's (one record per sample, corner
 *     and two features), the dense levels' (one per corner and run of
 *     consecutive samples in one cell) when the hashed levels' T rows each
 *     plus the dense levels' (N+1)^3 rows fit 4096 x 2^14 keys, and
 *     dL/dW^c's (one per run and pair of x-adjacent cell corners inside the
 *     volume) when it fits too and res is a power of two up to 4096; what
 *     does not fit keeps run-summed atomics.  After the call the
 *     workspace's first 32-bit word holds the number of records written;
 *   - with a ray list, the rays are processed in a spatially coherent order
 *     (a counting sort by the Morton index of their pixel's cell in a
 *     64 x 64 grid over the image), which keeps neighbouring rays' gathers
 *     in one L2; the results are the same;
 *   - with a residual network or the frequency-encoded field, the split
 *     adjoint's per-sample values.
 * NULL: atomics for the table; with a residual network or the
 * frequency-encoded field, MNR_E_INVALID. */
mnr_status mnr_render_backward(const mnr_field* field, const mnr_motion* motion,
                               const mnr_pose* pose, const mnr_camera* cam, int32_t H, int32_t W,
                               int32_t spp, const mnr_opts* opts, const int32_t* pixel_ids,
                               int32_t n_rays, const float* t_chunks, const float* grad_rgba,
                               float* grad_table, float* const* grad_w, float* grad_weights,
                               float* grad_bones, float* const* grad_res, void* workspace,
                               void* adjoint_ws, uint64_t adjoint_ws_bytes, void* stream);

/* Bytes of the adjoint workspace for a batch of n_rays rays of spp samples:
 * binned-scatter room for a record per sample, keyed level and corner and
 * for 4 per sample and bone (12 bytes each, twice) plus bin histograms and
 * the summing items -- about 5.4 KB per sample for the 16 levels of a
 * 2^19-row table and 24 bones, none when the batch (>= 2^31 records) or
 * table (hashed levels of more than 4096 x 2^14 rows) is too large for the
 * binned path -- plus, with a residual network or the frequency-encoded
 * field, 84 bytes per sample slot (n_rays * ceil(spp / 64) * 64 slots,
 * rounded up to 256 bytes) and 256 bytes, and for the frequency-encoded
 * field 512 bytes more per sample slot (its saved hidden activations);
 * then 4 bytes per ray (the processing order).  0: nothing to use it
 * for. */
uint64_t mnr_adjoint_ws_bytes(const mnr_field* field, const mnr_motion* motion, int32_t n_rays, int32_t spp);

/* Patch ray batch for training (Sec. 5.2: n_patches patches of size x size
 * pixels per image, so that patch losses can be taken): patch k's top-left
 * corner is drawn uniformly from the positions where the patch fits, from
 * SplitMix64 outputs (seed, 2k) and (seed, 2k + 1); out_ids (host int32
 * [n_patches * size * size]) lists each patch's pixels row by row, patches
 * in order.  MNR_E_SHAPE when a patch does not fit the image. */
mnr_status mnr_patch_rays(int32_t H, int32_t W, int32_t n_patches, int32_t size, uint64_t seed, int32_t* out_ids);

/* Squared-error loss of Eq. 14's MSE term over RGB: loss = mean over rays
 * and channels of (rgb - target)^2.  target: dev [n_rays][3].  Writes
 * grad_rgba dev [n_rays][4] (alpha gradient 0) and, if loss_out != NULL,
 * the loss to dev float loss_out[0]. */
mnr_status mnr_mse_loss(const float* rgba, const float* target, int32_t n_rays,
                        float* grad_rgba, float* loss_out, void* stream);

/* Canonical blend weights from free logits (Sec. 4.2: W^c is produced per
 * voxel; the build's W^c is a per-voxel softmax over n_channels).
 * logits, weights: dev float [n_channels][n_voxels]. */
mnr_status mnr_softmax_fwd(const float* logits, float* weights, int32_t n_channels,
                           int64_t n_voxels, void* stream);
/* Softmax adjoint: grad_logits[c] += w[c] * (g[c] - sum_k w[k] g[k]). */
mnr_status mnr_softmax_bwd(const float* weights, const float* grad_weights, float* grad_logits,
                           int32_t n_channels, int64_t n_voxels, void* stream);

/* Adam (Sec. 5.2: beta1 = 0.9, beta2 = 0.99).  Updates dev float param,
 * m, v [n] in place from grad [n] at step `step` (1-based, bias corrected),
 * then, if lowp != NULL, writes the rounded (RNE) copy of param to lowp in
 * lowp_dtype (F16 or BF16). */
mnr_status mnr_adam_step(float* param, const float* grad, float* m, float* v, int64_t n,
                         float lr, float beta1, float beta2, float eps, int32_t step,
                         void* lowp, mnr_dtype lowp_dtype, void* stream);

/* Skeleton-motion CNN (Sec. 4.2, Eq. 10, Fig. 7): the source of the
 * canonical blend-weight logits, from a constant latent z:
 *   a0 = LeakyReLU(w_fc z)                       (c0 channels at one voxel)
 *   a_k = LeakyReLU(TConv_k(a_{k-1})), k = 1..4, logits = TConv_5(a_4),
 * TConv = 3-D transposed convolution, kernel 4, stride 2, padding 1 (the
 * grid doubles 1 -> 32), LeakyReLU slope 0.2, no biases.  logits: dev
 * [c5][32^3], x fastest; c5 = n_bones + 1 feeds mnr_softmax_fwd for a
 * motion volume of res 32.  Dev FP32 weights: w_fc [c0][latent],
 * w[k] [c_k][c_{k+1}][4][4][4] (input channel, output channel, kz, ky,
 * kx).  1 <= latent <= 4096, 1 <= c_k <= 1024. */
typedef struct {
  int32_t latent;
  int32_t channels[6];
  const float* z;
  const float* w_fc;
  const float* w[5];
} mnr_skel_cnn;

/* Floats of the activations a0..a4 the forward saves for the adjoint, and
 * of the adjoint's scratch; 0 for an invalid network. */
uint64_t mnr_skel_cnn_act_floats(const mnr_skel_cnn* cnn);
uint64_t mnr_skel_cnn_scratch_floats(const mnr_skel_cnn* cnn);
/* act: dev [mnr_skel_cnn_act_floats]; logits: dev [c5][32^3]. */
mnr_status mnr_skel_cnn_forward(const mnr_skel_cnn* cnn, float* act, float* logits, void* stream);
/* ACCUMULATES dL/dw_fc and dL/dw[k] (dev, same shapes) from grad_logits
 * (dev [c5][32^3]) and the forward's act; scratch: dev
 * [mnr_skel_cnn_scratch_floats]. */
mnr_status mnr_skel_cnn_backward(const mnr_skel_cnn* cnn, const float* act, const float* grad_logits,
                                 float* grad_w_fc, float* const* grad_w, float* scratch, void* stream);

/* dst = round-to-nearest-even(src) in dtype (F16 or BF16); n elements. */
mnr_status mnr_convert(const float* src, void* dst, mnr_dtype dtype, int64_t n, void* stream);
/* Zero n_bytes of dev memory with a kernel (safe inside captured graphs). */
mnr_status mnr_zero(void* dst, size_t n_bytes, void* stream);

/* One training step (Sec. 5.2): forward, MSE loss, adjoint, softmax adjoint
 * and Adam on every learnable tensor.  The field's table/MLP pointers are
 * the low-precision copies read by the renderer (they may alias the fp32
 * masters when the dtypes are F32).  Learning rates: lr_field for the
 * table and MLP, lr_motion for the logits.  All buffers are caller-owned
 * device memory; the state struct lists them. */
typedef struct {
  float* table_master; float* table_grad; float* table_m; float* table_v; /* [L*T*F]; NULL for the
                                                                             frequency-encoded field */
  float* w_master[MNR_MAX_LAYERS]; float* w_grad[MNR_MAX_LAYERS];
  float* w_m[MNR_MAX_LAYERS]; float* w_v[MNR_MAX_LAYERS];
  float* logits; float* logits_grad; float* logits_m; float* logits_v;    /* [(n_bones+1)*res^3] */
  float* weights_grad;                                                    /* dL/dW^c scratch */
  float* rgba; float* grad_rgba;                                          /* [n_rays][4] scratch */
  float* t_chunks;                                    /* [n_rays][ceil(spp/64) + 1] scratch */
  float* loss;                                                            /* [1] */
  void* workspace;                                           /* MNR_WORKSPACE_BYTES, or NULL */
  void* adjoint_ws; uint64_t adjoint_ws_bytes;   /* see mnr_render_backward; required with a residual network
                                                    or the frequency-encoded field */
  /* Residual motion network (when motion->res_w[0] != NULL): FP32 masters,
   * gradients and Adam moments of W1..W5, W_omega (shapes as motion->res_w);
   * Adam at lr_res updates the masters and rewrites the BF16 copies
   * motion->res_w[k] (which the step therefore writes). */
  float* res_master[6]; float* res_grad[6]; float* res_m[6]; float* res_v[6];
  float lr_res;
  float lr_field, lr_motion, beta1, beta2, eps;
  int32_t step;                                                           /* 1-based */
  int32_t train_motion;  /* 0 = logits frozen; 1 = Adam on the logits; 2 = only dL/dlogits into logits_grad
                            (their source, e.g. the skeleton-motion CNN, is the caller's to update) */
} mnr_train_state;

mnr_status mnr_train_step(const mnr_field* field, const mnr_motion* motion, const mnr_pose* pose,
                          const mnr_camera* cam, int32_t H, int32_t W, int32_t spp,
                          const mnr_opts* opts, const int32_t* pixel_ids, int32_t n_rays,
                          const float* target, mnr_train_state* state, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* METANERF_H */
