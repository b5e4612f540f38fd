// Device-side types and helpers shared by the gfx950 kernels.
//
// Wave64 throughout.  MFMA fragment conventions used by the MLP (gfx950):
//   v_mfma_f32_16x16x4_f32 : A[i][k] in lane i + 16k; B[k][j] in lane j + 16k;
//   v_mfma_f32_16x16x32_bf16: A[i][k] in lane i + 16(k/8), element k%8;
//                             B[k][j] in lane j + 16(k/8), element k%8;
//   both: D[i][j] in lane j + 16(i/4), element i%4.
// A layer's output tile (16 neurons x 16 samples) therefore leaves neuron
// 16t + 4g + e of sample c in lane c + 16g, element e; the next layer takes
// exactly those registers as its B operand by permuting the K order of the
// weights (done once, when weights are staged into LDS).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/metanerf.h"

namespace mnr {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

constexpr int WAVE = 64;
constexpr int WAVES_PER_BLOCK = 4;
constexpr int BLOCK = WAVE * WAVES_PER_BLOCK;
constexpr int HIDDEN = 64;      // hidden width
constexpr int IN_FEAT = 32;     // encoding width (16 levels x 2 features)
constexpr float EPS_L = 1e-6f;  // lower clamp of the skinning-weight sum

// Everything a render / adjoint launch needs, passed by value (kernarg
// segment, < 4 KiB) so that per-frame constants arrive through scalar loads.
struct FieldArgs {
  const void* table;
  const void* w[MNR_MAX_LAYERS];
  int32_t level_res[MNR_MAX_LEVELS];
  uint32_t dense_mask;  // bit l: level l stored densely
  int32_t n_levels, log2_T, n_layers;
  float gmin[3], gscale[3];  // u = (x - gmin) * gscale
  const char* dpk;           // optional packed copy of the dense levels (NULL: gather from table)
  uint64_t dpk_off[MNR_MAX_LEVELS];  // byte offset of each dense level in dpk
  int32_t n_packed;          // leading dense levels read from dpk (0 without it)
  int32_t freq;              // 1: frequency-encoded field with the skip MLP (no grid)
};

// Largest volume resolution with a packed copy: one bone's packed plane
// (R (R+1)^2 float4) must stay below the 2^31-byte buffer-offset range.
constexpr int MAX_PACKED_RES = 256;

struct MotionArgs {
  const float* weights;
  const f4* packed;  // optional packed copy of the bone channels (NULL: gather from weights)
  int32_t res, n_bones;
  float mmin[3], mscale[3];  // q = (y - mmin) * mscale, in voxel units
};

struct RayArgs {
  double Rwc[9];
  double origin[3];
  double fx, fy, cx, cy;
  double bmin[3], bmax[3];
  int32_t H, W, spp, n_rays;
  const int32_t* pixel_ids;  // NULL: full frame in 16x16-tile order
  const int32_t* order;      // ray list only: row of the ray that slot b processes (NULL: row b)
  int32_t tiles_x;           // full-frame tiling
  float ert_tau;
  float bg[3];
  int32_t stratified;
  uint64_t seed;
};

// Residual non-rigid motion network (BF16 weights; w[0] == NULL: off).
struct ResArgs {
  const __bf16* w[6];  // W1 [64][32], W2 [64][64], W3 [64][64], W4 [64][96], W5 [3][64], W_omega [64][n_omega]
  float win[4];        // Hann window weight of each frequency band
  float omega[MNR_MAX_BONES * 3];
  int32_t n_omega;
};

// Where the adjoint writes its gradient records (keys == NULL: it adds the
// gradients with global atomics instead).  Record i: key keys[i], values
// vals[i].  Grid table: key = the row's place among the keyed levels' rows,
// values = the two features' gradients.  Blend weights (when wc != 0):
// key = wc_key0 + element of dL/dW^c ([bone][z][y][x]), values = the
// gradients of that element and of the next one along x (zero when that is
// outside the volume): one record per pair of x-adjacent cell corners.
struct RecordSink {
  uint32_t* cursor;  // records written so far (zero before the adjoint)
  uint32_t* keys;
  f2* vals;
  uint32_t cap;      // capacity in records
  int32_t dense;     // 1: the dense levels leave as records too (keys after the hashed levels')
  int32_t wc;        // 1: the blend-weight gradient leaves as records too (else global atomics)
  uint32_t wc_key0;  // its first key
  uint32_t* vmax;    // [2] bound on |value| (float bits, integer max) of the table's and the blend
                     // weights' records: the binned sums' fixed-point scale (zero before the adjoint)
};

// Per-sample scratch of the split adjoint (used with the residual motion
// network): SoA arrays of `stride` floats, sample i of ray slot r at
// r * (nchunks * 64) + i.  Written and read by the adjoint's kernels in
// turn (the forward pass stores nothing per sample).
enum SplitField {
  SPLIT_X = 0,    // observed point x (3)
  SPLIT_XS = 3,   // skinned point x_skel (3)
  SPLIT_XF = 6,   // x_final = x_skel + x_res (3)
  SPLIT_L = 9,    // weight sum L; 0 for samples that are not live
  SPLIT_G = 10,   // dL/dx_final (3); without the residual network also dL/dx_skel
  SPLIT_GL = 13,  // dL/dL
  SPLIT_GO = 14,  // dL/d(raw field outputs) (4), frequency-encoded field
  SPLIT_GS = 18,  // dL/dx_skel (3), written by the residual network's adjoint
  SPLIT_N = 21
};
// Saved hidden activations of the frequency-encoded field's MLP per
// 64-sample chunk: 4 layers x 4 tiles x 2 halves x 64 lanes of 8 BF16.
constexpr int FREQ_ACT_VECS = 4 * 4 * 2 * 64;
constexpr int64_t FREQ_ACT_BYTES = FREQ_ACT_VECS * 16;
struct SplitArgs {
  float* buf;      // [SPLIT_N][stride], or NULL (fused adjoint)
  int64_t stride;
  float* dbias;    // [64]: sum over samples of dL/d(pre-activation of the residual network's layer 1)
  void* act;       // frequency-encoded field: FREQ_ACT_BYTES per chunk (chunk = ray row x nchunks + chunk)
};

struct RenderArgs {
  FieldArgs f;
  MotionArgs m;
  ResArgs res;
  RayArgs r;
  float G[MNR_MAX_BONES][12];
  float* out;                        // [n_rays][4]
  float* t_chunks;                   // [n_rays][nchunks] (forward writes, adjoint reads)
  unsigned long long* n_eval;        // optional counter
  int32_t* queues;                   // optional: 8 per-XCD work counters, zero at launch
  // adjoint only
  const float* grad_rgba;            // [n_rays][4]
  float* grad_table;
  float* grad_w[MNR_MAX_LAYERS];
  float* grad_weights;
  float* grad_G;                     // optional [n_bones][12]
  RecordSink rec;                    // optional: table and blend-weight gradients as records
  SplitArgs split;                   // split adjoint (residual motion network, frequency-encoded field)
  float* grad_res[6];                // residual network: W1..W5, W_omega (FP32)
};

// Server tick work table (device memory, uploaded per tick).
struct WorkItem {
  int32_t slot, tile;
};
struct WorkTable {
  int32_t counter;  // next item; 0 at upload
  int32_t n_items;
  int32_t pad[2];
  WorkItem items[1];  // n_items entries (allocated for the tick capacity)
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// SplitMix64 output n of the stream seeded with `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t n) {
  uint64_t z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Pixel id of ray slot b: explicit list, or full frame in 16x16 tiles
// (rows of tiles, row-major inside a tile) so that consecutive rays are
// 2-D neighbours.  Returns -1 for tile slots outside the image.
// Ray-list row processed by slot b: a spatially coherent order of the list
// when there is one (neighbouring slots share an XCD's work queue, so their
// gathers share its L2), else b.
__device__ __forceinline__ int ray_row(const RayArgs& r, int b) { return r.order ? r.order[b] : b; }

// Pixel of ray-list row b, or of full-frame slot b.
__device__ __forceinline__ int ray_pixel(const RayArgs& r, int b) {
  if (r.pixel_ids) return r.pixel_ids[b];
  const int tile = b >> 8, inner = b & 255;
  const int u = (tile % r.tiles_x) * 16 + (inner & 15);
  const int v = (tile / r.tiles_x) * 16 + (inner >> 4);
  return (u < r.W && v < r.H) ? v * r.W + u : -1;
}

// Per-ray set-up in double precision (shared by every lane of the wave):
// pinhole direction, slab clip against the body box.  Returns false on a
// miss.  p0 = o + t_near d, delta = (t_far - t_near) / spp.
struct RaySetup {
  float p0[3], d[3];
  float delta;
};

__device__ inline bool setup_ray(const RayArgs& r, int pix, RaySetup& s) {
  const double u = (double)(pix % r.W), v = (double)(pix / r.W);
  const double dc0 = (u + 0.5 - r.cx) / r.fx, dc1 = (v + 0.5 - r.cy) / r.fy, dc2 = 1.0;
  double d[3];
  for (int a = 0; a < 3; ++a) d[a] = r.Rwc[a] * dc0 + r.Rwc[3 + a] * dc1 + r.Rwc[6 + a] * dc2;
  const double inv = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int a = 0; a < 3; ++a) d[a] *= inv;
  double tmin = -INFINITY, tmax = INFINITY;
  for (int a = 0; a < 3; ++a) {
    const double o = r.origin[a];
    if (fabs(d[a]) < 1e-12) {
      if (o < r.bmin[a] || o > r.bmax[a]) return false;
    } else {
      const double t1 = (r.bmin[a] - o) / d[a], t2 = (r.bmax[a] - o) / d[a];
      tmin = fmax(tmin, fmin(t1, t2));
      tmax = fmin(tmax, fmax(t1, t2));
    }
  }
  const double tn = fmax(tmin, 0.0);
  if (!(tmax > tn)) return false;
  for (int a = 0; a < 3; ++a) {
    s.p0[a] = (float)(r.origin[a] + tn * d[a]);
    s.d[a] = (float)d[a];
  }
  s.delta = (float)((tmax - tn) / r.spp);
  return true;
}

// ---- wave-level scans (lane order = sample order along the ray) ----------

__device__ __forceinline__ float shfl_up(float v, int k) { return __shfl_up(v, k, WAVE); }
__device__ __forceinline__ float shfl_down(float v, int k) { return __shfl_down(v, k, WAVE); }

// Inclusive prefix product over lanes 0..lane.
__device__ __forceinline__ float wave_prefix_prod(float v) {
  const int l = lane_id();
#pragma unroll
  for (int k = 1; k < WAVE; k <<= 1) {
    const float o = shfl_up(v, k);
    if (l >= k) v *= o;
  }
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int k = WAVE / 2; k > 0; k >>= 1) v += __shfl_xor(v, k, WAVE);
  return v;
}

// Dynamic work pulling for one wave.  The units are split into 8 contiguous
// ranges, one per XCD queue; units close in index are close in the image,
// so each XCD's L2 serves a compact band of the frame (and the part of the
// body seen there).  A wave starts on its own XCD's range (q = blockIdx.x %
// 8), then steals from the next ones.  Returns the next unit, or -1 once
// every range is exhausted.
__device__ __forceinline__ int pull_unit(int32_t* queues, int n_units, int& q, int& tried) {
  const int per = (n_units + 7) >> 3;
  for (;;) {
    int local = 0;
    if (__lane_id() == 0) local = atomicAdd(queues + q, 1);
    local = __builtin_amdgcn_readfirstlane(local);
    const int unit = q * per + local;
    if (local < per && unit < n_units) return unit;
    if (++tried >= 8) return -1;
    q = (q + 1) & 7;
  }
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

}  // namespace mnr
