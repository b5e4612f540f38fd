// C-ABI entry points: validation on the host, argument packing, launches on
// the caller's stream.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "host_common.h"
#include "kernels.h"

namespace mnr {

static thread_local char g_err[512];

void clear_error() { g_err[0] = 0; }

mnr_status fail(mnr_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

static mnr_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return MNR_OK;
  return fail(MNR_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

static bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

static mnr_status check_box(const float* lo, const float* hi, const char* who) {
  if (!finite3(lo) || !finite3(hi)) return fail(MNR_E_INVALID, "%s: non-finite box", who);
  for (int a = 0; a < 3; ++a)
    if (!(hi[a] > lo[a])) return fail(MNR_E_INVALID, "%s: box_max must exceed box_min", who);
  return MNR_OK;
}

static mnr_status validate_freq_field(const mnr_field* f) {
  if (f->mlp_dtype != MNR_BF16)
    return fail(MNR_E_UNSUPPORTED, "field: the frequency-encoded field needs the BF16 MLP path");
  if (f->n_layers != 5) return fail(MNR_E_SHAPE, "field: the frequency-encoded field has 5 layers, got %d", f->n_layers);
  const int want[6] = {64, 64, 64, 64, 64, 4};
  for (int k = 0; k < 6; ++k)
    if (f->width[k] != want[k]) return fail(MNR_E_SHAPE, "field: frequency-field widths must be 64,64,64,64,64,4");
  for (int k = 0; k < 5; ++k)
    if (!f->w[k]) return fail(MNR_E_INVALID, "field: null weight pointer for layer %d", k);
  return check_box(f->box_min, f->box_max, "field");
}

mnr_status validate_field(const mnr_field* f) {
  if (!f) return fail(MNR_E_INVALID, "field: null pointer");
  if (f->encoding == MNR_ENC_FREQ) return validate_freq_field(f);
  if (f->encoding != MNR_ENC_GRID) return fail(MNR_E_INVALID, "field: unknown encoding %d", f->encoding);
  if (!f->table) return fail(MNR_E_INVALID, "field: null pointer");
  if (f->n_feat != 2) return fail(MNR_E_SHAPE, "field: n_feat must be 2, got %d", f->n_feat);
  if (f->n_levels < 1 || f->n_levels > MNR_MAX_LEVELS || f->n_levels * f->n_feat != 32)
    return fail(MNR_E_SHAPE, "field: n_levels * n_feat must be 32 (n_levels %d)", f->n_levels);
  if (f->log2_T < 4 || f->log2_T > 24) return fail(MNR_E_SHAPE, "field: log2_T must be in [4, 24], got %d", f->log2_T);
  for (int l = 0; l < f->n_levels; ++l)
    if (f->level_res[l] < 1 || f->level_res[l] > 65535)
      return fail(MNR_E_SHAPE, "field: level_res[%d] = %d out of [1, 65535]", l, f->level_res[l]);
  if (f->table_dtype != MNR_F32 && f->table_dtype != MNR_F16) return fail(MNR_E_DTYPE, "field: table dtype must be F32 or F16");
  if (f->mlp_dtype != MNR_F32 && f->mlp_dtype != MNR_BF16) return fail(MNR_E_DTYPE, "field: MLP dtype must be F32 or BF16");
  if (f->n_layers < 2 || f->n_layers > 4) return fail(MNR_E_SHAPE, "field: n_layers must be in [2, 4], got %d", f->n_layers);
  if (f->width[0] != 32 || f->width[f->n_layers] != 4)
    return fail(MNR_E_SHAPE, "field: widths must run 32 -> ... -> 4");
  for (int k = 1; k < f->n_layers; ++k)
    if (f->width[k] != 64) return fail(MNR_E_SHAPE, "field: hidden width %d must be 64", f->width[k]);
  for (int k = 0; k < f->n_layers; ++k)
    if (!f->w[k]) return fail(MNR_E_INVALID, "field: null weight pointer for layer %d", k);
  if (f->dense_packed && ((uintptr_t)f->dense_packed & 15))
    return fail(MNR_E_INVALID, "field: dense_packed not 16-byte aligned");
  return check_box(f->box_min, f->box_max, "field");
}

mnr_status validate_common(const mnr_field* f, const mnr_motion* m, const mnr_pose* p, const mnr_camera* c,
                                  int H, int W, int spp, const mnr_opts* o, const int32_t* pixel_ids, int n_rays,
                                  const void* out) {
  if (mnr_status s = validate_field(f)) return s;
  if (mnr_status s = validate_pose(p)) return s;
  if (!m || !m->weights) return fail(MNR_E_INVALID, "motion: null pointer");
  if (m->n_bones != p->n_joints) return fail(MNR_E_SHAPE, "motion: n_bones %d != pose joints %d", m->n_bones, p->n_joints);
  if (m->res < 2 || m->res > 512) return fail(MNR_E_SHAPE, "motion: res must be in [2, 512], got %d", m->res);
  if (mnr_status s = check_box(m->box_min, m->box_max, "motion")) return s;
  if (m->packed && m->res > MAX_PACKED_RES)
    return fail(MNR_E_SHAPE, "motion: packed copy needs res <= %d, got %d", MAX_PACKED_RES, m->res);
  if (m->packed && ((uintptr_t)m->packed & 15)) return fail(MNR_E_INVALID, "motion: packed copy not 16-byte aligned");
  if (m->res_w[0]) {
    for (int k = 1; k < 6; ++k)
      if (!m->res_w[k]) return fail(MNR_E_INVALID, "motion: residual weight %d is null", k);
    if (!std::isfinite(m->res_alpha)) return fail(MNR_E_INVALID, "motion: non-finite res_alpha");
    if (f->mlp_dtype != MNR_BF16)
      return fail(MNR_E_UNSUPPORTED, "motion: the residual motion network needs the BF16 MLP path");
  }
  if (!c) return fail(MNR_E_INVALID, "camera: null pointer");
  if (!(c->fx > 0) || !(c->fy > 0) || !std::isfinite(c->fx) || !std::isfinite(c->fy) || !std::isfinite(c->cx) ||
      !std::isfinite(c->cy))
    return fail(MNR_E_INVALID, "camera: bad intrinsics");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(c->R_wc[i])) return fail(MNR_E_INVALID, "camera: non-finite rotation");
  if (!finite3(c->T)) return fail(MNR_E_INVALID, "camera: non-finite translation");
  if (mnr_status s = check_box(c->box_min, c->box_max, "camera")) return s;
  if (H < 1 || W < 1 || (int64_t)H * W > (1 << 28)) return fail(MNR_E_SHAPE, "image %dx%d out of range", H, W);
  if (spp < 1 || spp > MNR_MAX_SPP) return fail(MNR_E_SHAPE, "spp must be in [1, %d], got %d", MNR_MAX_SPP, spp);
  if (n_rays < 0) return fail(MNR_E_SHAPE, "n_rays must be >= 0");
  if (!pixel_ids && n_rays != 0 && n_rays != H * W) return fail(MNR_E_SHAPE, "full frame needs n_rays == H*W");
  if (!out && n_rays > 0) return fail(MNR_E_INVALID, "null output");
  if (o && (!(o->ert_tau >= 0) || !finite3(o->bg))) return fail(MNR_E_INVALID, "opts: bad ert_tau or bg");
  return MNR_OK;
}

// Packed copy of one dense level: (N+1) z-planes of N x N groups of four
// rows (2 features each).
static uint64_t dense_level_bytes(int N, mnr_dtype dt) {
  return (uint64_t)(N + 1) * N * N * 4 * 2 * (dt == MNR_F32 ? 4 : 2);
}

static bool level_is_dense(const mnr_field* f, int l) {
  const int64_t n1 = f->level_res[l] + 1;
  return n1 * n1 * n1 <= (int64_t(1) << f->log2_T);
}

void field_args(FieldArgs& F, const mnr_field* f) {
  std::memset(&F, 0, sizeof(F));
  for (int k = 0; k < f->n_layers; ++k) F.w[k] = f->w[k];
  F.n_layers = f->n_layers;
  for (int i = 0; i < 3; ++i) {
    F.gmin[i] = f->box_min[i];
    F.gscale[i] = (float)(1.0 / ((double)f->box_max[i] - f->box_min[i]));
  }
  if (f->encoding == MNR_ENC_FREQ) {  // no grid: levels, table and packed copy unused
    F.freq = 1;
    return;
  }
  F.table = f->table;
  F.dpk = (const char*)f->dense_packed;
  uint64_t off = 0;
  bool prefix = true;
  for (int l = 0; l < f->n_levels; ++l) {
    F.level_res[l] = f->level_res[l];
    if (level_is_dense(f, l)) {
      F.dense_mask |= 1u << l;
      F.dpk_off[l] = off;
      off += dense_level_bytes(f->level_res[l], f->table_dtype);
      if (prefix && F.dpk) F.n_packed = l + 1;
    } else {
      prefix = false;
    }
  }
  F.n_levels = f->n_levels;
  F.log2_T = f->log2_T;
}

void pack_args(RenderArgs& a, const mnr_field* f, const mnr_motion* m, const mnr_pose* p, const mnr_camera* c,
                      int H, int W, int spp, const mnr_opts* o, const int32_t* pixel_ids, int n_rays) {
  std::memset(&a, 0, sizeof(a));
  field_args(a.f, f);
  for (int i = 0; i < 3; ++i) {
    a.m.mmin[i] = m->box_min[i];
    a.m.mscale[i] = (float)((m->res - 1) / ((double)m->box_max[i] - m->box_min[i]));
  }
  a.m.weights = m->weights;
  a.m.packed = (const f4*)m->packed;
  a.m.res = m->res;
  a.m.n_bones = m->n_bones;
  if (m->res_w[0]) {
    for (int k = 0; k < 6; ++k) a.res.w[k] = (const __bf16*)m->res_w[k];
    for (int k = 0; k < 4; ++k) {  // truncated Hann window over the bands
      const double t = std::fmin(std::fmax((double)m->res_alpha - k, 0.0), 1.0);
      a.res.win[k] = (float)(0.5 * (1.0 - std::cos(M_PI * t)));
    }
    a.res.n_omega = 3 * p->n_joints;  // Omega: the observed pose theta^o's joint angles (Eq. 11)
    double om[3 * MNR_MAX_BONES];
    pose_angles_f64(p, om);
    for (int j = 0; j < 3 * p->n_joints; ++j) a.res.omega[j] = (float)om[j];
  }
  double G[MNR_MAX_BONES * 12];
  fk_bones_f64(p, G);
  for (int j = 0; j < p->n_joints; ++j)
    for (int k = 0; k < 12; ++k) a.G[j][k] = (float)G[12 * j + k];
  RayArgs& r = a.r;
  for (int i = 0; i < 9; ++i) r.Rwc[i] = c->R_wc[i];
  for (int i = 0; i < 3; ++i) {  // camera centre o = -R^T T
    r.origin[i] = -(r.Rwc[0 * 3 + i] * c->T[0] + r.Rwc[1 * 3 + i] * c->T[1] + r.Rwc[2 * 3 + i] * c->T[2]);
    r.bmin[i] = c->box_min[i];
    r.bmax[i] = c->box_max[i];
  }
  r.fx = c->fx; r.fy = c->fy; r.cx = c->cx; r.cy = c->cy;
  r.H = H; r.W = W; r.spp = spp; r.n_rays = n_rays;
  r.pixel_ids = pixel_ids;
  r.tiles_x = (W + 15) / 16;
  if (o) {
    r.ert_tau = o->ert_tau;
    for (int i = 0; i < 3; ++i) r.bg[i] = o->bg[i];
    r.stratified = o->stratified;
    r.seed = o->seed;
  } else {
    r.ert_tau = 1e-6f;
  }
}

int slot_count(int H, int W, const int32_t* pixel_ids, int n_rays) {
  if (pixel_ids) return n_rays;
  return ((W + 15) / 16) * ((H + 15) / 16) * 256;
}

}  // namespace mnr

using namespace mnr;

extern "C" {

const char* mnr_status_str(mnr_status s) {
  switch (s) {
    case MNR_OK: return "ok";
    case MNR_E_INVALID: return "invalid argument";
    case MNR_E_SHAPE: return "unsupported shape";
    case MNR_E_DTYPE: return "unsupported dtype";
    case MNR_E_OOM: return "over memory budget";
    case MNR_E_HIP: return "HIP error";
    case MNR_E_BUSY: return "busy";
    case MNR_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* mnr_last_error(void) { return g_err; }

const char* mnr_version(void) { return "metanerf-gfx950 0.1"; }

}  // extern "C"

// Work-queue counters of mnr_render_noalloc: a file-scope device array in
// place of the caller's workspace, MNR_NOALLOC_SCRATCH_BYTES per GPU, held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host it only names the symbol): the address each device
// gives it is looked up once per device and kept in g_scratch_dev.
static __device__ __align__(256) int32_t scratch[MNR_NOALLOC_SCRATCH_BYTES / sizeof(int32_t)];
static_assert(MNR_NOALLOC_SCRATCH_BYTES >= MNR_WORKSPACE_BYTES, "the queues need MNR_WORKSPACE_BYTES");

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[MAX_DEVICES];

// Device address of `scratch` on the current device (looked up on the first
// call on each device, with that device current).
static mnr_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "render_noalloc: hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) return fail(MNR_E_UNSUPPORTED, "render_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_status(e, "render_noalloc: hipGetSymbolAddress");
    if (!p) return fail(MNR_E_HIP, "render_noalloc: null scratch address");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return MNR_OK;
}

// ---- binned scatter of the table gradient (scatter.hip) ----

static uint64_t align256(uint64_t b) { return (b + 255) & ~(uint64_t)255; }

// Elements of MLP layer k: width[k+1] x width[k], except the frequency-
// encoded field's W4, whose input is [h3; gamma] (64 x 128).
static int64_t layer_elems(const mnr_field* f, int k) {
  if (f->encoding == MNR_ENC_FREQ && k == 3) return 64 * 128;
  return (int64_t)f->width[k] * f->width[k + 1];
}

// Rows of a dense level: (N+1)^3.
static int64_t dense_rows(const mnr_field* f, int l) {
  const int64_t n1 = (int64_t)f->level_res[l] + 1;
  return n1 * n1 * n1;
}

// Key map of the binned scatter: the hashed levels (T keys each), then,
// when the key space holds them too, the dense levels ((N+1)^3 keys each,
// in level order; else they keep run-summed atomics), then, from a multiple
// of 2^MAX_BIN_SHIFT, the blend-weight gradient's n_bones x res^3 elements
// when they fit and res is a power of two up to 2^12 (else global atomics).
// Returns the number of keys (0: nothing keyed).
static int64_t key_map(const mnr_field* f, const mnr_motion* m, KeyMap* map, bool* dense, bool* wc) {
  const int64_t limit = (int64_t)MAX_BINS << MAX_BIN_SHIFT;
  KeyMap k{};
  k.log2_T = f->log2_T;
  int64_t n_keys = 0;
  bool with_dense = false;
  if (f->encoding == MNR_ENC_GRID) {
    for (int l = 0; l < f->n_levels; ++l)
      if (!level_is_dense(f, l)) {
        k.start[k.n] = (uint32_t)n_keys;
        k.level[k.n++] = l;
        n_keys += (int64_t)1 << f->log2_T;
      }
    int64_t all = n_keys;
    for (int l = 0; l < f->n_levels; ++l)
      if (level_is_dense(f, l)) all += dense_rows(f, l);
    with_dense = all <= limit;
    if (with_dense)
      for (int l = 0; l < f->n_levels; ++l)
        if (level_is_dense(f, l)) {
          k.start[k.n] = (uint32_t)n_keys;
          k.level[k.n++] = l;
          n_keys += dense_rows(f, l);
        }
  }
  k.start[k.n] = (uint32_t)n_keys;
  const int64_t R = m ? m->res : 0;
  const int64_t wc_keys = m ? (int64_t)m->n_bones * R * R * R : 0;
  const int64_t wc0 = (n_keys + ((int64_t)1 << MAX_BIN_SHIFT) - 1) & ~(((int64_t)1 << MAX_BIN_SHIFT) - 1);
  const bool with_wc = wc_keys > 0 && (R & (R - 1)) == 0 && R <= 4096 && wc0 + wc_keys <= limit;
  k.wc_start = k.wc_end = (uint32_t)n_keys;
  if (with_wc) {
    k.wc_start = (uint32_t)wc0;
    k.wc_end = (uint32_t)(wc0 + wc_keys);
    n_keys = wc0 + wc_keys;
  }
  if (map) *map = k;
  if (dense) *dense = with_dense;
  if (wc) *wc = with_wc;
  return n_keys;
}

// Carves the caller's scatter workspace; returns its size (0: nothing
// keyed, or the batch or table is too large for the binned path).
static uint64_t scatter_layout(const mnr_field* f, const mnr_motion* m, int n_rays, int spp, char* ws,
                               ScatterPlan* p) {
  KeyMap map;
  bool dense = false, wc = false;
  const int64_t n_keys = key_map(f, m, &map, &dense, &wc);
  if (n_keys == 0 || n_rays <= 0 || spp <= 0) return 0;
  // per sample: 8 records per keyed level, 4 per bone (corner pairs)
  const uint64_t per_sample = (uint64_t)map.n * 8 + (wc ? (uint64_t)m->n_bones * 4 : 0);
  const uint64_t cap = (uint64_t)n_rays * spp * per_sample;
  if (cap >= ((uint64_t)1 << 31)) return 0;
  const int shift = scatter_bin_shift(n_keys);
  if (shift > MAX_BIN_SHIFT) return 0;
  const int n_bins = (int)((n_keys + ((int64_t)1 << shift) - 1) >> shift);
  const int n_tiles = (int)((cap + BIN_TILE_RECORDS - 1) / BIN_TILE_RECORDS);
  // a bin of t records is summed by ceil(t / ACC_PART_RECORDS) blocks
  const int max_items = n_bins + (int)((cap + ACC_PART_RECORDS - 1) / ACC_PART_RECORDS);
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off += align256(bytes);
    return ws ? ws + o : nullptr;
  };
  char* cursor = take(256);
  char* keys = take(cap * 4);
  char* vals = take(cap * 8);
  char* skeys = take(cap * 4);
  char* svals = take(cap * 8);
  char* hist = take((uint64_t)n_bins * n_tiles * 4);
  char* seg = take((uint64_t)BIN_SEGS * n_bins * 4);
  char* total = take((uint64_t)n_bins * 4);
  char* base = take((uint64_t)n_bins * 4);
  char* item_base = take((uint64_t)n_bins * 4);
  char* item_bin = take((uint64_t)max_items * 4);
  char* n_items = take(4);
  if (p) {
    p->cursor = (uint32_t*)cursor;
    p->vmax = (uint32_t*)cursor + 16;  // (the cursor's 256 bytes are cleared before every adjoint)
    p->keys = (uint32_t*)keys;
    p->vals = (f2*)vals;
    p->skeys = (uint32_t*)skeys;
    p->svals = (f2*)svals;
    p->hist = (uint32_t*)hist;
    p->seg = (uint32_t*)seg;
    p->total = (uint32_t*)total;
    p->base = (uint32_t*)base;
    p->item_base = (uint32_t*)item_base;
    p->item_bin = (uint32_t*)item_bin;
    p->n_items = (uint32_t*)n_items;
    p->cap = (uint32_t)cap;
    p->shift = shift;
    p->n_bins = n_bins;
    p->n_tiles_cap = n_tiles;
    p->max_items = max_items;
    p->n_keys = n_keys;
    p->map = map;
    p->dense = dense;
    p->wc = wc;
  }
  return off;
}

// Per-sample scratch of the split adjoints (residual motion network,
// frequency-encoded field): the SPLIT_N arrays of n_rays * ceil(spp / 64) *
// 64 floats, 64 floats of layer-1 bias gradient, and for the
// frequency-encoded field the saved hidden activations (FREQ_ACT_BYTES per
// 64-sample chunk).
static uint64_t split_layout(const mnr_field* f, const mnr_motion* m, int n_rays, int spp, char* ws,
                             SplitArgs* sp) {
  const bool res = m && m->res_w[0], freq = f && f->encoding == MNR_ENC_FREQ;
  if (!(res || freq) || n_rays <= 0 || spp <= 0) return 0;
  const int64_t chunks = (int64_t)n_rays * ((spp + 63) / 64);
  const int64_t stride = chunks * 64;
  const uint64_t arrays = align256((uint64_t)SPLIT_N * stride * 4);
  const uint64_t act = freq ? (uint64_t)chunks * FREQ_ACT_BYTES : 0;
  if (sp) {
    sp->buf = (float*)ws;
    sp->stride = stride;
    sp->dbias = (float*)(ws + arrays);
    sp->act = act ? (void*)(ws + arrays + 256) : nullptr;
  }
  return arrays + 256 + act;
}

// The adjoint workspace: the binned scatter's part (table and blend-weight
// gradient records), then the split adjoint's (with a residual network or
// the frequency-encoded field), then (with either) a ray list's processing
// order (n_rays rows).
static uint64_t adjoint_layout(const mnr_field* f, const mnr_motion* m, int n_rays, int spp, char* ws,
                               ScatterPlan* p, SplitArgs* sp, int32_t** order = nullptr) {
  const uint64_t a = scatter_layout(f, m, n_rays, spp, ws, p);
  const uint64_t b = split_layout(f, m, n_rays, spp, ws ? ws + a : nullptr, sp);
  const uint64_t c = (a + b) ? align256((uint64_t)n_rays * 4) : 0;
  if (order) *order = (ws && c) ? (int32_t*)(ws + a + b) : nullptr;
  return a + b + c;
}

// Validates a caller's adjoint workspace and points the adjoint at it.
static mnr_status adjoint_setup(const mnr_field* f, const mnr_motion* m, int n_rays, int spp, void* ws,
                                uint64_t ws_bytes, RecordSink& rec, ScatterPlan& p, SplitArgs& sp,
                                int32_t*& order) {
  rec = RecordSink{nullptr, nullptr, nullptr, 0, 0, 0, 0u, nullptr};
  sp = SplitArgs{nullptr, 0, nullptr, nullptr};
  order = nullptr;
  if (!ws) {
    if (m->res_w[0]) return fail(MNR_E_INVALID, "the residual network's adjoint needs the adjoint workspace");
    if (f->encoding == MNR_ENC_FREQ)
      return fail(MNR_E_INVALID, "the frequency-encoded field's adjoint needs the adjoint workspace");
    return MNR_OK;
  }
  if ((uintptr_t)ws & 255) return fail(MNR_E_INVALID, "adjoint workspace not 256-byte aligned");
  ScatterPlan pp{};
  SplitArgs ss{nullptr, 0, nullptr, nullptr};
  int32_t* ord = nullptr;
  const uint64_t need = adjoint_layout(f, m, n_rays, spp, (char*)ws, &pp, &ss, &ord);
  if (need == 0) return fail(MNR_E_UNSUPPORTED, "adjoint workspace: nothing to use it for (nothing keyed, no residual network, not the frequency-encoded field, or a batch or table too large)");
  if (ws_bytes < need)
    return fail(MNR_E_SHAPE, "adjoint workspace has %llu bytes, needs %llu", (unsigned long long)ws_bytes,
                (unsigned long long)need);
  if (scatter_layout(f, m, n_rays, spp, nullptr, nullptr)) {
    p = pp;
    rec = RecordSink{p.cursor, p.keys, p.vals, p.cap, p.dense ? 1 : 0, p.wc ? 1 : 0, p.map.wc_start, p.vmax};
  }
  sp = ss;
  order = ord;
  return MNR_OK;
}

// With a ray list and room in the adjoint workspace: the spatially coherent
// processing order, computed on the stream.
static hipError_t order_rays(RenderArgs& a, int32_t* order, hipStream_t st) {
  if (!a.r.pixel_ids || !order) return hipSuccess;
  a.r.order = order;
  return launch_ray_order(a.r.pixel_ids, a.r.n_rays, a.r.H, a.r.W, order, st);
}

// The adjoint's launches: with the residual network or the frequency-
// encoded field, the split chain (residual forward, field adjoint, residual
// and skinning adjoints), else the fused kernel; the binned scatter after
// every kernel that writes records.
static hipError_t adjoint_launches(const RenderArgs& a, const ScatterPlan& plan, int slots, const mnr_field* f,
                                   float* grad_table, hipStream_t st) {
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  if (a.rec.keys) ok(launch_zero(plan.cursor, 256, st));
  const bool res = a.res.w[0] != nullptr;
  if (res) {
    ok(launch_zero(a.split.dbias, 64 * sizeof(float), st));
    ok(launch_res_forward(a, slots, st));
  }
  if (a.f.freq) ok(launch_freq_backward(a, slots, st));
  else ok(launch_render_bwd(a, slots, f->table_dtype, f->mlp_dtype, f->n_layers - 2, st));
  if (res) ok(launch_res_backward(a, slots, st));
  if (a.split.buf) ok(launch_skin_backward(a, slots, st));
  if (a.rec.keys) ok(launch_binned_scatter(plan, grad_table, a.grad_weights, st));
  return e;
}

static mnr_status render_impl(const mnr_field* field, const mnr_motion* motion, const mnr_pose* pose,
                              const mnr_camera* cam, int32_t H, int32_t W, int32_t spp, const mnr_opts* opts,
                              const int32_t* pixel_ids, int32_t n_rays, float* out_rgba, float* t_chunks,
                              unsigned long long* n_evaluated, void* workspace, void* stream) {
  RenderArgs a;
  pack_args(a, field, motion, pose, cam, H, W, spp, opts, pixel_ids, n_rays);
  a.out = out_rgba;
  a.t_chunks = t_chunks;
  a.n_eval = n_evaluated;
  a.queues = (int32_t*)workspace;
  if (workspace) {
    if (mnr_status s = hip_status(launch_zero(workspace, MNR_WORKSPACE_BYTES, (hipStream_t)stream), "workspace")) return s;
  }
  return hip_status(launch_render_fwd(a, slot_count(H, W, pixel_ids, n_rays), field->table_dtype, field->mlp_dtype,
                                      field->n_layers - 2, (hipStream_t)stream),
                    "render launch");
}

extern "C" {

mnr_status mnr_render(const mnr_field* field, const mnr_motion* motion, const mnr_pose* pose, const mnr_camera* cam,
                      int32_t H, int32_t W, int32_t spp, const mnr_opts* opts, const int32_t* pixel_ids,
                      int32_t n_rays, float* out_rgba, float* t_chunks, unsigned long long* n_evaluated,
                      void* workspace, void* stream) {
  clear_error();
  if (mnr_status s = validate_common(field, motion, pose, cam, H, W, spp, opts, pixel_ids, n_rays, out_rgba)) return s;
  if (n_rays == 0) return MNR_OK;
  return render_impl(field, motion, pose, cam, H, W, spp, opts, pixel_ids, n_rays, out_rgba, t_chunks, n_evaluated,
                     workspace, stream);
}

mnr_status mnr_render_noalloc(const mnr_field* field, const mnr_motion* motion, const mnr_pose* pose,
                              const mnr_camera* cam, int32_t H, int32_t W, int32_t spp, const mnr_opts* opts,
                              const int32_t* pixel_ids, int32_t n_rays, float* out_rgba, float* t_chunks,
                              unsigned long long* n_evaluated, void* stream) {
  clear_error();
  if (mnr_status s = validate_common(field, motion, pose, cam, H, W, spp, opts, pixel_ids, n_rays, out_rgba)) return s;
  if (n_rays == 0) return MNR_OK;
  void* ws = nullptr;
  if (mnr_status s = scratch_address(&ws)) return s;
  return render_impl(field, motion, pose, cam, H, W, spp, opts, pixel_ids, n_rays, out_rgba, t_chunks, n_evaluated,
                     ws, stream);
}

uint64_t mnr_adjoint_ws_bytes(const mnr_field* field, const mnr_motion* motion, int32_t n_rays, int32_t spp) {
  if (!field || validate_field(field) != MNR_OK) return 0;
  return adjoint_layout(field, motion, n_rays, spp, nullptr, nullptr, nullptr);
}

mnr_status mnr_render_backward(const mnr_field* field, const mnr_motion* motion, const mnr_pose* pose,
                               const mnr_camera* cam, int32_t H, int32_t W, int32_t spp, const mnr_opts* opts,
                               const int32_t* pixel_ids, int32_t n_rays, const float* t_chunks,
                               const float* grad_rgba, float* grad_table, float* const* grad_w, float* grad_weights,
                               float* grad_bones, float* const* grad_res, void* workspace, void* adjoint_ws,
                               uint64_t adjoint_ws_bytes, void* stream) {
  clear_error();
  if (mnr_status s = validate_common(field, motion, pose, cam, H, W, spp, opts, pixel_ids, n_rays, t_chunks)) return s;
  if (motion->res_w[0]) {
    if (!grad_res) return fail(MNR_E_INVALID, "backward: null grad_res with a residual network");
    for (int k = 0; k < 6; ++k)
      if (!grad_res[k]) return fail(MNR_E_INVALID, "backward: null grad_res[%d]", k);
  }
  const bool freq = field->encoding == MNR_ENC_FREQ;
  if (!grad_rgba || (!grad_table && !freq) || !grad_w || !grad_weights)
    return fail(MNR_E_INVALID, "backward: null gradient buffer");
  for (int k = 0; k < field->n_layers; ++k)
    if (!grad_w[k]) return fail(MNR_E_INVALID, "backward: null grad_w[%d]", k);
  if (n_rays == 0) return MNR_OK;
  RenderArgs a;
  pack_args(a, field, motion, pose, cam, H, W, spp, opts, pixel_ids, n_rays);
  a.t_chunks = (float*)t_chunks;
  a.grad_rgba = grad_rgba;
  a.grad_table = grad_table;
  for (int k = 0; k < field->n_layers; ++k) a.grad_w[k] = grad_w[k];
  a.grad_weights = grad_weights;
  a.grad_G = grad_bones;
  if (motion->res_w[0])
    for (int k = 0; k < 6; ++k) a.grad_res[k] = grad_res[k];
  ScatterPlan plan{};
  int32_t* order = nullptr;
  if (mnr_status s = adjoint_setup(field, motion, n_rays, spp, adjoint_ws, adjoint_ws_bytes, a.rec, plan, a.split,
                                   order))
    return s;
  a.queues = (int32_t*)workspace;
  hipStream_t st = (hipStream_t)stream;
  if (workspace) {
    if (mnr_status s = hip_status(launch_zero(workspace, MNR_WORKSPACE_BYTES, st), "workspace")) return s;
  }
  if (mnr_status s = hip_status(order_rays(a, order, st), "ray order")) return s;
  return hip_status(adjoint_launches(a, plan, slot_count(H, W, pixel_ids, n_rays), field, grad_table, st),
                    "backward launch");
}

mnr_status mnr_mse_loss(const float* rgba, const float* target, int32_t n_rays, float* grad_rgba, float* loss_out,
                        void* stream) {
  clear_error();
  if (n_rays < 0) return fail(MNR_E_SHAPE, "mse: n_rays < 0");
  if (n_rays == 0) return MNR_OK;
  if (!rgba || !target || !grad_rgba) return fail(MNR_E_INVALID, "mse: null pointer");
  return hip_status(launch_mse(rgba, target, n_rays, grad_rgba, loss_out, (hipStream_t)stream), "mse launch");
}

mnr_status mnr_softmax_fwd(const float* logits, float* weights, int32_t n_channels, int64_t n_voxels, void* stream) {
  clear_error();
  if (!logits || !weights) return fail(MNR_E_INVALID, "softmax: null pointer");
  if (n_channels < 1 || n_channels > 64 || n_voxels < 0) return fail(MNR_E_SHAPE, "softmax: bad shape");
  if (n_voxels == 0) return MNR_OK;
  return hip_status(launch_softmax_fwd(logits, weights, n_channels, n_voxels, (hipStream_t)stream), "softmax launch");
}

static uint64_t splitmix64_host(uint64_t seed, uint64_t n) {  // n-th output of SplitMix64 (Steele et al. 2014)
  uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

mnr_status mnr_patch_rays(int32_t H, int32_t W, int32_t n_patches, int32_t size, uint64_t seed, int32_t* out_ids) {
  clear_error();
  if (!out_ids) return fail(MNR_E_INVALID, "patch_rays: null output");
  if (H < 1 || W < 1 || n_patches < 1 || size < 1 || size > H || size > W)
    return fail(MNR_E_SHAPE, "patch_rays: %d patches of %d^2 do not fit a %dx%d image", n_patches, size, H, W);
  int32_t* o = out_ids;
  for (int k = 0; k < n_patches; ++k) {
    const uint64_t ny = (uint64_t)(H - size + 1), nx = (uint64_t)(W - size + 1);
    const int y0 = (int)(((splitmix64_host(seed, 2 * (uint64_t)k) >> 11) * ny) >> 53);
    const int x0 = (int)(((splitmix64_host(seed, 2 * (uint64_t)k + 1) >> 11) * nx) >> 53);
    for (int y = 0; y < size; ++y)
      for (int x = 0; x < size; ++x) *o++ = (y0 + y) * W + x0 + x;
  }
  return MNR_OK;
}

uint64_t mnr_field_packed_bytes(const mnr_field* f) {
  clear_error();
  if (validate_field(f) != MNR_OK || f->encoding == MNR_ENC_FREQ) return 0;
  uint64_t b = 0;
  for (int l = 0; l < f->n_levels; ++l)
    if (level_is_dense(f, l)) b += dense_level_bytes(f->level_res[l], f->table_dtype);
  return b;
}

mnr_status mnr_field_pack(const mnr_field* f, void* stream) {
  clear_error();
  if (mnr_status s = validate_field(f)) return s;
  if (f->encoding == MNR_ENC_FREQ) return MNR_OK;  // no grid levels to pack
  if (!f->dense_packed) return fail(MNR_E_INVALID, "field_pack: null dense_packed");
  FieldArgs F;
  field_args(F, f);
  if (F.dense_mask == 0) return MNR_OK;
  return hip_status(launch_pack_dense(F, f->table_dtype, (hipStream_t)stream), "field_pack launch");
}

uint64_t mnr_motion_packed_bytes(int32_t res, int32_t n_bones) {
  if (res < 2 || res > MAX_PACKED_RES || n_bones < 1 || n_bones > MNR_MAX_BONES) return 0;
  return (uint64_t)n_bones * res * (res + 1) * (res + 1) * sizeof(f4);
}

mnr_status mnr_motion_pack(const mnr_motion* m, void* stream) {
  clear_error();
  if (!m || !m->weights || !m->packed) return fail(MNR_E_INVALID, "motion_pack: null pointer");
  if (((uintptr_t)m->packed & 15)) return fail(MNR_E_INVALID, "motion_pack: packed copy not 16-byte aligned");
  if (mnr_motion_packed_bytes(m->res, m->n_bones) == 0)
    return fail(MNR_E_SHAPE, "motion_pack: res %d / n_bones %d out of range", m->res, m->n_bones);
  return hip_status(launch_pack_motion(m->weights, (f4*)m->packed, m->n_bones, m->res, (hipStream_t)stream),
                    "motion_pack launch");
}

mnr_status mnr_softmax_bwd(const float* weights, const float* grad_weights, float* grad_logits, int32_t n_channels,
                           int64_t n_voxels, void* stream) {
  clear_error();
  if (!weights || !grad_weights || !grad_logits) return fail(MNR_E_INVALID, "softmax_bwd: null pointer");
  if (n_channels < 1 || n_channels > 64 || n_voxels < 0) return fail(MNR_E_SHAPE, "softmax_bwd: bad shape");
  if (n_voxels == 0) return MNR_OK;
  return hip_status(launch_softmax_bwd(weights, grad_weights, grad_logits, n_channels, n_voxels, (hipStream_t)stream),
                    "softmax_bwd launch");
}

mnr_status mnr_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, float lr, float beta1,
                         float beta2, float eps, int32_t step, void* lowp, mnr_dtype lowp_dtype, void* stream) {
  clear_error();
  if (!param || !grad || !m || !v) return fail(MNR_E_INVALID, "adam: null pointer");
  if (n < 0 || step < 1) return fail(MNR_E_SHAPE, "adam: n >= 0 and step >= 1 required");
  if (!(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0 && std::isfinite(lr)))
    return fail(MNR_E_INVALID, "adam: bad hyper-parameters");
  if (lowp && lowp_dtype != MNR_F16 && lowp_dtype != MNR_BF16) return fail(MNR_E_DTYPE, "adam: low-precision copy must be F16 or BF16");
  if (n == 0) return MNR_OK;
  return hip_status(launch_adam(param, grad, m, v, n, lr, beta1, beta2, eps, step, lowp, lowp_dtype, (hipStream_t)stream),
                    "adam launch");
}

mnr_status mnr_convert(const float* src, void* dst, mnr_dtype dtype, int64_t n, void* stream) {
  clear_error();
  if (!src || !dst) return fail(MNR_E_INVALID, "convert: null pointer");
  if (dtype != MNR_F16 && dtype != MNR_BF16) return fail(MNR_E_DTYPE, "convert: dtype must be F16 or BF16");
  if (n < 0) return fail(MNR_E_SHAPE, "convert: n < 0");
  if (n == 0) return MNR_OK;
  return hip_status(launch_convert(src, dst, dtype, n, (hipStream_t)stream), "convert launch");
}

mnr_status mnr_zero(void* dst, size_t n_bytes, void* stream) {
  clear_error();
  if (!dst && n_bytes) return fail(MNR_E_INVALID, "zero: null pointer");
  if (n_bytes % 4) return fail(MNR_E_SHAPE, "zero: size must be a multiple of 4 bytes");
  if (n_bytes == 0) return MNR_OK;
  return hip_status(launch_zero(dst, n_bytes, (hipStream_t)stream), "zero launch");
}

mnr_status mnr_train_step(const mnr_field* field, const mnr_motion* motion, const mnr_pose* pose,
                          const mnr_camera* cam, int32_t H, int32_t W, int32_t spp, const mnr_opts* opts,
                          const int32_t* pixel_ids, int32_t n_rays, const float* target, mnr_train_state* st,
                          void* stream) {
  clear_error();
  if (!st || !target) return fail(MNR_E_INVALID, "train_step: null state or target");
  if (mnr_status s = validate_common(field, motion, pose, cam, H, W, spp, opts, pixel_ids, n_rays, st->rgba)) return s;
  const bool freq = field->encoding == MNR_ENC_FREQ;  // no grid table: only the MLP (and motion) train
  if (motion->res_w[0])
    for (int k = 0; k < 6; ++k)
      if (!st->res_master[k] || !st->res_grad[k] || !st->res_m[k] || !st->res_v[k])
        return fail(MNR_E_INVALID, "train_step: null residual-network state buffer %d", k);
  if ((!freq && (!st->table_master || !st->table_grad || !st->table_m || !st->table_v)) || !st->weights_grad ||
      !st->grad_rgba || !st->loss || !st->t_chunks)
    return fail(MNR_E_INVALID, "train_step: null state buffer");
  for (int k = 0; k < field->n_layers; ++k)
    if (!st->w_master[k] || !st->w_grad[k] || !st->w_m[k] || !st->w_v[k])
      return fail(MNR_E_INVALID, "train_step: null state buffer for layer %d", k);
  if (st->train_motion < 0 || st->train_motion > 2) return fail(MNR_E_INVALID, "train_step: train_motion must be 0, 1 or 2");
  if (st->train_motion == 2 && !st->logits_grad) return fail(MNR_E_INVALID, "train_step: null logits_grad");
  if (st->train_motion == 1 && (!st->logits || !st->logits_grad || !st->logits_m || !st->logits_v))
    return fail(MNR_E_INVALID, "train_step: null logits state");
  if (!freq && field->table_dtype == MNR_F32 && field->table != st->table_master)
    return fail(MNR_E_INVALID, "train_step: an F32 table must be the master copy itself");
  for (int k = 0; k < field->n_layers; ++k)
    if (field->mlp_dtype == MNR_F32 && field->w[k] != st->w_master[k])
      return fail(MNR_E_INVALID, "train_step: F32 weights must be the master copies themselves");
  if (st->step < 1) return fail(MNR_E_SHAPE, "train_step: step must be >= 1");
  if (n_rays == 0) return MNR_OK;
  ScatterPlan plan{};
  RecordSink rec{};
  SplitArgs split{};
  int32_t* order = nullptr;
  if (mnr_status r = adjoint_setup(field, motion, n_rays, spp, st->adjoint_ws, st->adjoint_ws_bytes, rec, plan, split,
                                   order))
    return r;
  hipStream_t s = (hipStream_t)stream;
  const int64_t T = int64_t(1) << field->log2_T;
  const int64_t n_table = freq ? 0 : (int64_t)field->n_levels * T * field->n_feat;
  const int64_t n_vox = (int64_t)motion->res * motion->res * motion->res;
  const int64_t n_wc = (int64_t)(motion->n_bones + 1) * n_vox;
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t r) { if (e == hipSuccess) e = r; return r == hipSuccess; };
  // every gradient buffer (and the render queues) cleared in one launch
  ZeroList zl{};
  auto clear = [&](void* p, int64_t bytes) {
    zl.p[zl.n] = p;
    zl.bytes[zl.n++] = bytes;
  };
  if (n_table) clear(st->table_grad, n_table * 4);
  for (int k = 0; k < field->n_layers; ++k) clear(st->w_grad[k], layer_elems(field, k) * 4);
  clear(st->weights_grad, n_wc * 4);
  const int64_t n_omega = 3 * (int64_t)motion->n_bones;
  const int64_t res_n[6] = {64 * 32, 64 * 64, 64 * 64, 64 * 96, 3 * 64, 64 * n_omega};  // W1..W5, W_omega
  if (motion->res_w[0])
    for (int k = 0; k < 6; ++k) clear(st->res_grad[k], res_n[k] * 4);
  if (st->train_motion == 2) clear(st->logits_grad, n_wc * 4);  // (the softmax adjoint accumulates into it)
  if (st->workspace) clear(st->workspace, MNR_WORKSPACE_BYTES);
  ok(launch_zero_list(zl, s));
  RenderArgs a;
  pack_args(a, field, motion, pose, cam, H, W, spp, opts, pixel_ids, n_rays);
  const int slots = slot_count(H, W, pixel_ids, n_rays);
  a.out = st->rgba;
  a.t_chunks = st->t_chunks;
  a.queues = (int32_t*)st->workspace;
  ok(order_rays(a, order, s));  // forward and adjoint in the same coherent order
  ok(launch_render_fwd(a, slots, field->table_dtype, field->mlp_dtype, field->n_layers - 2, s));
  ok(launch_mse(st->rgba, target, n_rays, st->grad_rgba, st->loss, s));
  a.grad_rgba = st->grad_rgba;
  a.grad_table = st->table_grad;
  for (int k = 0; k < field->n_layers; ++k) a.grad_w[k] = st->w_grad[k];
  a.grad_weights = st->weights_grad;
  a.rec = rec;
  a.split = split;
  if (motion->res_w[0])
    for (int k = 0; k < 6; ++k) a.grad_res[k] = st->res_grad[k];
  if (st->workspace) ok(launch_zero(st->workspace, MNR_WORKSPACE_BYTES, s));
  ok(adjoint_launches(a, plan, slots, field, st->table_grad, s));
  if (motion->res_w[0]) {  // Adam on the residual network's FP32 masters, then its BF16 copies
    AdamList rl{};
    for (int k = 0; k < 6; ++k) {
      rl.p[k] = st->res_master[k];
      rl.g[k] = st->res_grad[k];
      rl.m[k] = st->res_m[k];
      rl.v[k] = st->res_v[k];
      rl.low[k] = (void*)motion->res_w[k];
      rl.n[k] = res_n[k];
    }
    rl.count = 6;
    ok(launch_adam_list(rl, st->lr_res, st->beta1, st->beta2, st->eps, st->step, MNR_BF16, s));
  }
  if (n_table)
    ok(launch_adam(st->table_master, st->table_grad, st->table_m, st->table_v, n_table, st->lr_field, st->beta1,
                   st->beta2, st->eps, st->step, field->table_dtype == MNR_F32 ? nullptr : (void*)field->table,
                   field->table_dtype, s));
  if (field->dense_packed && a.f.dense_mask) ok(launch_pack_dense(a.f, field->table_dtype, s));
  AdamList ml{};  // the MLP's layers in one launch
  for (int k = 0; k < field->n_layers; ++k) {
    ml.p[k] = st->w_master[k];
    ml.g[k] = st->w_grad[k];
    ml.m[k] = st->w_m[k];
    ml.v[k] = st->w_v[k];
    ml.low[k] = field->mlp_dtype == MNR_F32 ? nullptr : (void*)field->w[k];
    ml.n[k] = layer_elems(field, k);
  }
  ml.count = field->n_layers;
  ok(launch_adam_list(ml, st->lr_field, st->beta1, st->beta2, st->eps, st->step, field->mlp_dtype, s));
  if (st->train_motion == 2)  // dL/dlogits for the skeleton CNN's adjoint (logits_grad was cleared above)
    ok(launch_softmax_bwd(motion->weights, st->weights_grad, st->logits_grad, motion->n_bones + 1, n_vox, s));
  if (st->train_motion == 1) {  // softmax adjoint, Adam and softmax in one pass, then the packed copy
    ok(launch_motion_step(st->logits, (float*)motion->weights, st->weights_grad, st->logits_grad, st->logits_m,
                          st->logits_v, motion->n_bones + 1, n_vox, st->lr_motion, st->beta1, st->beta2, st->eps,
                          st->step, s));
    if (motion->packed)
      ok(launch_pack_motion(motion->weights, (f4*)motion->packed, motion->n_bones, motion->res, s));
  }
  return hip_status(e, "train_step launch");
}

}  // extern "C"
