// Host-side launchers of the gfx950 kernels (implemented in the .hip files).
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_common.h"

namespace mnr {

// Persistent grid size of one kernel instantiation: compute units times the
// blocks per CU that its LDS and registers allow.  The first launch on any
// thread raises the kernel's dynamic-LDS limit and queries the occupancy
// under std::call_once; concurrent launchers (the server's scheduler thread
// and callers on other streams) wait for it and then only read the result.
// One process drives one GPU model, so the value is kept per instantiation,
// not per device.
struct PersistentGrid {
  std::once_flag once;
  int blocks = 1;
};

template <typename KernelT>
inline int persistent_blocks(KernelT kern, int threads, int lds, PersistentGrid& g) {
  std::call_once(g.once, [&] {
    int dev = 0, cus = 0, per_cu = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, threads, lds);
    g.blocks = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  });
  return g.blocks;
}

// Fused forward renderer.  n_slots: number of ray slots (n_rays, or the
// 16x16-tiled full frame).  nhh: number of 64->64 hidden layers.
hipError_t launch_render_fwd(const RenderArgs& a, int n_slots, mnr_dtype table_dt, mnr_dtype mlp_dt, int nhh,
                             hipStream_t st);

// Adjoint of the forward renderer (accumulates gradients).
hipError_t launch_render_bwd(const RenderArgs& a, int n_slots, mnr_dtype table_dt, mnr_dtype mlp_dt, int nhh,
                             hipStream_t st);

// Split adjoint with the residual motion network (res_bwd.hip): the warp
// and residual forward into the split scratch before the field's adjoint,
// and after it the residual network's and the skinning adjoints.
hipError_t launch_res_forward(const RenderArgs& a, int n_slots, hipStream_t st);
hipError_t launch_res_backward(const RenderArgs& a, int n_slots, hipStream_t st);
hipError_t launch_skin_backward(const RenderArgs& a, int n_slots, hipStream_t st);
hipError_t launch_freq_backward(const RenderArgs& a, int n_slots, hipStream_t st);

// Server tick: render the (slot, tile) items of wt with the requests' descriptors.
hipError_t launch_serve(const RenderArgs* slots, WorkTable* wt, mnr_dtype table_dt, mnr_dtype mlp_dt, int nhh, bool res,
                        bool freq, hipStream_t st);

// Binned scatter-add of the adjoint's table-gradient records (scatter.hip).
constexpr int MAX_BINS = 4096;
constexpr int MAX_BIN_SHIFT = 14;       // largest bin: 2^14 rows (summed in 2^12-row parts)
constexpr int BIN_TILE_RECORDS = 8192;  // records per histogram / scatter block
constexpr int ACC_PART_RECORDS = 65536; // records per summing block: larger bins are split
constexpr int BIN_SEGS = 64;            // tile segments of the per-bin scans
constexpr int BIN_SCAN_BINS = 256;      // bins per block of the segment scans
struct KeyMap {  // keyed level j: keys [start[j], start[j + 1]) are rows 0, 1, ... of table level level[j]
  int32_t level[MNR_MAX_LEVELS];
  uint32_t start[MNR_MAX_LEVELS + 1];
  int32_t n;                 // keyed levels: the hashed ones (T keys each), then the dense ones ((N+1)^3 each)
  int32_t log2_T;
  // keys [wc_start, wc_end): elements of dL/dW^c (x-pair records: value 0 at
  // the key, value 1 at the next element); wc_start is a multiple of
  // 2^MAX_BIN_SHIFT and the volume's x extent divides 2^12, so no pair
  // crosses a bin or a summing part
  uint32_t wc_start, wc_end;
};
struct ScatterPlan {
  uint32_t* cursor;          // records written by the adjoint
  uint32_t* vmax;            // [2] bounds on |value| of the table's and the blend weights' records
  uint32_t* keys;            // [cap]
  f2* vals;                  // [cap]
  uint32_t* skeys;           // [cap] records in bin order
  f2* svals;                 // [cap]
  uint32_t* hist;            // [n_tiles_cap][n_bins]
  uint32_t* seg;             // [BIN_SEGS][n_bins]
  uint32_t* total;           // [n_bins]
  uint32_t* base;            // [n_bins]
  uint32_t* item_base;       // [n_bins] first summing item of each bin
  uint32_t* item_bin;        // [max_items] bin of each summing item
  uint32_t* n_items;         // summing items of this launch
  uint32_t cap;
  int shift, n_bins, n_tiles_cap, max_items;
  int64_t n_keys;            // keys of all keyed levels
  KeyMap map;
  bool dense;                // the dense levels are keyed too
  bool wc;                   // so is dL/dW^c
};
int scatter_bin_shift(int64_t n_keys);
hipError_t launch_binned_scatter(const ScatterPlan& p, float* grad_table, float* grad_weights, hipStream_t st);

hipError_t launch_mse(const float* rgba, const float* target, int n, float* grad, float* loss, hipStream_t st);
hipError_t launch_softmax_fwd(const float* logits, float* w, int C, int64_t V, hipStream_t st);
hipError_t launch_softmax_bwd(const float* w, const float* g, float* gl, int C, int64_t V, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int step, void* lowp, mnr_dtype dt, hipStream_t st);
hipError_t launch_convert(const float* src, void* dst, mnr_dtype dt, int64_t n, hipStream_t st);
// Softmax adjoint, Adam on the logits and softmax of the new logits, in one pass.
hipError_t launch_motion_step(float* logits, float* w, const float* g, float* gl, float* m, float* v, int C,
                              int64_t V, float lr, float b1, float b2, float eps, int step, hipStream_t st);
hipError_t launch_zero(void* dst, size_t bytes, hipStream_t st);
// Spatially coherent processing order of a ray list (order[slot] = row).
hipError_t launch_ray_order(const int32_t* pixel_ids, int n, int H, int W, int32_t* order, hipStream_t st);
// Several fills, or Adam on several tensors (same hyper-parameters, BF16 or
// F16 copies or none), in one launch each: the training step's small
// tensors would otherwise cost a launch apiece.
constexpr int MAX_LIST = 24;
struct ZeroList {
  void* p[MAX_LIST];
  int64_t bytes[MAX_LIST];
  int n;
};
hipError_t launch_zero_list(const ZeroList& z, hipStream_t st);
struct AdamList {
  float* p[MAX_LIST];
  const float* g[MAX_LIST];
  float* m[MAX_LIST];
  float* v[MAX_LIST];
  void* low[MAX_LIST];  // the low-precision copy (NULL: none)
  int64_t n[MAX_LIST];
  int count;
};
hipError_t launch_adam_list(const AdamList& l, float lr, float b1, float b2, float eps, int step, mnr_dtype low_dt,
                            hipStream_t st);
// Packed copy of the bone channels of a blend-weight volume (2x2 x-y corners
// per float4; layout in mnr_motion_packed_bytes' declaration).
hipError_t launch_pack_motion(const float* w, f4* packed, int n_bones, int R, hipStream_t st);
// Packed copy of the dense grid levels (2x2 x-y corner groups; layout in
// mnr_field_packed_bytes' declaration).  f.dpk and f.dpk_off must be set.
hipError_t launch_pack_dense(const FieldArgs& f, mnr_dtype table_dt, hipStream_t st);

}  // namespace mnr
