// Server tick kernel: persistent blocks pull (request slot, tile) items
// from a device-side table and render each 16x16 tile with the same
// ray-block code as a full-frame mnr_render (each wave a quadrant: four
// blocks of 16 rays x 4 samples; splitting the tile's 32 blocks of 8 x 8
// between the waves through an LDS counter measured no better, since
// consecutive ticks already overlap).  MLP weights are restaged into LDS
// only when consecutive tiles of a block belong to different users (with
// the residual motion network, to different requests: the request's pose
// enters that network as a bias staged with its weights).
#include "field_device.h"
#include "kernels.h"

namespace mnr {

template <typename TableT, int P, int NHH, bool RES, bool FREQ>
__global__ void __launch_bounds__(BLOCK) serve_kernel(const RenderArgs* __restrict__ slots, WorkTable* __restrict__ wt) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  __shared__ int s_item;
  char* wl = lds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  char* feat = lds + weight_lds_bytes<P, NHH, RES, FREQ>() + wave * feat_bytes<P, FREQ>();
  const void* staged = nullptr;  // first-layer weight pointer of the staged user
  int staged_slot = -1;          // with the residual network: the staged request (its pose enters as a bias)
  const int n_items = wt->n_items;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&wt->counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();  // s_item is rewritten only after every wave has read it
    if (it >= n_items) break;
    const WorkItem w = wt->items[it];
    const RenderArgs& a = slots[w.slot];
    if (a.f.w[0] != staged || (RES && w.slot != staged_slot)) {  // block-uniform
      stage_all<P, NHH, RES, FREQ>(wl, a);
      staged = a.f.w[0];
      staged_slot = w.slot;
      __syncthreads();
    }
    render_tile_packet<TableT, P, NHH, RES, FREQ>(a, w.tile, wave, lane, wl, feat);
  }
}

// slots == nullptr: only query occupancy and set the LDS limit (done once,
// outside any graph capture).
template <typename TableT, int P, int NHH, bool RES, bool FREQ>
static hipError_t launch_serve_t(const RenderArgs* slots, WorkTable* wt, hipStream_t st) {
  constexpr int lds = weight_lds_bytes<P, NHH, RES, FREQ>() + WAVES_PER_BLOCK * feat_bytes<P, FREQ>();
  static_assert(lds <= 160 * 1024, "LDS of the tick kernel");
  auto kern = serve_kernel<TableT, P, NHH, RES, FREQ>;
  static PersistentGrid pg;
  const int max_blocks = persistent_blocks(kern, BLOCK, lds, pg);
  if (!slots) return hipGetLastError();
  hipLaunchKernelGGL(kern, dim3(max_blocks), dim3(BLOCK), lds, st, slots, wt);
  return hipGetLastError();
}

template <int P, int NHH, bool RES>
static hipError_t launch_serve_p(const RenderArgs* slots, WorkTable* wt, mnr_dtype tdt, hipStream_t st) {
  if (tdt == MNR_F16) return launch_serve_t<_Float16, P, NHH, RES, false>(slots, wt, st);
  return launch_serve_t<float, P, NHH, RES, false>(slots, wt, st);
}

template <bool RES>
static hipError_t launch_serve_bf16(const RenderArgs* slots, WorkTable* wt, mnr_dtype tdt, int nhh, hipStream_t st) {
  switch (nhh) {
    case 0: return launch_serve_p<MNR_BF16, 0, RES>(slots, wt, tdt, st);
    case 1: return launch_serve_p<MNR_BF16, 1, RES>(slots, wt, tdt, st);
    default: return launch_serve_p<MNR_BF16, 2, RES>(slots, wt, tdt, st);
  }
}

// Every user of a server shares one field format; the residual motion
// network and the frequency-encoded field run on the BF16 path only.
hipError_t launch_serve(const RenderArgs* slots, WorkTable* wt, mnr_dtype table_dt, mnr_dtype mlp_dt, int nhh,
                        bool res, bool freq, hipStream_t st) {
  if (freq)
    return res ? launch_serve_t<float, MNR_BF16, 0, true, true>(slots, wt, st)
               : launch_serve_t<float, MNR_BF16, 0, false, true>(slots, wt, st);
  if (mlp_dt == MNR_BF16)
    return res ? launch_serve_bf16<true>(slots, wt, table_dt, nhh, st)
               : launch_serve_bf16<false>(slots, wt, table_dt, nhh, st);
  switch (nhh) {
    case 0: return launch_serve_p<MNR_F32, 0, false>(slots, wt, table_dt, st);
    case 1: return launch_serve_p<MNR_F32, 1, false>(slots, wt, table_dt, st);
    default: return launch_serve_p<MNR_F32, 2, false>(slots, wt, table_dt, st);
  }
}

}  // namespace mnr
