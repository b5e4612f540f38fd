// Server tick kernel: persistent blocks pull (request slot, tile) items
// from a device-side table and render each 16x16 tile with the same
// ray-block code as a full-frame mnr_render (each wave a quadrant: four
// blocks of 16 rays x 4 samples; splitting the tile's 32 blocks of 8 x 8
// between the waves through an LDS counter measured no better, since
// consecutive ticks already overlap).  MLP weights are restaged into LDS only
// when consecutive tiles of a block belong to different users.
#include "field_device.h"
#include "kernels.h"

namespace mnr {

template <typename TableT, int P, int NHH>
__global__ void __launch_bounds__(BLOCK) serve_kernel(const RenderArgs* __restrict__ slots, WorkTable* __restrict__ wt) {
  using S = MlpShape<P>;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  __shared__ int s_item;
  char* wl = lds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  char* feat = lds + S::bytes_total(NHH) + wave * S::feat_bytes_per_wave();
  const void* staged = nullptr;  // first-layer weight pointer of the staged user
  const int n_items = wt->n_items;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&wt->counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();  // s_item is rewritten only after every wave has read it
    if (it >= n_items) break;
    const WorkItem w = wt->items[it];
    const RenderArgs& a = slots[w.slot];
    if (a.f.w[0] != staged) {  // block-uniform
      stage_weights<P, NHH>(wl, a.f);
      staged = a.f.w[0];
      __syncthreads();
    }
    render_tile_packet<TableT, P, NHH>(a, w.tile, wave, lane, wl, feat);
  }
}

// slots == nullptr: only query occupancy and set the LDS limit (done once,
// outside any graph capture).
template <typename TableT, int P, int NHH>
static hipError_t launch_serve_t(const RenderArgs* slots, WorkTable* wt, hipStream_t st) {
  using S = MlpShape<P>;
  const int lds = S::bytes_total(NHH) + WAVES_PER_BLOCK * S::feat_bytes_per_wave();
  auto kern = serve_kernel<TableT, P, NHH>;
  static PersistentGrid pg;
  const int max_blocks = persistent_blocks(kern, BLOCK, lds, pg);
  if (!slots) return hipGetLastError();
  hipLaunchKernelGGL(kern, dim3(max_blocks), dim3(BLOCK), lds, st, slots, wt);
  return hipGetLastError();
}

template <int P, int NHH>
static hipError_t launch_serve_p(const RenderArgs* slots, WorkTable* wt, mnr_dtype tdt, hipStream_t st) {
  if (tdt == MNR_F16) return launch_serve_t<_Float16, P, NHH>(slots, wt, st);
  return launch_serve_t<float, P, NHH>(slots, wt, st);
}

hipError_t launch_serve(const RenderArgs* slots, WorkTable* wt, mnr_dtype table_dt, mnr_dtype mlp_dt, int nhh,
                        hipStream_t st) {
  if (mlp_dt == MNR_BF16) {
    switch (nhh) {
      case 0: return launch_serve_p<MNR_BF16, 0>(slots, wt, table_dt, st);
      case 1: return launch_serve_p<MNR_BF16, 1>(slots, wt, table_dt, st);
      default: return launch_serve_p<MNR_BF16, 2>(slots, wt, table_dt, st);
    }
  }
  switch (nhh) {
    case 0: return launch_serve_p<MNR_F32, 0>(slots, wt, table_dt, st);
    case 1: return launch_serve_p<MNR_F32, 1>(slots, wt, table_dt, st);
    default: return launch_serve_p<MNR_F32, 2>(slots, wt, table_dt, st);
  }
}

}  // namespace mnr
