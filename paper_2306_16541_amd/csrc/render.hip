// Fused forward renderers (Sec. 4, Fig. 2).
//
// render_fwd_kernel (ray lists, e.g. training batches): one wavefront owns
// one ray at a time and walks it in chunks of 64 samples, one per lane:
//   sample inside the body box (Sec. 4.4) -> inverse LBS (Eq. 7-9)
//   -> grid encoding -> MLP on MFMA (Eq. 13) -> front-to-back compositing
//   with the likelihood augmentation (Eq. 3, Sec. 4.4) as a wave
//   prefix-product; transmittance is carried across chunks and the ray stops
//   after the chunk where it falls below ert_tau.
// render_packet_kernel (full frames): one wavefront owns a small block of
// neighbouring pixels and marches its rays in lockstep, G consecutive
// samples of each ray per iteration (lane G r + k: sample j + k of ray r):
// 8 rays x 8 samples when pulling work from the queues, 16 rays x 4
// samples on the static path.  The 64 samples of an iteration lie within a
// few voxels of each other, so the skinning-volume and grid gathers of a
// wave share cache lines; the G lanes of a ray composite its G samples in
// order (a per-ray recurrence) and each ray stops as soon as its
// transmittance is below ert_tau.
// Both use a persistent grid: blocks stage the MLP weights into LDS once
// and loop over work.  With a workspace, waves pull work from per-XCD
// queues over contiguous bands of the frame (block b runs on XCD b % 8),
// so each XCD's L2 sees spatially coherent gathers; without one, 16x16
// tiles (or 256-ray groups) are dealt round-robin to the XCDs.
#include "field_device.h"
#include "kernels.h"

namespace mnr {

// Waves per block of the frame and ray-list kernels: the MLP weights in LDS
// are shared by the block, so bigger blocks leave more LDS per CU for the
// per-wave feature buffers.  Twelve waves (three per SIMD, what the kernels'
// registers allow) fit one block in the 160 KiB of LDS: FP32 44 + 12 x 8
// KiB, BF16 22 + 12 x 4 KiB (+ 34 KiB with the residual network), the
// frequency field 42 + 12 x 8 KiB.  The frequency field with the residual
// network needs 34 KiB more and takes eight.  The BF16 ray-list kernel
// (training batches of a few thousand rays) measured faster with eight.
// Samples per ray per step of the full-frame kernel's dynamic path: its
// ray blocks hold 64 / FRAME_G = 8 rays (4 x 2 pixels), 32 per 16x16 tile.
// Measured at 512x512x128 (FP32 / mixed): 5.63 / 3.40 ms with 4, 5.24 /
// 3.27 with 8, 5.29 / 3.71 with 16 samples per step.
constexpr int FRAME_G = 8;

template <int P, bool RES, bool FREQ, bool RAY_LIST>
constexpr int block_waves() { return ((RES && FREQ) || (RAY_LIST && P != MNR_F32)) ? 8 : 12; }

// Ray slot handled by iteration `it` of wave `w` of block `blk`.
template <int NW>
__device__ __forceinline__ int ray_slot(int blk, int nblk, int w, int it, int n_slots) {
  const int xcd = blk & 7, lb = blk >> 3;
  const int nb = (nblk - xcd + 7) >> 3;  // blocks on this XCD
  const int k = (it * nb + lb) * NW + w;  // k-th ray of this XCD
  const int slot = ((k >> 8) * 8 + xcd) * 256 + (k & 255);
  return slot < n_slots ? slot : -1;
}

template <int NW>
__device__ __forceinline__ int n_iters(int nblk, int n_slots) {
  // Enough iterations for the least-loaded XCD to cover its tiles.
  const int tiles = (n_slots + 255) >> 8;
  const int tiles_per_xcd = (tiles + 7) >> 3;
  const int nb_min = nblk >> 3 > 0 ? nblk >> 3 : 1;
  return (tiles_per_xcd * 256 + nb_min * NW - 1) / (nb_min * NW);
}


template <typename TableT, int P, int NHH, int NW, bool RES, bool FREQ = false>
__global__ void __launch_bounds__(64 * NW) render_fwd_kernel(const RenderArgs a, int n_slots) {
  using S = MlpShape<P>;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  char* wl = lds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  char* feat = lds + weight_lds_bytes<P, NHH, RES, FREQ>() + wave * feat_bytes<P, FREQ>();

  stage_all<P, NHH, RES, FREQ>(wl, a);
  __syncthreads();

  const int S_ = a.r.spp;
  const int nchunks = (S_ + 63) >> 6;
  const int iters = n_iters<NW>(gridDim.x, n_slots);

  int q = blockIdx.x & 7, tried = 0;
  for (int it = 0;; ++it) {
    int slot;
    if (a.queues) {  // dynamic: pull rays from per-XCD queues
      slot = pull_unit(a.queues, n_slots, q, tried);
      if (slot < 0) break;
    } else {
      if (it >= iters) break;
      slot = ray_slot<NW>(blockIdx.x, gridDim.x, wave, it, n_slots);
      if (slot < 0) continue;
    }
    const int row = ray_row(a.r, slot);
    const int pix = ray_pixel(a.r, row);
    if (!a.r.pixel_ids && pix < 0) continue;  // tile slot outside the image
    const int orow = a.r.pixel_ids ? row : pix;
    RaySetup rs;
    const bool hit = pix >= 0 && pix < a.r.H * a.r.W && setup_ray(a.r, pix, rs);
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, Tr = 1.f;
    unsigned live_count = 0;
    int done = 0;  // chunks processed
    if (hit) {
      for (int ch = 0; ch < nchunks; ++ch) {
        if (a.t_chunks && lane == 0) a.t_chunks[(size_t)orow * (nchunks + 1) + ch] = Tr;
        done = ch + 1;
        SampleState st;
        f4 out;
        const uint64_t live_mask =
            chunk_eval<TableT, P, NHH, RES, FREQ>(a, rs, orow, ch, lane, wl, feat, (f4*)feat, st, out);
        if (live_mask == 0) continue;  // nothing visible in this chunk (alpha' = 0)
        live_count += __popcll(live_mask);
        const bool live = st.live;
        const float L = st.L;

        // Composite: alpha = 1 - exp(-sigma delta), alpha' = alpha min(L, 1).
        const float sigma = fmaxf(out[3], 0.f);
        const float alpha = -expm1f(-sigma * rs.delta);
        const float ap = live ? alpha * fminf(L, 1.f) : 0.f;
        const float incl = wave_prefix_prod(1.f - ap);
        float excl = shfl_up(incl, 1);
        if (lane == 0) excl = 1.f;
        const float w = Tr * excl * ap;
        const float c0 = 1.f / (1.f + expf(-out[0]));
        const float c1 = 1.f / (1.f + expf(-out[1]));
        const float c2 = 1.f / (1.f + expf(-out[2]));
        C0 += wave_sum(w * c0);
        C1 += wave_sum(w * c1);
        C2 += wave_sum(w * c2);
        Tr *= __shfl(incl, 63, WAVE);
        if (Tr < a.r.ert_tau) break;
      }
    }
    if (a.t_chunks) {
      for (int ch = done + lane; ch < nchunks; ch += 64) a.t_chunks[(size_t)orow * (nchunks + 1) + ch] = -1.f;
      if (lane == 0) a.t_chunks[(size_t)orow * (nchunks + 1) + nchunks] = (float)min(done * 64, S_);
    }
    if (lane == 0) {
      f4 res = {C0 + Tr * a.r.bg[0], C1 + Tr * a.r.bg[1], C2 + Tr * a.r.bg[2], 1.f - Tr};
      *(f4*)(a.out + (size_t)orow * 4) = res;
      if (a.n_eval && live_count) atomicAdd(a.n_eval, (unsigned long long)live_count);
    }
  }
}


// With a workspace, waves pull 4x4 ray blocks (16 per tile) from per-XCD
// queues; without one, NW / 4 consecutive 16x16 tiles per block iteration
// (each wave a quadrant: four 4x4 blocks in turn), tile groups dealt
// round-robin to the XCDs.
template <typename TableT, int P, int NHH, int NW, bool RES, bool FREQ = false>
__global__ void __launch_bounds__(64 * NW) render_packet_kernel(const RenderArgs a, int n_tiles) {
  using S = MlpShape<P>;
  constexpr int TPB = NW / 4;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  char* wl = lds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  char* feat = lds + weight_lds_bytes<P, NHH, RES, FREQ>() + wave * feat_bytes<P, FREQ>();

  stage_all<P, NHH, RES, FREQ>(wl, a);
  __syncthreads();
  if (a.queues) {  // dynamic: each wave pulls ray blocks (4 G per tile) from per-XCD queues
    int q = blockIdx.x & 7, tried = 0;
    for (;;) {
      const int unit = pull_unit(a.queues, n_tiles * 4 * FRAME_G, q, tried);
      if (unit < 0) break;
      render_tile_rays<TableT, P, NHH, RES, FREQ, FRAME_G>(a, unit / (4 * FRAME_G), unit % (4 * FRAME_G), lane, wl,
                                                           feat);
    }
    return;
  }
  const int xcd = blockIdx.x & 7, lb = blockIdx.x >> 3;
  const int nb = ((int)gridDim.x - xcd + 7) >> 3;  // blocks on this XCD
  const int n_groups = (n_tiles + TPB - 1) / TPB;
  for (int k = lb;; k += nb) {
    const int group = k * 8 + xcd;
    if (group >= n_groups) break;
    const int tile = group * TPB + (wave >> 2);
    if (tile < n_tiles) render_tile_packet<TableT, P, NHH, RES, FREQ>(a, tile, wave & 3, lane, wl, feat);
  }
}

template <typename TableT, int P, int NHH, bool RES, bool FREQ = false>
static hipError_t launch_fwd_t(const RenderArgs& a, int n_slots, hipStream_t st) {
  constexpr int NW = block_waves<P, RES, FREQ, false>();
  static_assert(weight_lds_bytes<P, NHH, RES, FREQ>() + NW * feat_bytes<P, FREQ>() <= 160 * 1024, "LDS per block");
  if (!a.r.pixel_ids) {  // full frame: 4x4 ray blocks
    const int lds = weight_lds_bytes<P, NHH, RES, FREQ>() + NW * feat_bytes<P, FREQ>();
    auto kern = render_packet_kernel<TableT, P, NHH, NW, RES, FREQ>;
    static PersistentGrid pg;
    const int n_tiles = n_slots / 256;
    const int mb = persistent_blocks(kern, 64 * NW, lds, pg);
    const int groups = a.queues ? (n_tiles * 4 * FRAME_G + NW - 1) / NW : (n_tiles + NW / 4 - 1) / (NW / 4);
    const int grid = groups < mb ? groups : mb;
    hipLaunchKernelGGL(kern, dim3(grid > 0 ? grid : 1), dim3(64 * NW), lds, st, a, n_tiles);
    return hipGetLastError();
  }
  constexpr int NWR = block_waves<P, RES, FREQ, true>();
  const int lds = weight_lds_bytes<P, NHH, RES, FREQ>() + NWR * feat_bytes<P, FREQ>();
  auto kern = render_fwd_kernel<TableT, P, NHH, NWR, RES, FREQ>;
  static PersistentGrid pg;
  const int mb = persistent_blocks(kern, 64 * NWR, lds, pg);
  const int need = (n_slots + NWR - 1) / NWR;
  int grid = need < mb ? need : mb;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * NWR), lds, st, a, n_slots);
  return hipGetLastError();
}

template <int P, int NHH, bool RES>
static hipError_t launch_fwd_p(const RenderArgs& a, int n_slots, mnr_dtype tdt, hipStream_t st) {
  if (tdt == MNR_F16) return launch_fwd_t<_Float16, P, NHH, RES>(a, n_slots, st);
  return launch_fwd_t<float, P, NHH, RES>(a, n_slots, st);
}

template <bool RES>
static hipError_t launch_fwd_bf16(const RenderArgs& a, int n_slots, mnr_dtype table_dt, int nhh, hipStream_t st) {
  switch (nhh) {
    case 0: return launch_fwd_p<MNR_BF16, 0, RES>(a, n_slots, table_dt, st);
    case 1: return launch_fwd_p<MNR_BF16, 1, RES>(a, n_slots, table_dt, st);
    default: return launch_fwd_p<MNR_BF16, 2, RES>(a, n_slots, table_dt, st);
  }
}

// The residual motion network (a.res.w[0] != NULL) exists on the BF16 path
// only; the host rejects it for F32 MLPs before launching.
hipError_t launch_render_fwd(const RenderArgs& a, int n_slots, mnr_dtype table_dt, mnr_dtype mlp_dt,
                             int nhh, hipStream_t st) {
  if (a.f.freq)  // the frequency-encoded field: BF16 only, no grid table
    return a.res.w[0] ? launch_fwd_t<float, MNR_BF16, 0, true, true>(a, n_slots, st)
                      : launch_fwd_t<float, MNR_BF16, 0, false, true>(a, n_slots, st);
  if (mlp_dt == MNR_BF16)
    return a.res.w[0] ? launch_fwd_bf16<true>(a, n_slots, table_dt, nhh, st)
                      : launch_fwd_bf16<false>(a, n_slots, table_dt, nhh, st);
  switch (nhh) {
    case 0: return launch_fwd_p<MNR_F32, 0, false>(a, n_slots, table_dt, st);
    case 1: return launch_fwd_p<MNR_F32, 1, false>(a, n_slots, table_dt, st);
    default: return launch_fwd_p<MNR_F32, 2, false>(a, n_slots, table_dt, st);
  }
}

}  // namespace mnr
