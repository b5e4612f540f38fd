// Hand-written adjoint of the fused renderer (training, Sec. 5.2).
//
// One wavefront per ray, walking the chunks the forward pass processed from
// last to first.  Nothing per-sample is stored by the forward pass: each
// chunk is recomputed (sample, inverse LBS, encoding, MLP) and then
//   1. compositing adjoint (Eq. 3 with alpha' = alpha * min(L, 1),
//      composite_adjoint): dL/d(outputs) and dL/dL from the saved
//      chunk-start transmittance, S after the last processed sample being
//      the background colour (opacity 0);
//   2. MLP adjoint on MFMA, 16 samples at a time: activations recomputed
//      with the forward weights, dX = W^T dY with transposed weight
//      fragments, dW = dY X^T accumulated on the MFMAs in the wave's
//      registers and added to the block's LDS sums at the end;
//   3. encoding adjoint: scatter-add into the table gradient and the
//      encoding's spatial derivative back to the skinned point x_skel;
//      consecutive samples in the same cell are summed in the wave first
//      (with a record sink only at the dense levels, whose runs are long),
//      and with a record sink the levels write (key, gradient) records
//      instead of atomics, summed afterwards without float atomics
//      (scatter.hip);
//   4. skinning adjoint (Eq. 7, 9): dx_skel/dw_i = (y_i - x_skel)/L and the
//      likelihood term dalpha'/dL = alpha [L < 1], scattered through the
//      trilinear weights into dL/dW^c (records of x-adjacent corner pairs
//      with a record sink); optionally dL/dG_i through the points
//      y_i = G_i x and the weights' spatial gradient.
#include "adjoint_device.h"
#include "kernels.h"

namespace mnr {

template <int P>
struct BwdShape {
  using S = MlpShape<P>;
  using TB = typename std::conditional<P == MNR_F32, float, __bf16>::type;  // transpose buffer element
  static constexpr int KT_OUTT = (P == MNR_F32) ? 1 : 2;  // padded K tiles of the transposed output layer
  static constexpr int KG64 = (P == MNR_F32) ? 4 : 2;     // k-groups of a 64-wide K
  static constexpr int bytes_first_t() { return 2 * KG64 * S::FRAG; }
  static constexpr int bytes_hidden_t() { return 4 * KG64 * S::FRAG; }
  static constexpr int bytes_out_t() { return 4 * 1 * S::FRAG; }
  static constexpr int bytes_t(int nhh) { return bytes_first_t() + nhh * bytes_hidden_t() + bytes_out_t(); }
  // Block sums of dW in LDS, rows padded by 4 floats: the lanes of one
  // atomic (rows 4g + j, columns c of a 16 x 16 tile) then hit distinct
  // banks instead of four lanes per bank.
  static constexpr int LD_FIRST = IN_FEAT + 4, LD_HID = HIDDEN + 4;
  static constexpr int off_hidden(int l) { return HIDDEN * LD_FIRST + l * HIDDEN * LD_HID; }
  static constexpr int dw_floats(int nhh) { return off_hidden(nhh) + 4 * LD_HID; }
  static constexpr int tbuf_bytes() { return 2 * 64 * 16 * (int)sizeof(TB); }
  static constexpr int wave_bytes() { return S::feat_bytes_per_wave() + 64 * IN_FEAT * 4 + tbuf_bytes(); }
  static constexpr int dg_floats() { return MNR_MAX_BONES * 12; }  // block sums of dL/dG
  // The block's dW sums are needed only after the main loop, when the
  // weights are dead: they overlay the weights' LDS.
  static constexpr int lds_bytes(int nhh, int nw) {
    return S::bytes_total(nhh) + bytes_t(nhh) + dg_floats() * 4 + nw * wave_bytes();
  }
  static_assert(dw_floats(2) * 4 <= S::bytes_total(2) + bytes_t(2), "the dW sums fit over the weights");
};

// Stage W^T of a layer W [M][K] as the A operand of an (K x Mpad) product.
template <int P, typename WT>
__device__ void stage_layer_t(char* lds, const WT* __restrict__ w, int M, int K, int Kpad) {
  const int kg = (P == MNR_F32) ? Kpad / 16 : Kpad / 32;
  for (int e = threadIdx.x; e < K * Kpad; e += blockDim.x) {
    const int m = e / Kpad, k = e - m * Kpad;  // element (m, k) of W^T = W[k][m]
    const float v = (k < M) ? (float)w[(size_t)k * K + m] : 0.0f;
    if (P == MNR_F32)
      *(float*)(lds + frag_offset<P>(m, k, kg)) = v;
    else
      *(__bf16*)(lds + frag_offset<P>(m, k, kg)) = (__bf16)v;
  }
}

template <int P, int NHH>
__device__ void stage_weights_t(char* lds, const FieldArgs& f) {
  typedef typename std::conditional<P == MNR_F32, float, __bf16>::type WT;
  using B = BwdShape<P>;
  stage_layer_t<P>(lds, (const WT*)f.w[0], HIDDEN, IN_FEAT, HIDDEN);
  for (int l = 0; l < NHH; ++l)
    stage_layer_t<P>(lds + B::bytes_first_t() + l * B::bytes_hidden_t(), (const WT*)f.w[1 + l], HIDDEN, HIDDEN,
                     HIDDEN);
  stage_layer_t<P>(lds + B::bytes_first_t() + NHH * B::bytes_hidden_t(), (const WT*)f.w[1 + NHH], 4, HIDDEN,
                   (P == MNR_F32) ? 16 : 32);
}

__device__ __forceinline__ f4 relu_mask(f4 d, f4 h) {
  return f4{h[0] > 0.f ? d[0] : 0.f, h[1] > 0.f ? d[1] : 0.f, h[2] > 0.f ? d[2] : 0.f, h[3] > 0.f ? d[3] : 0.f};
}

// A wave's running sums of dW in registers, D layout: tile (mt, kt),
// element j of lane c + 16 g is dW[16 mt + 4 g + j][16 kt + c].  They
// accumulate on the MFMAs across every tile the wave processes and reach
// the block's LDS sums once, at the end: float atomics on LDS cost more
// than the products themselves.
template <int P, int NHH>
struct DwAcc {
  f4 out[1][4];        // output layer, 4 x 64
  f4 hid[NHH][4][4];   // hidden layers, 64 x 64
  f4 first[4][2];      // first layer, 64 x 32
};

// acc += dY (MT tiles, D layout) x X^T (NT tiles, D layout) over the 16
// samples of one tile, both operands transposed through the wave's buffer.
template <int P, int MT, int NT>
__device__ __forceinline__ void accumulate_dw(typename BwdShape<P>::TB* tb, const f4 (&d)[4], const f4 (&h)[4],
                                              f4 (&acc)[MT][NT], int lane) {
  using TB = typename BwdShape<P>::TB;
  TB* td = tb;            // [64 neurons][16 samples]
  TB* th = tb + 64 * 16;  // [64 neurons][16 samples]
  const int c = lane & 15, g = lane >> 4;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) td[(16 * t + 4 * g + j) * 16 + c] = (TB)d[t][j];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) th[(16 * t + 4 * g + j) * 16 + c] = (TB)h[t][j];
  wave_sync_lds();
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) {
      f4 a = acc[mt][kt];
      if constexpr (P == MNR_F32) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
          a = __builtin_amdgcn_mfma_f32_16x16x4f32(td[(16 * mt + c) * 16 + 4 * s + g],
                                                   th[(16 * kt + c) * 16 + 4 * s + g], a, 0, 0, 0);
      } else {
        bf16x8 av, bv;
        if (g < 2) {
          av = *(const bf16x8*)(td + (16 * mt + c) * 16 + 8 * g);
          bv = *(const bf16x8*)(th + (16 * kt + c) * 16 + 8 * g);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) av[e] = bv[e] = (__bf16)0.0f;
        }
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, a, 0, 0, 0);
      }
      acc[mt][kt] = a;
    }
  }
  wave_sync_lds();
}

// Add a wave's register sums (MT x NT tiles, rows < M_out) into the
// block's LDS sums (row stride ld), with plain read-add-write: the caller
// lets one wave at a time do it.
template <int MT, int NT>
__device__ __forceinline__ void flush_dw(const f4 (&acc)[MT][NT], float* dw, int M_out, int ld, int lane) {
  const int c = lane & 15, g = lane >> 4;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int kt = 0; kt < NT; ++kt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 16 * mt + 4 * g + j;
        if (row < M_out) dw[row * ld + 16 * kt + c] += acc[mt][kt][j];
      }
}

// MLP adjoint for sample tile nt.  dout: output-layer gradient in D layout
// (lanes 0..15 hold d/do of sample 16nt + lane).  Adds the tile's dW to the
// wave's register sums and writes d/dfeature of the 16 samples into
// dfeat[sample][32].
template <int P, int NHH>
__device__ __forceinline__ void mlp_tile_backward(const char* wl, const char* wt, const char* feat, int nt, int lane,
                                                  f4 dout, typename BwdShape<P>::TB* tb, DwAcc<P, NHH>& acc,
                                                  float* dfeat) {
  using S = MlpShape<P>;
  using B = BwdShape<P>;
  f4 x[4], hid[NHH + 1][4], tmp[4];
  load_input<P>(feat, nt, lane, x);
  mma_layer<P, 4, 2>(wl, x, tmp, lane);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) hid[0][mt] = relu4(tmp[mt]);
#pragma unroll
  for (int l = 0; l < NHH; ++l) {
    mma_layer<P, 4, 4>(wl + S::bytes_first() + l * S::bytes_hidden(), hid[l], tmp, lane);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) hid[l + 1][mt] = relu4(tmp[mt]);
  }
  const f4 z = {0.f, 0.f, 0.f, 0.f};
  f4 d[4] = {dout, z, z, z};
  // output layer
  accumulate_dw<P, 1, 4>(tb, d, hid[NHH], acc.out, lane);
  mma_layer<P, 4, B::KT_OUTT>(wt + B::bytes_first_t() + NHH * B::bytes_hidden_t(), d, tmp, lane);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) d[mt] = relu_mask(tmp[mt], hid[NHH][mt]);
  // hidden layers, last to first
#pragma unroll
  for (int l = NHH - 1; l >= 0; --l) {
    accumulate_dw<P, 4, 4>(tb, d, hid[l], acc.hid[l], lane);
    mma_layer<P, 4, 4>(wt + B::bytes_first_t() + l * B::bytes_hidden_t(), d, tmp, lane);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) d[mt] = relu_mask(tmp[mt], hid[l][mt]);
  }
  // first layer
  accumulate_dw<P, 4, 2>(tb, d, x, acc.first, lane);
  mma_layer<P, 2, 4>(wt, d, tmp, lane);
  const int c = lane & 15, g = lane >> 4;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int j = 0; j < 4; ++j) dfeat[(16 * nt + c) * IN_FEAT + 16 * mt + 4 * g + j] = tmp[mt][j];
}

// Ray slot mapping shared with the forward kernel (16x16 tiles dealt to XCDs).
template <int NW>
__device__ __forceinline__ int bwd_ray_slot(int blk, int nblk, int w, int it, int n_slots) {
  const int xcd = blk & 7, lb = blk >> 3;
  const int nb = (nblk - xcd + 7) >> 3;
  const int k = (it * nb + lb) * NW + w;
  const int slot = ((k >> 8) * 8 + xcd) * 256 + (k & 255);
  return slot < n_slots ? slot : -1;
}

// SPLIT (the residual motion network is on): the sample's query point
// x_final and its weight sum come from the split scratch, written by
// res_fwd_kernel, and instead of the skinning adjoint the kernel stores
// dL/dx_final and dL/dL there for res_bwd_kernel and skin_bwd_kernel.
template <typename TableT, int P, int NHH, int NW, bool SPLIT = false>
__global__ void __launch_bounds__(64 * NW) render_bwd_kernel(const RenderArgs a, int n_slots) {
  using S = MlpShape<P>;
  using B = BwdShape<P>;
  using TB = typename B::TB;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  char* wl = lds;
  char* wt = wl + S::bytes_total(NHH);
  static_assert(B::dw_floats(NHH) * 4 <= S::bytes_total(NHH) + B::bytes_t(NHH), "the dW sums fit over the weights");
  float* dw = (float*)lds;  // after the main loop only: over the weights
  float* dg = (float*)(wt + B::bytes_t(NHH));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  char* wbase = (char*)(dg + B::dg_floats()) + wave * B::wave_bytes();
  char* feat = wbase;
  float* dfeat = (float*)(wbase + S::feat_bytes_per_wave());
  TB* tb = (TB*)(wbase + S::feat_bytes_per_wave() + 64 * IN_FEAT * 4);

  stage_weights<P, NHH>(wl, a.f);
  stage_weights_t<P, NHH>(wt, a.f);
  for (int i = threadIdx.x; i < B::dg_floats(); i += blockDim.x) dg[i] = 0.f;
  __syncthreads();

  const size_t T = (size_t)1 << a.f.log2_T;
  const uint32_t tmask = (uint32_t)T - 1u;
  const int S_ = a.r.spp;
  const int nchunks = (S_ + 63) >> 6;
  const int R = a.m.res;
  const size_t plane = (size_t)R * R * R;
  const int tiles = (n_slots + 255) >> 8;
  const int nb_min = (gridDim.x >> 3) > 0 ? (gridDim.x >> 3) : 1;
  const int iters = (((tiles + 7) >> 3) * 256 + nb_min * NW - 1) / (nb_min * NW);

  DwAcc<P, NHH> acc;
  {
    const f4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) acc.out[0][kt] = z;
#pragma unroll
    for (int l = 0; l < NHH; ++l)
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) acc.hid[l][mt][kt] = z;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) acc.first[mt][kt] = z;
  }
  int q = blockIdx.x & 7, tried = 0;
  uint32_t tab_mb = 0u, wc_mb = 0u;  // largest |value| of the lane's table / blend-weight records (float bits)
  for (int it = 0;; ++it) {
    int slot;
    if (a.queues) {  // dynamic: pull rays from per-XCD queues
      slot = pull_unit(a.queues, n_slots, q, tried);
      if (slot < 0) break;
    } else {
      if (it >= iters) break;
      slot = bwd_ray_slot<NW>(blockIdx.x, gridDim.x, wave, it, n_slots);
      if (slot < 0) continue;
    }
    const int row = ray_row(a.r, slot);
    const int pix = ray_pixel(a.r, row);
    if (!a.r.pixel_ids && pix < 0) continue;
    const int orow = a.r.pixel_ids ? row : pix;
    RaySetup rs;
    if (!(pix >= 0 && pix < a.r.H * a.r.W && setup_ray(a.r, pix, rs))) continue;
    const f4 gout = *(const f4*)(a.grad_rgba + (size_t)orow * 4);
    float Sc[4] = {a.r.bg[0], a.r.bg[1], a.r.bg[2], 0.f};  // S after the last processed sample
    const float* tc = a.t_chunks + (size_t)orow * (nchunks + 1);
    const int n_done = (int)tc[nchunks];  // samples the forward pass processed
    for (int ch = nchunks - 1; ch >= 0; --ch) {
      const float T0 = tc[ch];
      if (T0 < 0.f || ch * 64 >= n_done) continue;  // not reached by the forward pass
      SampleState st;
      f4 out;
      const int i = ch * 64 + lane;
      const int64_t sj = ((int64_t)orow * nchunks + ch) * 64 + lane;  // split scratch slot
      uint64_t live_mask;
      if constexpr (SPLIT) {
        const float* sb = a.split.buf;
        const int64_t ss = a.split.stride;
        st.xs[0] = sb[SPLIT_XF * ss + sj];
        st.xs[1] = sb[(SPLIT_XF + 1) * ss + sj];
        st.xs[2] = sb[(SPLIT_XF + 2) * ss + sj];
        st.L = i < n_done ? sb[SPLIT_L * ss + sj] : 0.f;
        live_mask = field_eval<TableT, P, NHH, false, false, true>(a, i < n_done, lane, wl, feat, (f4*)dfeat, st, out);
      } else {
        const float s = ((float)i + sample_jitter(a.r, orow, i)) * rs.delta;
        st.x[0] = fmaf(s, rs.d[0], rs.p0[0]);
        st.x[1] = fmaf(s, rs.d[1], rs.p0[1]);
        st.x[2] = fmaf(s, rs.d[2], rs.p0[2]);
        live_mask = field_eval<TableT, P, NHH>(a, i < n_done, lane, wl, feat, (f4*)dfeat, st, out);
      }
      if (live_mask == 0) continue;  // alpha' = 0 everywhere: S passes through unchanged

      // ---- 1. compositing adjoint -------------------------------------------------
      float g_o[4], g_L;
      composite_adjoint(T0, rs.delta, out, st.L, st.live, gout, Sc, g_o, g_L);

      // ---- 2. MLP adjoint -----------------------------------------------------------
      f4* gobuf = (f4*)dfeat;
      gobuf[lane] = f4{g_o[0], g_o[1], g_o[2], g_o[3]};
      wave_sync_lds();
      f4 dout[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) dout[nt] = (lane < 16) ? gobuf[nt * 16 + lane] : f4{0.f, 0.f, 0.f, 0.f};
      wave_sync_lds();
#pragma unroll 1
      for (int nt = 0; nt < 4; ++nt) mlp_tile_backward<P, NHH>(wl, wt, feat, nt, lane, dout[nt], tb, acc, dfeat);
      wave_sync_lds();

      // ---- 3. encoding adjoint ------------------------------------------------------
      // All lanes take part (the run detection shuffles across the wave);
      // lanes that are not live contribute zeros and issue nothing.
      const bool live = st.live;
      float u[3], g_u[3] = {0.f, 0.f, 0.f};
      unit_coords(a.f, st.xs, u);
#pragma unroll
      for (int q = 0; q < 3; ++q) u[q] = live ? u[q] : 0.f;
      const float* df = dfeat + lane * IN_FEAT;
      // With a record sink, the table gradient leaves as records (binned
      // and summed after this kernel) instead of global atomics: one
      // reservation per chunk, then for hashed level h and corner k the live
      // lanes write records base + (8 h + k) n_live + rank; a dense level
      // (when keyed) writes one record per corner and run of consecutive
      // samples in one cell, after the hashed levels' records.  Keys: h T +
      // row for hashed level h, then the dense levels' rows one level after
      // the other ((N+1)^3 keys each).  The blend-weight records (when
      // keyed) take the rest of the reservation.  A reservation past the
      // capacity falls back to global atomics.
      uint32_t rec_base = 0, rec_end = 0, n_live = 0, rank = 0, n_hashed = 0;
      bool rec_ok = false;
      WcRecords wcr{false, 0u, 0u};
      if (a.rec.keys) {
        const uint64_t lm = __ballot(live);
        n_live = (uint32_t)__popcll(lm);
        rank = (uint32_t)__popcll(lm & ((1ull << lane) - 1ull));
        n_hashed = (uint32_t)__popc(~a.f.dense_mask & ((1u << a.f.n_levels) - 1u));
        uint32_t n_runs = 0;  // runs over the dense levels
        if (a.rec.dense) {
#pragma unroll 1
          for (int l = 0; l < a.f.n_levels; ++l) {
            if (!((a.f.dense_mask >> l) & 1u)) continue;
            const GridCell gc = grid_cell(u, a.f.level_res[l]);
            const CellRuns cr = cell_runs(live, gc.i0[0], gc.i0[1], gc.i0[2]);
            n_runs += (uint32_t)__popcll(__ballot(live && cr.owner));
          }
        }
        const uint32_t n_tab = (n_live * n_hashed + n_runs) * 8u;
        uint32_t n_wc = 0;
        if constexpr (!SPLIT) {
          if (a.rec.wc) n_wc = wc_record_count(a, st.x, live);
        }
        const uint32_t cnt = n_tab + n_wc;
        uint32_t b = 0;
        if (lane == 0 && cnt) b = atomicAdd(a.rec.cursor, cnt);
        rec_base = __builtin_amdgcn_readfirstlane(b);
        rec_end = rec_base + cnt;
        rec_ok = (uint64_t)rec_base + cnt <= (uint64_t)a.rec.cap;
        wcr = WcRecords{rec_ok && n_wc > 0, rec_base + n_tab, rec_end};
      }
      // (a) spatial derivative of the encoding: table reads only.  (b) then
      // the gradient scatter, which reads nothing: on this GPU one counter
      // covers loads and stores, so stores issued between loads would hold
      // up every later wait on a load.
      if (live) {
#pragma unroll 1
        for (int l = 0; l < a.f.n_levels; ++l) {
          const int N = a.f.level_res[l];
          const bool dense = (a.f.dense_mask >> l) & 1u;
          const GridCell gc = grid_cell(u, N);
          const float d0 = df[2 * l], d1 = df[2 * l + 1];
          const __amdgpu_buffer_rsrc_t lrs = level_rsrc<TableT>(a.f, l);
          float gp[3] = {0.f, 0.f, 0.f};
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const f2 v = load_row<TableT>(lrs, grid_row(gc, N, dense, tmask, k));
            const float wx = (k & 1) ? gc.f[0] : 1.f - gc.f[0];
            const float wy = (k & 2) ? gc.f[1] : 1.f - gc.f[1];
            const float wz = (k & 4) ? gc.f[2] : 1.f - gc.f[2];
            const float dot = d0 * v[0] + d1 * v[1];
            gp[0] += dot * ((k & 1) ? 1.f : -1.f) * wy * wz;
            gp[1] += dot * ((k & 2) ? 1.f : -1.f) * wx * wz;
            gp[2] += dot * ((k & 4) ? 1.f : -1.f) * wx * wy;
          }
#pragma unroll
          for (int q = 0; q < 3; ++q) g_u[q] = fmaf(gp[q], (float)N, g_u[q]);
        }
      }
      uint32_t dense_off = 0;                       // runs of the dense levels written so far
      uint32_t dense_key = n_hashed << a.f.log2_T;  // first key of the next dense level
#pragma unroll 1
      for (int l = 0; l < a.f.n_levels; ++l) {
        const int N = a.f.level_res[l];
        const bool dense = (a.f.dense_mask >> l) & 1u;
        const GridCell gc = grid_cell(u, N);
        const float d0 = live ? df[2 * l] : 0.f, d1 = live ? df[2 * l + 1] : 0.f;
        float wk[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          wk[k] = ((k & 1) ? gc.f[0] : 1.f - gc.f[0]) * ((k & 2) ? gc.f[1] : 1.f - gc.f[1]) *
                  ((k & 4) ? gc.f[2] : 1.f - gc.f[2]);
        if (rec_ok && !dense) {  // hashed level: records
          if (live) {
            // |wk d| <= max|wk| max|d| (rounding is monotone); maxima taken on
            // the bits, so that NaN and infinity carry through
            uint32_t wb = 0u;
#pragma unroll
            for (int k = 0; k < 8; ++k) wb = max(wb, __float_as_uint(fabsf(wk[k])));
            const float dmax = __uint_as_float(max(__float_as_uint(fabsf(d0)), __float_as_uint(fabsf(d1))));
            tab_mb = max(tab_mb, __float_as_uint(fabsf(dmax * __uint_as_float(wb))));
            const uint32_t h = (uint32_t)__popc(~a.f.dense_mask & ((1u << l) - 1u));
            const uint32_t key0 = h << a.f.log2_T;  // the hashed levels take the first keys
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const uint32_t idx = rec_base + (h * 8u + (uint32_t)k) * n_live + rank;
              a.rec.keys[idx] = key0 + grid_row(gc, N, dense, tmask, k);
              a.rec.vals[idx] = f2{wk[k] * d0, wk[k] * d1};
            }
          }
          continue;
        }
        // Table gradient: one atomic per corner and feature per run of
        // consecutive samples in the same cell, carrying the run's sum.
        float v[16];
#pragma unroll
        for (int k = 0; k < 8; ++k) { v[2 * k] = wk[k] * d0; v[2 * k + 1] = wk[k] * d1; }
        const CellRuns cr = cell_runs(live, gc.i0[0], gc.i0[1], gc.i0[2]);
        run_sums<16>(cr, v);
        if (rec_ok && a.rec.dense) {  // dense level: one record per corner and run
          const uint64_t hm = __ballot(live && cr.owner);
          const uint32_t n_runs = (uint32_t)__popcll(hm);
          if (live && cr.owner) {
            const uint32_t r = (uint32_t)__popcll(hm & ((1ull << lane) - 1ull));
            const uint32_t first = rec_base + n_live * n_hashed * 8u + dense_off * 8u;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const uint32_t idx = first + (uint32_t)k * n_runs + r;
              if (idx < rec_end) {  // (the counting pass found the same runs)
                a.rec.keys[idx] = dense_key + grid_row(gc, N, dense, tmask, k);
                a.rec.vals[idx] = f2{v[2 * k], v[2 * k + 1]};
              }
              tab_mb = max(tab_mb, max(__float_as_uint(fabsf(v[2 * k])), __float_as_uint(fabsf(v[2 * k + 1]))));
            }
          }
          dense_off += n_runs;
          dense_key += (uint32_t)(N + 1) * (uint32_t)(N + 1) * (uint32_t)(N + 1);
          continue;
        }
        if (live && cr.owner) {
          float* gt = a.grad_table + (size_t)l * T * 2;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const uint32_t row = grid_row(gc, N, dense, tmask, k);
            unsafeAtomicAdd(gt + 2 * (size_t)row, v[2 * k]);
            unsafeAtomicAdd(gt + 2 * (size_t)row + 1, v[2 * k + 1]);
          }
        }
      }
      float g_xs[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float ur = (st.xs[q] - a.f.gmin[q]) * a.f.gscale[q];
        g_xs[q] = (live && ur > 0.f && ur < 1.f) ? g_u[q] * a.f.gscale[q] : 0.f;
      }

      // ---- 4. skinning adjoint ------------------------------------------------------
      if constexpr (SPLIT) {  // hand dL/dx_final and dL/dL to the residual network's adjoint
        float* sb = a.split.buf;
        const int64_t ss = a.split.stride;
        if (i < n_done) {
          sb[SPLIT_G * ss + sj] = g_xs[0];
          sb[(SPLIT_G + 1) * ss + sj] = g_xs[1];
          sb[(SPLIT_G + 2) * ss + sj] = g_xs[2];
          sb[SPLIT_GL * ss + sj] = live ? g_L : 0.f;
        }
      } else {
        skin_adjoint(a, st.x, st.xs, st.L, g_xs, g_L, live, dg, wcr, wc_mb);
      }
      wave_sync_lds();
    }
  }
  if (a.rec.keys) flush_value_bounds(a.rec, tab_mb, wc_mb);
  // the weights are dead now: their LDS takes the block's dW sums, and the
  // waves' register sums go there one wave at a time
  __syncthreads();
  for (int i = threadIdx.x; i < B::dw_floats(NHH); i += blockDim.x) dw[i] = 0.f;
  __syncthreads();
  for (int w = 0; w < NW; ++w) {
    if (wave == w) {
      flush_dw(acc.out, dw + B::off_hidden(NHH), 4, B::LD_HID, lane);
#pragma unroll
      for (int l = 0; l < NHH; ++l) flush_dw(acc.hid[l], dw + B::off_hidden(l), HIDDEN, B::LD_HID, lane);
      flush_dw(acc.first, dw, HIDDEN, B::LD_FIRST, lane);
    }
    __syncthreads();
  }
  // flush the block's bone-transform gradients: every wave of every block
  // adds into the same few cache lines, so the sums stay in LDS until here
  if (a.grad_G)
    for (int i = threadIdx.x; i < a.m.n_bones * 12; i += blockDim.x)
      if (dg[i] != 0.f) unsafeAtomicAdd(a.grad_G + i, dg[i]);
  // flush the block's MLP weight gradients
  const int n_first = HIDDEN * IN_FEAT, n_hid = HIDDEN * HIDDEN;
  for (int i = threadIdx.x; i < n_first + NHH * n_hid + 4 * HIDDEN; i += blockDim.x) {
    float v;
    float* dst;
    if (i < n_first) {
      const int r = i / IN_FEAT;
      v = dw[r * B::LD_FIRST + (i - r * IN_FEAT)];
      dst = a.grad_w[0] + i;
    } else {
      const int e = i - n_first, l = e / n_hid, k = e - l * n_hid, r = k / HIDDEN;  // l == NHH: output layer
      v = dw[B::off_hidden(l) + r * B::LD_HID + (k - r * HIDDEN)];
      dst = a.grad_w[1 + l] + k;
    }
    if (v != 0.f) unsafeAtomicAdd(dst, v);
  }
}

static_assert(BwdShape<MNR_BF16>::lds_bytes(2, 4) <= 160 * 1024, "LDS of the BF16 adjoint");
static_assert(BwdShape<MNR_F32>::lds_bytes(2, 2) <= 160 * 1024, "LDS of the FP32 adjoint");

template <typename TableT, int P, int NHH, bool SPLIT>
static hipError_t launch_bwd_s(const RenderArgs& a, int n_slots, hipStream_t st) {
  constexpr int NW = (P == MNR_F32) ? 2 : 4;  // (one wave per SIMD at most: the BF16 kernel's registers)
  const int lds = BwdShape<P>::lds_bytes(NHH, NW);
  auto kern = render_bwd_kernel<TableT, P, NHH, NW, SPLIT>;
  static PersistentGrid pg;
  const int max_blocks = persistent_blocks(kern, 64 * NW, lds, pg);
  const int need = (n_slots + NW - 1) / NW;
  int grid = need < max_blocks ? need : max_blocks;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * NW), lds, st, a, n_slots);
  return hipGetLastError();
}

template <typename TableT, int P, int NHH>
static hipError_t launch_bwd_t(const RenderArgs& a, int n_slots, hipStream_t st) {
  if constexpr (P == MNR_BF16)  // the residual motion network (hence the split) is BF16 only
    if (a.split.buf) return launch_bwd_s<TableT, P, NHH, true>(a, n_slots, st);
  return launch_bwd_s<TableT, P, NHH, false>(a, n_slots, st);
}

template <int P, int NHH>
static hipError_t launch_bwd_p(const RenderArgs& a, int n_slots, mnr_dtype tdt, hipStream_t st) {
  if (tdt == MNR_F16) return launch_bwd_t<_Float16, P, NHH>(a, n_slots, st);
  return launch_bwd_t<float, P, NHH>(a, n_slots, st);
}

hipError_t launch_render_bwd(const RenderArgs& a, int n_slots, mnr_dtype table_dt, mnr_dtype mlp_dt, int nhh,
                             hipStream_t st) {
  if (mlp_dt == MNR_BF16) {
    switch (nhh) {
      case 0: return launch_bwd_p<MNR_BF16, 0>(a, n_slots, table_dt, st);
      case 1: return launch_bwd_p<MNR_BF16, 1>(a, n_slots, table_dt, st);
      default: return launch_bwd_p<MNR_BF16, 2>(a, n_slots, table_dt, st);
    }
  }
  switch (nhh) {
    case 0: return launch_bwd_p<MNR_F32, 0>(a, n_slots, table_dt, st);
    case 1: return launch_bwd_p<MNR_F32, 1>(a, n_slots, table_dt, st);
    default: return launch_bwd_p<MNR_F32, 2>(a, n_slots, table_dt, st);
  }
}

}  // namespace mnr
