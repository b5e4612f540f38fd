// Adjoint of the paper's own canonical field (Sec. 4.4, Eq. 13, Fig. 9):
// c, sigma = MLP_nerf(gamma(x_final)) with the 10-band positional encoding
// gamma and the skip of gamma into layer 4 (training, Sec. 5.2).
//
// The forward weights (42 KiB BF16), their transposes (44 KiB) and FP32
// block sums of the weight gradients (81 KiB) do not fit one kernel's LDS,
// so the adjoint is split like the residual network's, handing per-sample
// values through the split scratch (SplitArgs):
//   freq_save_kernel  per ray, chunks last to first: the sample's query
//                     point (inverse LBS here, or x_final from the residual
//                     network's forward kernel), gamma, the skip MLP on
//                     MFMA with its four hidden activations saved (BF16, the
//                     values the next layer consumed), and the compositing
//                     adjoint, storing dL/d(outputs) and dL/dL;
//   freq_bwd_kernel   per 16-sample tile, the MLP's adjoint from the saved
//                     activations: dL/dW1..W5 (each wave summing its own
//                     rows in MFMA accumulators, block sums in LDS at the
//                     end) and
//                     dL/dx_final = (d gamma / dx)^T dL/dgamma, where
//                     dL/dgamma collects the first layer's and the skip's
//                     terms (gamma recomputed with its inputs in an order
//                     that gives each lane one sincospi per band and axis,
//                     W1's and W4's gamma columns permuted to match);
// then the residual network's adjoint (if it is on) and the skinning
// adjoint (res_bwd.hip).
#include "adjoint_device.h"
#include "kernels.h"

namespace mnr {

constexpr int FREQ_SAVE_WAVES = 4;
constexpr int FREQ_BWD_WAVES = 4;

// Transposed weights as A operands of dX = W^T dY (BF16 fragments):
// W1^T, W2^T, W3^T (64 x 64), W4^T (128 x 64: h3's rows, then gamma's),
// W5^T (64 x 4, padded to 32 columns).
struct FreqTShape {
  static constexpr int FRAG = 64 * 16;
  static constexpr int T1 = 4 * 2 * FRAG, T2 = 4 * 2 * FRAG, T3 = 4 * 2 * FRAG, T4 = 8 * 2 * FRAG, T5 = 4 * 1 * FRAG;
  static constexpr int o2 = T1, o3 = o2 + T2, o4 = o3 + T3, o5 = o4 + T4;
  static constexpr int bytes() { return o5 + T5; }
};

// Block sums of the weight gradients (FP32, row-major with rows padded by
// 4 floats for conflict-free LDS atomics): W1, W2, W3 [64][64],
// W4 [64][128], W5 [4][64].
struct FreqGrad {
  static constexpr int L1 = 68, L2 = 68, L3 = 68, L4 = 132, L5 = 68;  // row strides
  static constexpr int o2 = 64 * L1, o3 = o2 + 64 * L2, o4 = o3 + 64 * L3, o5 = o4 + 64 * L4;
  static constexpr int floats() { return o5 + 4 * L5; }
};

constexpr int FREQ_SAVE_WAVE_BYTES = FreqShape::feat_bytes_per_wave() + 64 * 16;  // gamma + output buffer
constexpr int FREQ_SAVE_LDS = FreqShape::bytes() + FREQ_SAVE_WAVES * FREQ_SAVE_WAVE_BYTES;
constexpr int FREQ_BWD_LDS = FreqTShape::bytes() + FreqGrad::floats() * 4 + FREQ_BWD_WAVES * RES_TB_BYTES;
static_assert(FREQ_SAVE_LDS <= 80 * 1024, "two forward blocks per compute unit");
static_assert(FREQ_BWD_LDS <= 160 * 1024, "LDS of the frequency field's adjoint");

// ---- 1. forward with saved activations, compositing adjoint -----------------

template <bool RES>
__global__ void __launch_bounds__(64 * FREQ_SAVE_WAVES) freq_save_kernel(const RenderArgs a, int n_slots) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  char* wl = lds;
  char* feat = lds + FreqShape::bytes() + wave * FREQ_SAVE_WAVE_BYTES;
  f4* obuf = (f4*)(feat + FreqShape::feat_bytes_per_wave());
  stage_freq(wl, a.f);
  __syncthreads();
  const int nchunks = (a.r.spp + 63) >> 6;
  float* sb = a.split.buf;
  const int64_t ss = a.split.stride;
  for (int slot = blockIdx.x * FREQ_SAVE_WAVES + wave; slot < n_slots; slot += gridDim.x * FREQ_SAVE_WAVES) {
    int orow, n_done;
    RaySetup rs;
    if (!split_ray(a, slot, orow, rs, n_done, nchunks)) continue;
    const f4 gout = *(const f4*)(a.grad_rgba + (size_t)orow * 4);
    float Sc[4] = {a.r.bg[0], a.r.bg[1], a.r.bg[2], 0.f};  // S after the last processed sample
    const float* tc = a.t_chunks + (size_t)orow * (nchunks + 1);
    for (int ch = nchunks - 1; ch >= 0; --ch) {
      const float T0 = tc[ch];
      if (T0 < 0.f || ch * 64 >= n_done) continue;  // not reached by the forward pass
      const int i = ch * 64 + lane;
      const bool valid = i < n_done;
      const int64_t cj = (int64_t)orow * nchunks + ch;
      const int64_t sj = cj * 64 + lane;
      SampleState st;
      if constexpr (RES) {  // x_final and L from the residual network's forward kernel
        st.xs[0] = sb[SPLIT_XF * ss + sj];
        st.xs[1] = sb[(SPLIT_XF + 1) * ss + sj];
        st.xs[2] = sb[(SPLIT_XF + 2) * ss + sj];
        st.L = valid ? sb[SPLIT_L * ss + sj] : 0.f;
      } else {
        const float s = ((float)i + sample_jitter(a.r, orow, i)) * rs.delta;
        st.x[0] = fmaf(s, rs.d[0], rs.p0[0]);
        st.x[1] = fmaf(s, rs.d[1], rs.p0[1]);
        st.x[2] = fmaf(s, rs.d[2], rs.p0[2]);
        st.L = 0.f;
        st.xs[0] = st.xs[1] = st.xs[2] = 0.f;
        if (valid) {
          warp_sample(a.m, a.G, st.x, st.xs, st.L);
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            sb[(SPLIT_X + q) * ss + sj] = st.x[q];
            sb[(SPLIT_XS + q) * ss + sj] = st.xs[q];
            sb[(SPLIT_XF + q) * ss + sj] = st.xs[q];
          }
          sb[SPLIT_L * ss + sj] = st.L > 0.f ? st.L : 0.f;
        }
      }
      st.live = valid && st.L > 0.f;
      const uint64_t live_mask = __ballot(st.live);
      if (live_mask == 0) continue;  // alpha' = 0 everywhere: S passes through unchanged
      store_posenc10(feat, lane, st.xs, st.live);
      wave_sync_lds();
      bf16x8* act = (bf16x8*)a.split.act + cj * FREQ_ACT_VECS;
#pragma unroll 1
      for (int nt = 0; nt < 4; ++nt) {
        f4 o = {0.f, 0.f, 0.f, 0.f};
        if ((live_mask >> (16 * nt)) & 0xFFFFull) o = freq_tile<true>(wl, feat, nt, lane, act);
        if (lane < 16) obuf[nt * 16 + lane] = o;
      }
      wave_sync_lds();
      const f4 out = obuf[lane];
      float g_o[4], g_L;
      composite_adjoint(T0, rs.delta, out, st.L, st.live, gout, Sc, g_o, g_L);
      if (valid) {
#pragma unroll
        for (int q = 0; q < 4; ++q) sb[(SPLIT_GO + q) * ss + sj] = g_o[q];
        sb[SPLIT_GL * ss + sj] = st.live ? g_L : 0.f;
      }
      wave_sync_lds();
    }
  }
}

// ---- 2. the skip MLP's adjoint ----------------------------------------------

// The adjoint holds gamma's 64 inputs in its own order so that each lane
// evaluates one sincospi per (band, axis) pair and takes both its sine and
// its cosine: lane group g's slot n (D-layout input 16 (n / 4) + 4 g + n % 4)
// holds pair p = 8 g + n / 2 (band p / 3, axis p % 3), its sine for even n
// and its cosine for odd n; pairs 30 and 31 (g = 3, slots 12..15) hold the
// raw coordinates and the zero pad.  gamma_input(pos) is the forward's input
// index of adjoint position pos: W1's and W4's gamma columns are staged, and
// their weight gradients written back, through it.
__device__ __forceinline__ int gamma_input(int pos) {
  const int g = (pos >> 2) & 3, n = ((pos >> 4) << 2) | (pos & 3);
  const int p = 8 * g + (n >> 1);
  if (p >= 30) return n == 15 ? 63 : n - 12;
  const int band = p / 3;
  return 3 + 6 * band + 3 * (n & 1) + (p - 3 * band);
}

// stage_t with the input columns from gamma0 on taken in the adjoint's order.
__device__ void stage_t_gamma(char* lds, const __bf16* __restrict__ w, int M, int K, int Kpad, int gamma0) {
  for (int e = threadIdx.x; e < K * Kpad; e += blockDim.x) {
    const int m = e / Kpad, k = e - m * Kpad;  // element (m, k) of W^T
    const int col = m < gamma0 ? m : gamma0 + gamma_input(m - gamma0);
    const float v = (k < M) ? (float)w[(size_t)k * K + col] : 0.0f;
    *(__bf16*)(lds + frag_offset<MNR_BF16>(m, k, Kpad / 32)) = (__bf16)v;
  }
}

// gamma of sample x at lane group g's 16 slots, with d gamma / d x_q: value,
// the derivative and its axis q.  The arguments of sincospi are formed as
// the forward pass forms them, so the values round to the same BF16
// operands.
__device__ __forceinline__ void posenc10_lane(const float x[3], int g, f4 (&val)[4], float (&der)[16],
                                              int (&axis)[16]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int p = 8 * g + j, pc = p < 30 ? p : 29;
    const int band = pc / 3, q = pc - 3 * band;
    const float xq = q == 0 ? x[0] : (q == 1 ? x[1] : x[2]);
    const float f = (float)(1 << band);
    float sv, cv;
    sincospif(f * xq, &sv, &cv);
    const float fpi = f * 3.14159265358979f;
    float v0 = sv, v1 = cv, d0 = cv * fpi, d1 = -sv * fpi;
    int a0 = q, a1 = q;
    if (j >= 6 && p >= 30) {  // the raw coordinates (slots 12, 13, 14) and the pad (15)
      v0 = j == 6 ? x[0] : x[2];
      v1 = j == 6 ? x[1] : 0.f;
      d0 = 1.f;
      d1 = j == 6 ? 1.f : 0.f;
      a0 = j == 6 ? 0 : 2;
      a1 = j == 6 ? 1 : 0;
    }
    const int n0 = 2 * j, n1 = 2 * j + 1;
    val[n0 >> 2][n0 & 3] = v0;
    val[n1 >> 2][n1 & 3] = v1;
    der[n0] = d0;
    der[n1] = d1;
    axis[n0] = a0;
    axis[n1] = a1;
  }
}

__device__ __forceinline__ void load_act(const bf16x8* act, int layer, int nt, int lane, f4 (&h)[4]) {
  const bf16x8 p = act[(layer * 4 + nt) * 128 + lane], q = act[(layer * 4 + nt) * 128 + 64 + lane];
  h[0] = f4{(float)p[0], (float)p[1], (float)p[2], (float)p[3]};
  h[1] = f4{(float)p[4], (float)p[5], (float)p[6], (float)p[7]};
  h[2] = f4{(float)q[0], (float)q[1], (float)q[2], (float)q[3]};
  h[3] = f4{(float)q[4], (float)q[5], (float)q[6], (float)q[7]};
}

// The four waves of a block work on the same rays and chunks in two pairs:
// pair p takes the chunk's 16-sample tiles p and p + 2, both of its waves
// run the tile's whole backward chain (the dX products, cheap on the
// MFMAs), and wave h of the pair sums only rows 32 h .. 32 h + 31 of every
// weight gradient (W5's four rows: h = 0) in MFMA accumulators that stay in
// registers over all of the block's tiles; at the end the two pairs add
// their sums to LDS one after the other.  Wave h = 0 of a pair writes
// dL/dx_final.  Lane c + 16 g works on sample 16 nt + c.
__global__ void __launch_bounds__(64 * FREQ_BWD_WAVES) freq_bwd_kernel(const RenderArgs a, int n_slots) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  char* rt = lds;
  float* dw = (float*)(rt + FreqTShape::bytes());
  __bf16* tb = (__bf16*)((char*)(dw + FreqGrad::floats()) + wave * RES_TB_BYTES);
  stage_t_gamma(rt, (const __bf16*)a.f.w[0], HIDDEN, 64, HIDDEN, 0);
  stage_t(rt + FreqTShape::o2, (const __bf16*)a.f.w[1], HIDDEN, HIDDEN, HIDDEN);
  stage_t(rt + FreqTShape::o3, (const __bf16*)a.f.w[2], HIDDEN, HIDDEN, HIDDEN);
  stage_t_gamma(rt + FreqTShape::o4, (const __bf16*)a.f.w[3], HIDDEN, 2 * HIDDEN, HIDDEN, HIDDEN);
  stage_t(rt + FreqTShape::o5, (const __bf16*)a.f.w[4], 4, HIDDEN, 32);
  for (int i = threadIdx.x; i < FreqGrad::floats(); i += blockDim.x) dw[i] = 0.f;
  __syncthreads();
  const int nchunks = (a.r.spp + 63) >> 6;
  float* sb = a.split.buf;
  const int64_t ss = a.split.stride;
  const int c = lane & 15, g = lane >> 4;
  const f4 z4 = {0.f, 0.f, 0.f, 0.f};
  const int pair = wave >> 1, half = wave & 1;
  // the wave's rows of every weight gradient (W4: [h3; gamma] columns)
  f4 g1[2][4], g2[2][4], g3[2][4], g4[2][8], g5[1][4];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
#pragma unroll
    for (int t = 0; t < 4; ++t) g1[m][t] = g2[m][t] = g3[m][t] = z4;
#pragma unroll
    for (int t = 0; t < 8; ++t) g4[m][t] = z4;
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) g5[0][t] = z4;
  for (int slot = blockIdx.x; slot < n_slots; slot += gridDim.x) {
    int orow, n_done;
    RaySetup rs;
    if (!split_ray(a, slot, orow, rs, n_done, nchunks)) continue;
    const float* tc = a.t_chunks + (size_t)orow * (nchunks + 1);
    for (int ch = 0; ch < nchunks && ch * 64 < n_done; ++ch) {
      if (tc[ch] < 0.f) continue;
      const int i = ch * 64 + lane;
      const int64_t cj = (int64_t)orow * nchunks + ch;
      const int64_t sj = cj * 64 + lane;
      const bool live = i < n_done && sb[SPLIT_L * ss + sj] > 0.f;
      const uint64_t live_mask = __ballot(live);
      if (live_mask == 0) continue;
      float xf[3] = {0.f, 0.f, 0.f}, go[4] = {0.f, 0.f, 0.f, 0.f};
      if (live) {
#pragma unroll
        for (int q = 0; q < 3; ++q) xf[q] = sb[(SPLIT_XF + q) * ss + sj];
#pragma unroll
        for (int q = 0; q < 4; ++q) go[q] = sb[(SPLIT_GO + q) * ss + sj];
      }
      const bf16x8* act = (const bf16x8*)a.split.act + cj * FREQ_ACT_VECS;
#pragma unroll 1
      for (int nt = pair; nt < 4; nt += 2) {
        if (!((live_mask >> (16 * nt)) & 0xFFFFull)) continue;
        const int sl = 16 * nt + c;  // the lane's sample
        const bool slive = (live_mask >> sl) & 1ull;
        float x[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) x[q] = __shfl(xf[q], sl, WAVE);
        f4 gam[4];
        float der[16];
        int axis[16];
        posenc10_lane(x, g, gam, der, axis);
        if (!slive)  // the forward pass fed zeros for samples that are not live
#pragma unroll
          for (int t = 0; t < 4; ++t) gam[t] = z4;
        f4 h1[4], h2[4], h3[4], h4[4];
        load_act(act, 0, nt, lane, h1);
        load_act(act, 1, nt, lane, h2);
        load_act(act, 2, nt, lane, h3);
        load_act(act, 3, nt, lane, h4);
        // output layer: rows 0..3 of sample sl are dL/do
        f4 d5[2] = {z4, z4};
        {
          const float q0 = __shfl(go[0], sl, WAVE), q1 = __shfl(go[1], sl, WAVE);
          const float q2 = __shfl(go[2], sl, WAVE), q3 = __shfl(go[3], sl, WAVE);
          if (g == 0) d5[0] = f4{q0, q1, q2, q3};
        }
        f4 tmp[8], d[4], dgam[4], dr[2];
        if (half == 0) dw_acc<1, 4>(tb, d5, h4, g5, lane);
        mm_t<4, 1>(rt + FreqTShape::o5, d5, tmp, lane);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) d[mt] = relu_mask4(tmp[mt], h4[mt]);
        // layer 4: input [h3; gamma]
        dr[0] = half ? d[2] : d[0];
        dr[1] = half ? d[3] : d[1];
        dw_acc<2, 4, 0>(tb, dr, h3, g4, lane);
        dw_acc<2, 4, 4>(tb, dr, gam, g4, lane);
        mm_t<8, 2>(rt + FreqTShape::o4, d, tmp, lane);
#pragma unroll
        for (int t = 0; t < 4; ++t) dgam[t] = tmp[4 + t];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) d[mt] = relu_mask4(tmp[mt], h3[mt]);
        // layer 3
        dr[0] = half ? d[2] : d[0];
        dr[1] = half ? d[3] : d[1];
        dw_acc<2, 4>(tb, dr, h2, g3, lane);
        mm_t<4, 2>(rt + FreqTShape::o3, d, tmp, lane);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) d[mt] = relu_mask4(tmp[mt], h2[mt]);
        // layer 2
        dr[0] = half ? d[2] : d[0];
        dr[1] = half ? d[3] : d[1];
        dw_acc<2, 4>(tb, dr, h1, g2, lane);
        mm_t<4, 2>(rt + FreqTShape::o2, d, tmp, lane);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) d[mt] = relu_mask4(tmp[mt], h1[mt]);
        // layer 1: input gamma
        dr[0] = half ? d[2] : d[0];
        dr[1] = half ? d[3] : d[1];
        dw_acc<2, 4>(tb, dr, gam, g1, lane);
        if (half != 0) continue;
        mm_t<4, 2>(rt, d, tmp, lane);
#pragma unroll
        for (int t = 0; t < 4; ++t) dgam[t] += tmp[t];
        // dL/dx_final of sample sl: the lane's 16 inputs, then the 4 lane groups
        float gx[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int n = 0; n < 16; ++n) {
          const float v = dgam[n >> 2][n & 3] * der[n];
          gx[0] += axis[n] == 0 ? v : 0.f;
          gx[1] += axis[n] == 1 ? v : 0.f;
          gx[2] += axis[n] == 2 ? v : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          gx[q] += __shfl_xor(gx[q], 16, WAVE);
          gx[q] += __shfl_xor(gx[q], 32, WAVE);
        }
        if (g == 0 && slive)
#pragma unroll
          for (int q = 0; q < 3; ++q) sb[(SPLIT_G + q) * ss + cj * 64 + sl] = gx[q];
      }
    }
  }
  // the pairs add their rows to the block's LDS sums one after the other
  for (int pp = 0; pp < 2; ++pp) {
    if (pair == pp) {
      add_dw(g1, dw + 32 * half * FreqGrad::L1, 32, FreqGrad::L1, lane);
      add_dw(g2, dw + FreqGrad::o2 + 32 * half * FreqGrad::L2, 32, FreqGrad::L2, lane);
      add_dw(g3, dw + FreqGrad::o3 + 32 * half * FreqGrad::L3, 32, FreqGrad::L3, lane);
      add_dw(g4, dw + FreqGrad::o4 + 32 * half * FreqGrad::L4, 32, FreqGrad::L4, lane);
      if (half == 0) add_dw(g5, dw + FreqGrad::o5, 4, FreqGrad::L5, lane);
    }
    __syncthreads();
  }
  // flush: element k of layer l (row-major, K columns) sits at row k / K of
  // the padded block
  const int cols[5] = {64, 64, 64, 128, 64}, rows[5] = {64, 64, 64, 64, 4};
  const int ld[5] = {FreqGrad::L1, FreqGrad::L2, FreqGrad::L3, FreqGrad::L4, FreqGrad::L5};
  const int off[5] = {0, FreqGrad::o2, FreqGrad::o3, FreqGrad::o4, FreqGrad::o5};
#pragma unroll
  for (int l = 0; l < 5; ++l)
    for (int k = threadIdx.x; k < rows[l] * cols[l]; k += blockDim.x) {
      const int r = k / cols[l];
      const int c = k - r * cols[l];
      const float v = dw[off[l] + r * ld[l] + c];
      // W1's columns and W4's gamma columns back in the forward's input order
      const int col = l == 0 ? gamma_input(c) : (l == 3 && c >= 64 ? 64 + gamma_input(c - 64) : c);
      if (v != 0.f) unsafeAtomicAdd(a.grad_w[l] + r * cols[l] + col, v);
    }
}

template <bool RES>
static void launch_save(const RenderArgs& a, int n_slots, hipStream_t st) {
  static PersistentGrid pg;
  auto kern = freq_save_kernel<RES>;
  const int mb = persistent_blocks(kern, 64 * FREQ_SAVE_WAVES, FREQ_SAVE_LDS, pg);
  const int need = (n_slots + FREQ_SAVE_WAVES - 1) / FREQ_SAVE_WAVES;
  hipLaunchKernelGGL(kern, dim3(need < mb ? (need > 0 ? need : 1) : mb), dim3(64 * FREQ_SAVE_WAVES), FREQ_SAVE_LDS,
                     st, a, n_slots);
}

hipError_t launch_freq_backward(const RenderArgs& a, int n_slots, hipStream_t st) {
  if (a.res.w[0]) launch_save<true>(a, n_slots, st);
  else launch_save<false>(a, n_slots, st);
  static PersistentGrid pg;
  const int mb = persistent_blocks(freq_bwd_kernel, 64 * FREQ_BWD_WAVES, FREQ_BWD_LDS, pg);
  hipLaunchKernelGGL(freq_bwd_kernel, dim3(n_slots < mb ? (n_slots > 0 ? n_slots : 1) : mb),
                     dim3(64 * FREQ_BWD_WAVES), FREQ_BWD_LDS, st, a, n_slots);
  return hipGetLastError();
}

}  // namespace mnr
