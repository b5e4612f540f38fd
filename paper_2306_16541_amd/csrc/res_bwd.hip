// Adjoint of the residual non-rigid motion network (Sec. 4.3, Eq. 11-12),
// as a split adjoint (training, Sec. 5.2).
//
// With the residual network the field is queried at x_final = x_skel +
// MLP_res(gamma(x_skel), Omega), so the adjoint has to pass through a second
// MLP between the field's adjoint and the skinning adjoint.  The fused
// adjoint kernel has no LDS left for its weights, so the chain runs as four
// kernels over the same ray chunks, handing per-sample values through a
// scratch buffer (SplitArgs); the forward pass still saves nothing per
// sample:
//   res_fwd_kernel   x -> inverse LBS -> x_skel, L -> residual network ->
//                    x_final (stored with x, x_skel, L);
//   render_bwd_kernel<SPLIT>  the field's adjoint at x_final (compositing,
//                    MLP, encoding), storing dL/dx_final and dL/dL;
//   res_bwd_kernel   the residual network recomputed on MFMA and
//                    differentiated: dL/dW1..W5 (block sums in LDS), the
//                    sum of the first layer's pre-activation gradients (for
//                    dL/dW_omega), and dL/dx_skel = dL/dx_final +
//                    (d x_res / d x_skel)^T dL/dx_final (stored apart from
//                    dL/dx_final);
//   skin_bwd_kernel  the skinning adjoint with dL/dx_skel (dL/dW^c, dL/dG);
//   omega_grad_kernel  dL/dW_omega = (sum of layer-1 gradients) Omega^T.
#include "adjoint_device.h"
#include "kernels.h"

namespace mnr {

constexpr int RES_FWD_WAVES = 8;
constexpr int SKIN_WAVES = 8;

// ---- 1. forward of the warp and the residual network ------------------------

__global__ void __launch_bounds__(64 * RES_FWD_WAVES) res_fwd_kernel(const RenderArgs a, int n_slots) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  char* rl = lds;
  char* feat = lds + ResShape::bytes() + wave * MlpShape<MNR_BF16>::feat_bytes_per_wave();
  stage_residual(rl, a.res);
  __syncthreads();
  const int nchunks = (a.r.spp + 63) >> 6;
  float* sb = a.split.buf;
  const int64_t ss = a.split.stride;
  for (int slot = blockIdx.x * RES_FWD_WAVES + wave; slot < n_slots; slot += gridDim.x * RES_FWD_WAVES) {
    int orow, n_done;
    RaySetup rs;
    if (!split_ray(a, slot, orow, rs, n_done, nchunks)) continue;
    const float* tc = a.t_chunks + (size_t)orow * (nchunks + 1);
    for (int ch = 0; ch < nchunks && ch * 64 < n_done; ++ch) {
      if (tc[ch] < 0.f) continue;
      const int i = ch * 64 + lane;
      const bool valid = i < n_done;
      const int64_t sj = ((int64_t)orow * nchunks + ch) * 64 + lane;
      SampleState st;
      const float s = ((float)i + sample_jitter(a.r, orow, i)) * rs.delta;
      st.x[0] = fmaf(s, rs.d[0], rs.p0[0]);
      st.x[1] = fmaf(s, rs.d[1], rs.p0[1]);
      st.x[2] = fmaf(s, rs.d[2], rs.p0[2]);
      st.L = 0.f;
      st.xs[0] = st.xs[1] = st.xs[2] = 0.f;
      if (valid) warp_sample(a.m, a.G, st.x, st.xs, st.L);
      st.live = valid && st.L > 0.f;
      const float xs0 = st.xs[0], xs1 = st.xs[1], xs2 = st.xs[2];
      const uint64_t live_mask = __ballot(st.live);
      if (live_mask) residual_step(a.res, rl, feat, (f4*)feat, st, live_mask, lane);
      if (valid) {
        sb[SPLIT_X * ss + sj] = st.x[0];
        sb[(SPLIT_X + 1) * ss + sj] = st.x[1];
        sb[(SPLIT_X + 2) * ss + sj] = st.x[2];
        sb[SPLIT_XS * ss + sj] = xs0;
        sb[(SPLIT_XS + 1) * ss + sj] = xs1;
        sb[(SPLIT_XS + 2) * ss + sj] = xs2;
        sb[SPLIT_XF * ss + sj] = st.xs[0];
        sb[(SPLIT_XF + 1) * ss + sj] = st.xs[1];
        sb[(SPLIT_XF + 2) * ss + sj] = st.xs[2];
        sb[SPLIT_L * ss + sj] = st.live ? st.L : 0.f;
      }
      wave_sync_lds();
    }
  }
}

// ---- 2. the residual network's adjoint ---------------------------------------

// Transposed weights W_k^T as A operands (BF16 fragment layout), for
// dX = W^T dY: W1^T (32 x 64), W2^T, W3^T (64 x 64), W4^T (96 x 64), W5^T
// (64 x 3, padded to 32 columns).
struct ResTShape {
  static constexpr int FRAG = 64 * 16;
  static constexpr int T1 = 2 * 2 * FRAG, T2 = 4 * 2 * FRAG, T3 = 4 * 2 * FRAG, T4 = 6 * 2 * FRAG, T5 = 4 * 1 * FRAG;
  static constexpr int o2 = T1, o3 = o2 + T2, o4 = o3 + T3, o5 = o4 + T4;
  static constexpr int bytes() { return o5 + T5; }
};

// Block sums of the weight gradients (FP32, rows padded by 4 floats for
// conflict-free LDS atomics): W1 [64][32] (column 27, an input that gamma
// never uses, carries the bias gradient: see below), W2, W3 [64][64],
// W4 [64][96], W5 [3][64].
struct ResGrad {
  static constexpr int L1 = 36, L2 = 68, L3 = 68, L4 = 100, L5 = 68;  // row strides
  static constexpr int o2 = 64 * L1, o3 = o2 + 64 * L2, o4 = o3 + 64 * L3, o5 = o4 + 64 * L4;
  static constexpr int floats() { return o5 + 3 * L5; }
};
constexpr int BIAS_COL = 27;  // gamma has 27 values; inputs 27..31 are zero padding

constexpr int RES_BWD_WAVES = 4;
constexpr int RES_BWD_LDS = ResShape::bytes() + ResTShape::bytes() + ResGrad::floats() * 4 + RES_BWD_WAVES * RES_TB_BYTES;
static_assert(RES_BWD_LDS <= 160 * 1024, "LDS of the residual adjoint");

// gamma(x_skel) of the residual network (Hann-windowed, 27 values, zero
// padded to 32) at the 8 inputs k = 16 t + 4 g + e (t = 0, 1; e = 0..3)
// that lane group g holds in the D layout, with d gamma_k / d x_q(k):
// value, derivative, axis.  Values are formed as the forward pass forms
// them, so they round to the same BF16 operands.
__device__ __forceinline__ void res_posenc_lane(const float x[3], const float (&win)[4], int g, f4 (&val)[2],
                                                float (&der)[8], int (&axis)[8]) {
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 16 * t + 4 * g + e, n = 4 * t + e;
      float v = 0.f, d = 0.f;
      int q = 0;
      if (k < 3) {
        q = k;
        v = x[0];
        if (k == 1) v = x[1];
        if (k == 2) v = x[2];
        d = 1.f;
      } else if (k < 27) {
        const int band = (k - 3) / 6, r = (k - 3) - 6 * ((k - 3) / 6);
        q = r < 3 ? r : r - 3;
        const float xq = q == 0 ? x[0] : (q == 1 ? x[1] : x[2]);
        const float w = band == 0 ? win[0] : (band == 1 ? win[1] : (band == 2 ? win[2] : win[3]));
        float sv, cv;
        sincospif((float)(1 << band) * xq, &sv, &cv);
        v = w * (r < 3 ? sv : cv);
        d = w * (float)(1 << band) * 3.14159265358979f * (r < 3 ? cv : -sv);
      }
      val[t][e] = v;
      der[n] = d;
      axis[n] = q;
    }
}

// Four waves per block share the weights, their transposes and the
// gradient sums, and work on the same rays and chunks in two pairs: pair p
// takes the chunk's 16-sample tiles p and p + 2, both of its waves
// recompute the tile's forward pass and run the whole backward chain (the
// products are cheap on the MFMAs), and wave h of the pair sums only rows
// 32 h .. 32 h + 31 of every weight gradient (W5's three rows: h = 0) in
// MFMA accumulators that stay in registers over all of the block's tiles;
// at the end the two pairs add their sums to LDS one after the other.
// gamma and its derivative are formed in registers, in the D layout; wave
// h = 0 of a pair writes dL/dx_skel = dL/dx_final + (d gamma / d x_skel)^T
// dL/dgamma, to a field of its own (the other waves may still be reading
// dL/dx_final).
__global__ void __launch_bounds__(64 * RES_BWD_WAVES) res_bwd_kernel(const RenderArgs a, int n_slots) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  char* rl = lds;
  char* rt = rl + ResShape::bytes();
  float* dw = (float*)(rt + ResTShape::bytes());
  __bf16* tb = (__bf16*)((char*)(dw + ResGrad::floats()) + wave * RES_TB_BYTES);
  stage_residual(rl, a.res);
  stage_t(rt, a.res.w[0], HIDDEN, 32, HIDDEN);
  stage_t(rt + ResTShape::o2, a.res.w[1], HIDDEN, HIDDEN, HIDDEN);
  stage_t(rt + ResTShape::o3, a.res.w[2], HIDDEN, HIDDEN, HIDDEN);
  stage_t(rt + ResTShape::o4, a.res.w[3], HIDDEN, HIDDEN + 32, HIDDEN);
  stage_t(rt + ResTShape::o5, a.res.w[4], 3, HIDDEN, 32);
  for (int i = threadIdx.x; i < ResGrad::floats(); i += blockDim.x) dw[i] = 0.f;
  __syncthreads();
  const float* bias = (const float*)(rl + ResShape::obias);
  const float win[4] = {a.res.win[0], a.res.win[1], a.res.win[2], a.res.win[3]};
  const int nchunks = (a.r.spp + 63) >> 6;
  float* sb = a.split.buf;
  const int64_t ss = a.split.stride;
  const int c = lane & 15, g = lane >> 4;
  const f4 z4 = {0.f, 0.f, 0.f, 0.f};
  const int pair = wave >> 1, half = wave & 1;
  // the wave's rows of every weight gradient (W4: [h3; gamma] columns)
  f4 g1[2][2], g2[2][4], g3[2][4], g4[2][6], g5[1][4];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    g1[m][0] = g1[m][1] = z4;
#pragma unroll
    for (int t = 0; t < 4; ++t) g2[m][t] = g3[m][t] = z4;
#pragma unroll
    for (int t = 0; t < 6; ++t) g4[m][t] = z4;
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
      float xs[3] = {0.f, 0.f, 0.f}, gf[3] = {0.f, 0.f, 0.f};
      if (live) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          xs[q] = sb[(SPLIT_XS + q) * ss + sj];
          gf[q] = sb[(SPLIT_G + q) * ss + sj];
        }
      }
#pragma unroll 1
      for (int nt = pair; nt < 4; nt += 2) {
        if (!((live_mask >> (16 * nt)) & 0xFFFFull)) continue;
        const int sl = 16 * nt + c;  // the lane's sample
        const bool slive = (live_mask >> sl) & 1ull;
        float x3[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) x3[q] = __shfl(xs[q], sl, WAVE);
        f4 x[4];
        float der[8];
        int axis[8];
        {
          f4 v2[2];
          res_posenc_lane(x3, win, g, v2, der, axis);
          x[0] = slive ? v2[0] : z4;  // the forward pass fed zeros for samples that are not live
          x[1] = slive ? v2[1] : z4;
          x[2] = x[3] = z4;
        }
        // forward, as residual_step
        f4 h1[4], h2[4], h3[4], h4[4], tmp[6];
        mma_layer<MNR_BF16, 4, 2>(rl, x, h1, lane, bias);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) h1[mt] = relu4(h1[mt]);
        mma_layer<MNR_BF16, 4, 4>(rl + ResShape::o2, h1, h2, lane);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) h2[mt] = relu4(h2[mt]);
        mma_layer<MNR_BF16, 4, 4>(rl + ResShape::o3, h2, h3, lane);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) h3[mt] = relu4(h3[mt]);
        const f4 cat[6] = {h3[0], h3[1], h3[2], h3[3], x[0], x[1]};
        mma_layer<MNR_BF16, 4, 6>(rl + ResShape::o4, cat, h4, lane);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) h4[mt] = relu4(h4[mt]);
        // output gradient: rows 0..2 of sample sl are dL/dx_res = dL/dx_final
        const float q0 = __shfl(gf[0], sl, WAVE), q1 = __shfl(gf[1], sl, WAVE), q2 = __shfl(gf[2], sl, WAVE);
        f4 d5[2] = {g == 0 ? f4{q0, q1, q2, 0.f} : z4, z4};
        if (half == 0) dw_acc<1, 4>(tb, d5, h4, g5, lane);
        f4 d[4], rows[2], dg2[2];
        mm_t<4, 1>(rt + ResTShape::o5, d5, tmp, lane);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) d[mt] = relu_mask4(tmp[mt], h4[mt]);
        // layer 4: input [h3; gamma]
        rows[0] = half ? d[2] : d[0];
        rows[1] = half ? d[3] : d[1];
        dw_acc<2, 4, 0>(tb, rows, h3, g4, lane);
        dw_acc<2, 2, 4>(tb, rows, x, g4, lane);
        mm_t<6, 2>(rt + ResTShape::o4, d, tmp, lane);
        dg2[0] = tmp[4];
        dg2[1] = tmp[5];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) d[mt] = relu_mask4(tmp[mt], h3[mt]);
        // layer 3
        rows[0] = half ? d[2] : d[0];
        rows[1] = half ? d[3] : d[1];
        dw_acc<2, 4>(tb, rows, h2, g3, lane);
        mm_t<4, 2>(rt + ResTShape::o3, d, tmp, lane);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) d[mt] = relu_mask4(tmp[mt], h2[mt]);
        // layer 2
        rows[0] = half ? d[2] : d[0];
        rows[1] = half ? d[3] : d[1];
        dw_acc<2, 4>(tb, rows, h1, g2, lane);
        mm_t<4, 2>(rt + ResTShape::o2, d, tmp, lane);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) d[mt] = relu_mask4(tmp[mt], h1[mt]);
        // layer 1: the pose term enters as a bias, so the bias gradient is
        // the sum of d over the samples: gamma's unused input 27 is set to
        // 1 here (it is 0 in the forward pass) and its column of dW1
        // collects exactly that sum
        f4 xb[2] = {x[0], x[1]};
        if (g == 2) xb[1][3] = 1.f;  // input 16 + 4 g + 3 = 27
        rows[0] = half ? d[2] : d[0];
        rows[1] = half ? d[3] : d[1];
        dw_acc<2, 2>(tb, rows, xb, g1, lane);
        if (half != 0) continue;
        mm_t<2, 2>(rt, d, tmp, lane);
        dg2[0] += tmp[0];
        dg2[1] += tmp[1];
        // dL/dx_skel of sample sl: the lane's 8 inputs, then the 4 lane groups
        float gx[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int n = 0; n < 8; ++n) {
          const float v = dg2[n >> 2][n & 3] * der[n];
          gx[0] += axis[n] == 0 ? v : 0.f;
          gx[1] += axis[n] == 1 ? v : 0.f;
          gx[2] += axis[n] == 2 ? v : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          gx[q] += __shfl_xor(gx[q], 16, WAVE);
          gx[q] += __shfl_xor(gx[q], 32, WAVE);
        }
        const float gq[3] = {q0, q1, q2};
        if (g == 0 && slive)
#pragma unroll
          for (int q = 0; q < 3; ++q) sb[(SPLIT_GS + q) * ss + cj * 64 + sl] = gq[q] + gx[q];
      }
    }
  }
  // the pairs add their rows to the block's LDS sums one after the other
  for (int pp = 0; pp < 2; ++pp) {
    if (pair == pp) {
      add_dw(g1, dw + 32 * half * ResGrad::L1, 32, ResGrad::L1, lane);
      add_dw(g2, dw + ResGrad::o2 + 32 * half * ResGrad::L2, 32, ResGrad::L2, lane);
      add_dw(g3, dw + ResGrad::o3 + 32 * half * ResGrad::L3, 32, ResGrad::L3, lane);
      add_dw(g4, dw + ResGrad::o4 + 32 * half * ResGrad::L4, 32, ResGrad::L4, lane);
      if (half == 0) add_dw(g5, dw + ResGrad::o5, 3, ResGrad::L5, lane);
    }
    __syncthreads();
  }
  // flush the block's sums (element k of layer l sits at row k / K of the
  // padded block); column 27 of dW1 is the bias gradient
  const int cols[5] = {32, 64, 64, 96, 64}, rows[5] = {64, 64, 64, 64, 3};
  const int ld[5] = {ResGrad::L1, ResGrad::L2, ResGrad::L3, ResGrad::L4, ResGrad::L5};
  const int off[5] = {0, ResGrad::o2, ResGrad::o3, ResGrad::o4, ResGrad::o5};
#pragma unroll
  for (int l = 0; l < 5; ++l)
    for (int k = threadIdx.x; k < rows[l] * cols[l]; k += blockDim.x) {
      const int r = k / cols[l], c = k - r * cols[l];
      const float v = dw[off[l] + r * ld[l] + c];
      if (v == 0.f) continue;
      if (l == 0 && c == BIAS_COL) unsafeAtomicAdd(a.split.dbias + r, v);
      else unsafeAtomicAdd(a.grad_res[l] + k, v);
    }
}

// ---- 3. the skinning adjoint with dL/dx_skel ----------------------------------

__global__ void __launch_bounds__(64 * SKIN_WAVES) skin_bwd_kernel(const RenderArgs a, int n_slots) {
  __shared__ float dg[MNR_MAX_BONES * 12];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < MNR_MAX_BONES * 12; i += blockDim.x) dg[i] = 0.f;
  __syncthreads();
  const int nchunks = (a.r.spp + 63) >> 6;
  const float* sb = a.split.buf;
  const int64_t ss = a.split.stride;
  const int gfield = a.res.w[0] ? SPLIT_GS : SPLIT_G;  // dL/dx_skel
  uint32_t wc_mb = 0u;  // largest |value| of the lane's blend-weight records (float bits)
  for (int slot = blockIdx.x * SKIN_WAVES + wave; slot < n_slots; slot += gridDim.x * SKIN_WAVES) {
    int orow, n_done;
    RaySetup rs;
    if (!split_ray(a, slot, orow, rs, n_done, nchunks)) continue;
    const float* tc = a.t_chunks + (size_t)orow * (nchunks + 1);
    for (int ch = 0; ch < nchunks && ch * 64 < n_done; ++ch) {
      if (tc[ch] < 0.f) continue;
      const int i = ch * 64 + lane;
      const int64_t sj = ((int64_t)orow * nchunks + ch) * 64 + lane;
      const float L = i < n_done ? sb[SPLIT_L * ss + sj] : 0.f;
      const bool live = L > 0.f;
      if (__ballot(live) == 0) continue;
      float x[3] = {0.f, 0.f, 0.f}, xs[3] = {0.f, 0.f, 0.f}, gs[3] = {0.f, 0.f, 0.f}, gL = 0.f;
      if (live) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          x[q] = sb[(SPLIT_X + q) * ss + sj];
          xs[q] = sb[(SPLIT_XS + q) * ss + sj];
          gs[q] = sb[(gfield + q) * ss + sj];
        }
        gL = sb[SPLIT_GL * ss + sj];
      }
      WcRecords wcr{false, 0u, 0u};
      if (a.rec.keys && a.rec.wc) {  // blend-weight records: one reservation per chunk
        const uint32_t cnt = wc_record_count(a, x, live);
        uint32_t b = 0;
        if (lane == 0 && cnt) b = atomicAdd(a.rec.cursor, cnt);
        const uint32_t base = __builtin_amdgcn_readfirstlane(b);
        wcr = WcRecords{cnt > 0 && (uint64_t)base + cnt <= (uint64_t)a.rec.cap, base, base + cnt};
      }
      skin_adjoint(a, x, xs, L, gs, gL, live, dg, wcr, wc_mb);
    }
  }
  if (a.rec.keys) flush_value_bounds(a.rec, 0u, wc_mb);
  __syncthreads();
  if (a.grad_G)
    for (int i = threadIdx.x; i < a.m.n_bones * 12; i += blockDim.x)
      if (dg[i] != 0.f) unsafeAtomicAdd(a.grad_G + i, dg[i]);
}

// dL/dW_omega[i][j] += dbias[i] Omega[j].
__global__ void omega_grad_kernel(const RenderArgs a) {
  const int n = a.res.n_omega;
  for (int e = threadIdx.x + blockIdx.x * blockDim.x; e < HIDDEN * n; e += blockDim.x * gridDim.x)
    a.grad_res[5][e] += a.split.dbias[e / n] * a.res.omega[e % n];
}

hipError_t launch_res_forward(const RenderArgs& a, int n_slots, hipStream_t st) {
  const int lds = ResShape::bytes() + RES_FWD_WAVES * MlpShape<MNR_BF16>::feat_bytes_per_wave();
  static PersistentGrid pg;
  const int mb = persistent_blocks(res_fwd_kernel, 64 * RES_FWD_WAVES, lds, pg);
  const int need = (n_slots + RES_FWD_WAVES - 1) / RES_FWD_WAVES;
  hipLaunchKernelGGL(res_fwd_kernel, dim3(need < mb ? (need > 0 ? need : 1) : mb), dim3(64 * RES_FWD_WAVES), lds, st,
                     a, n_slots);
  return hipGetLastError();
}

hipError_t launch_res_backward(const RenderArgs& a, int n_slots, hipStream_t st) {
  static PersistentGrid pg;
  const int mb = persistent_blocks(res_bwd_kernel, 64 * RES_BWD_WAVES, RES_BWD_LDS, pg);
  hipLaunchKernelGGL(res_bwd_kernel, dim3(n_slots < mb ? (n_slots > 0 ? n_slots : 1) : mb),
                     dim3(64 * RES_BWD_WAVES), RES_BWD_LDS, st, a, n_slots);
  hipLaunchKernelGGL(omega_grad_kernel, dim3(16), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_skin_backward(const RenderArgs& a, int n_slots, hipStream_t st) {
  static PersistentGrid pg;
  const int mb = persistent_blocks(skin_bwd_kernel, 64 * SKIN_WAVES, 0, pg);
  const int need = (n_slots + SKIN_WAVES - 1) / SKIN_WAVES;
  hipLaunchKernelGGL(skin_bwd_kernel, dim3(need < mb ? (need > 0 ? need : 1) : mb), dim3(64 * SKIN_WAVES), 0, st, a,
                     n_slots);
  return hipGetLastError();
}

}  // namespace mnr
