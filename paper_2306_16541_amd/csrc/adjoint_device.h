// Device helpers of the adjoint kernels (training, Sec. 5.2): segmented
// run sums that cut the number of gradient atomics, the skinning adjoint of
// one sample per lane (Eq. 7 and 9), the compositing adjoint of a chunk
// (Eq. 3), and the BF16 MFMA pieces of an MLP adjoint, shared by the fused
// adjoint and the split ones (residual motion network, frequency-encoded
// field).
#pragma once
#include "field_device.h"

namespace mnr {

// Gradient scatter with fewer atomics (or records).  The 64 lanes of a
// wave are 64 consecutive samples of one ray, so at coarse grid levels (and
// in the blend-weight volume) neighbouring lanes often fall in the same cell
// and would add to the same addresses.  Such runs are summed across the
// wave first and only the last lane of a run (its owner) issues the atomics
// or writes the record.
struct CellRuns {
  int seg;     // run index of the lane (number of run starts at lanes <= lane)
  int steps;   // in-row scan steps needed for the longest run (0..4)
  bool owner;  // last lane of its run: holds the run's sum after run_sums
  bool b15;    // (wave-uniform) a run crosses from row 0 to 1 or from row 2 to 3
  bool b31;    // (wave-uniform) a run crosses from row 1 to 2
};

// Lane i - 1's value across the whole wave (DPP wave_shr:1; lane 0 keeps old).
__device__ __forceinline__ int wave_prev(int x, int old) {
  return __builtin_amdgcn_update_dpp(old, x, 0x138, 0xf, 0xf, false);
}

__device__ __forceinline__ CellRuns cell_runs(bool live, int x, int y, int z) {
  const int lane = lane_id();
  const int px = wave_prev(x, 0), py = wave_prev(y, 0), pz = wave_prev(z, 0);
  const int plive = wave_prev(live ? 1 : 0, 0);
  const bool head = !live || lane == 0 || !plive || px != x || py != y || pz != z;
  const uint64_t heads = __ballot(head);
  CellRuns r;
  r.seg = (int)__popcll(heads & (~0ull >> (63 - lane)));
  r.owner = lane == WAVE - 1 || (((heads >> lane) >> 1) & 1ull);
  r.b15 = !((heads >> 16) & (heads >> 48) & 1ull);
  r.b31 = !((heads >> 32) & 1ull);
  // Longest run within a row: a run of length >= 2^j + 1 needs 2^j
  // non-start lanes in a row after its start; count the doublings (at most
  // 4 within a 16-lane row; bits past lane 63 are starts).
  uint64_t z0 = ~heads;
  int steps = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (z0 == 0) break;
    ++steps;
    z0 &= z0 >> (1 << j);
  }
  r.steps = steps;
  return r;
}

// One step of the segmented scan: every lane adds the value DPP control
// CTRL brings from another lane (0 where it brings none) when that lane is
// in the same run.
template <int CTRL, int ROWS, int NV>
__device__ __forceinline__ void run_step(int seg, float (&v)[NV]) {
  const bool same = __builtin_amdgcn_update_dpp(-1, seg, CTRL, ROWS, 0xf, false) == seg;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const float o = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v[k]), CTRL,
                                                                          ROWS, 0xf, false));
    v[k] += same ? o : 0.f;
  }
}

// In-run prefix sums on DPP (no LDS traffic): afterwards the last lane of
// every run holds the sum of the run's values.  Segmented Hillis-Steele
// scan within each 16-lane row (row_shr 1, 2, 4, 8, as far as the longest
// run needs), then the row carries (row_bcast 15 into rows 1 and 3,
// row_bcast 31 into rows 2 and 3), each only where some run crosses.
template <int NV>
__device__ __forceinline__ void run_sums(const CellRuns& r, float (&v)[NV]) {
  if (r.steps >= 1) run_step<0x111, 0xf>(r.seg, v);
  if (r.steps >= 2) run_step<0x112, 0xf>(r.seg, v);
  if (r.steps >= 3) run_step<0x114, 0xf>(r.seg, v);
  if (r.steps >= 4) run_step<0x118, 0xf>(r.seg, v);
  if (r.b15) run_step<0x142, 0xa>(r.seg, v);
  if (r.b31) run_step<0x143, 0xc>(r.seg, v);
}

// The wave's largest value bounds (float bits) into the sink's bounds: one
// atomic per wave at the end of a kernel that wrote records.
__device__ __forceinline__ void flush_value_bounds(const RecordSink& rec, uint32_t tab_mb, uint32_t wc_mb) {
#pragma unroll
  for (int k = WAVE / 2; k > 0; k >>= 1) {
    tab_mb = max(tab_mb, (uint32_t)__shfl_xor((int)tab_mb, k, WAVE));
    wc_mb = max(wc_mb, (uint32_t)__shfl_xor((int)wc_mb, k, WAVE));
  }
  if (lane_id() == 0) {
    if (tab_mb) atomicMax(rec.vmax, tab_mb);
    if (wc_mb) atomicMax(rec.vmax + 1, wc_mb);
  }
}

// Corner pair q of a weight-volume cell (corners 2q at x0 and 2q + 1 at
// x0 + 1, both at y0 + (q & 1), z0 + (q >> 1)) has a corner inside the
// volume.  Points far from a bone map far outside its volume, so most
// cells of most bones have none.
__device__ __forceinline__ bool wc_pair_inside(const Tri& t, int R, int q) {
  return (unsigned)(t.i0[1] + (q & 1)) < (unsigned)R && (unsigned)(t.i0[2] + (q >> 1)) < (unsigned)R &&
         t.i0[0] >= -1 && t.i0[0] < R;
}

// Blend-weight gradient records of one chunk: per bone and run of live
// lanes in one cell of that bone's weight volume, one per corner pair with a
// corner inside the volume.  Computes the cells exactly as skin_adjoint
// does (the same explicit-FMA transform and cell rounding), so the count
// matches what it writes; skin_adjoint still never writes past the count.
__device__ __forceinline__ uint32_t wc_record_count(const RenderArgs& a, const float x[3], bool live) {
  uint32_t n = 0;
#pragma unroll 1
  for (int b = 0; b < a.m.n_bones; ++b) {
    float y[3];
    bone_apply(a.G[b], x, y);
    const Tri t = bone_cell(a.m, y);
    const CellRuns cr = cell_runs(live, t.i0[0], t.i0[1], t.i0[2]);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      n += (uint32_t)__popcll(__ballot(live && cr.owner && wc_pair_inside(t, a.m.res, q)));
  }
  return n;
}

// Where skin_adjoint writes the chunk's blend-weight records: [base, end)
// (records == false: global atomics).  It raises wc_mb (the lane's largest
// |value| written, as float bits: non-negative floats order as their bits,
// NaN above infinity) for the binned sums' scale.
struct WcRecords {
  bool records;
  uint32_t base, end;
};

// Skinning adjoint (Eq. 7, 9) of one sample per lane.  x: observed point,
// xs: x_skel, L: the weight sum, g_xs: dL/dx_skel, g_L: dL/dL (the
// likelihood factor alpha' = alpha min(L, 1)).  Per bone i:
// dL/dw_i = dL/dx_skel . (y_i - x_skel) / L + dL/dL, scattered through the
// trilinear weights into dL/dW^c (runs of lanes in one cell summed first;
// global atomics, or records for the binned scatter laid out bone after
// bone and corner pair after corner pair, one per run with a corner of the
// pair inside the volume); optionally dL/dG_i into
// the block's LDS sums dg[n_bones][12].  Every lane of the wave takes part
// (the run detection shuffles across it); lanes that are not live
// contribute nothing.
__device__ __forceinline__ void skin_adjoint(const RenderArgs& a, const float x[3], const float xs[3], float L,
                                             const float g_xs[3], float g_L, bool live, float* dg,
                                             const WcRecords wr, uint32_t& wc_mb) {
  const int lane = lane_id();
  const int R = a.m.res;
  const size_t plane = (size_t)R * R * R;
  const bool above = L > EPS_L;
  const float invL = 1.f / (above ? L : EPS_L);
  const float gL = live ? g_L : 0.f;
  uint32_t wc_off = wr.base;  // next record of the chunk
#pragma unroll 1
  for (int b = 0; b < a.m.n_bones; ++b) {
    float y[3];
    bone_apply(a.G[b], x, y);
    const float dx = above ? y[0] - xs[0] : y[0];
    const float dy = above ? y[1] - xs[1] : y[1];
    const float dz = above ? y[2] - xs[2] : y[2];
    const float gw = live ? (g_xs[0] * dx + g_xs[1] * dy + g_xs[2] * dz) * invL + gL : 0.f;
    const Tri t = bone_cell(a.m, y);
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      v[k] = gw * ((k & 1) ? t.f[0] : 1.f - t.f[0]) * ((k & 2) ? t.f[1] : 1.f - t.f[1]) *
             ((k & 4) ? t.f[2] : 1.f - t.f[2]);
    if (a.grad_G) {  // uniform: dL/dG_b = dL/dy_b [x 1]^T, summed over the wave, then the block
      // dL/dy_b = w_b / max(L, eps) dL/dx_skel + dL/dw_b grad_y w_b(y_b)
      float c[8];
      bone_corners(a.m, b, t, c);
      const float w = trilerp(c, t.f);
      const float fx = t.f[0], fy = t.f[1], fz = t.f[2];
      const float x00 = c[0] + fx * (c[1] - c[0]), x10 = c[2] + fx * (c[3] - c[2]);
      const float x01 = c[4] + fx * (c[5] - c[4]), x11 = c[6] + fx * (c[7] - c[6]);
      const float y0 = x00 + fy * (x10 - x00), y1 = x01 + fy * (x11 - x01);
      const float dqx = ((1.f - fy) * (1.f - fz)) * (c[1] - c[0]) + (fy * (1.f - fz)) * (c[3] - c[2]) +
                        ((1.f - fy) * fz) * (c[5] - c[4]) + (fy * fz) * (c[7] - c[6]);
      const float dqy = (1.f - fz) * (x10 - x00) + fz * (x11 - x01);
      const float dqz = y1 - y0;
      // (cells clamped to the volume's padding hold zeros: no weight, no gradient)
      const float gy[3] = {w * invL * g_xs[0] + gw * dqx * a.m.mscale[0],
                           w * invL * g_xs[1] + gw * dqy * a.m.mscale[1],
                           w * invL * g_xs[2] + gw * dqz * a.m.mscale[2]};
      const float xh[4] = {x[0], x[1], x[2], 1.f};
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float s = wave_sum(live ? gy[r] * xh[k] : 0.f);
          if (lane == 0) atomicAdd(dg + b * 12 + r * 4 + k, s);
        }
    }
    const CellRuns cr = cell_runs(live, t.i0[0], t.i0[1], t.i0[2]);
    run_sums<8>(cr, v);
    if (wr.records) {
      const int x0 = t.i0[0];
#pragma unroll
      for (int q = 0; q < 4; ++q) {  // pair q: corners 2q (x0) and 2q + 1 (x0 + 1) at y0 + (q & 1), z0 + (q >> 1)
        const bool in = live && cr.owner && wc_pair_inside(t, R, q);
        const uint64_t m = __ballot(in);
        if (in) {
          const uint32_t idx = wc_off + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
          const uint32_t row =
              a.rec.wc_key0 + (uint32_t)b * (uint32_t)plane + ((uint32_t)(t.i0[2] + (q >> 1)) * R + t.i0[1] + (q & 1)) * R;
          // x0 = -1: only the x0 + 1 corner is inside; x0 = R - 1: only x0
          const uint32_t key = x0 >= 0 ? row + (uint32_t)x0 : row;
          const f2 val = x0 >= 0 ? f2{v[2 * q], x0 + 1 < R ? v[2 * q + 1] : 0.f} : f2{v[2 * q + 1], 0.f};
          if (idx < wr.end) {
            a.rec.keys[idx] = key;
            a.rec.vals[idx] = val;
          }
          wc_mb = max(wc_mb, max(__float_as_uint(fabsf(val[0])), __float_as_uint(fabsf(val[1]))));
        }
        wc_off += (uint32_t)__popcll(m);
      }
    } else if (live && cr.owner) {
      float* gplane = a.grad_weights + b * plane;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int ix = t.i0[0] + (k & 1), iy = t.i0[1] + ((k >> 1) & 1), iz = t.i0[2] + (k >> 2);
        if ((unsigned)ix < (unsigned)R && (unsigned)iy < (unsigned)R && (unsigned)iz < (unsigned)R)
          unsafeAtomicAdd(gplane + ((size_t)iz * R + iy) * R + ix, v[k]);
      }
    }
  }
}

// Compositing adjoint (Eq. 3 with alpha' = alpha min(L, 1)) of one
// 64-sample chunk of a ray, lane i holding sample i: raw outputs o (three
// colour logits, density), weight sum L and liveness.  With
// S_i = alpha'_i c_i + (1 - alpha'_i) S_{i+1} (the opacity channel uses
// c = 1), dC/dc_i = T_i alpha'_i and dC/dalpha'_i = T_i (c_i - S_{i+1}):
// S_{i+1} comes from a reverse affine scan across the wave (division-free),
// T_i from the chunk-start transmittance T0 and a forward prefix product.
// Sc holds S after the chunk's last sample on entry and S at its first
// sample on return.  g_o: dL/do (zero for lanes that are not live); g_L:
// dL/dL through the likelihood factor.
__device__ __forceinline__ void composite_adjoint(float T0, float delta, const f4& out, float L, bool live,
                                                  const f4& gout, float (&Sc)[4], float (&g_o)[4], float& g_L) {
  const int lane = lane_id();
  const float sigma = fmaxf(out[3], 0.f);
  const float alpha = -expm1f(-sigma * delta);
  const float mL = fminf(L, 1.f);
  const float ap = live ? alpha * mL : 0.f;
  float c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) c[k] = 1.f / (1.f + expf(-out[k]));
  const float incl = wave_prefix_prod(1.f - ap);
  float excl = shfl_up(incl, 1);
  if (lane == 0) excl = 1.f;
  const float Ti = T0 * excl;
  // reverse affine scan: S_i = b_i + a_i S_{i+1}
  float A_ = 1.f - ap;
  float Bv[4] = {ap * c[0], ap * c[1], ap * c[2], ap};
#pragma unroll
  for (int k = 1; k < WAVE; k <<= 1) {
    const float Ak = shfl_down(A_, k);
    float Bk[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) Bk[q] = shfl_down(Bv[q], k);
    if (lane + k < WAVE) {
#pragma unroll
      for (int q = 0; q < 4; ++q) Bv[q] = fmaf(A_, Bk[q], Bv[q]);
      A_ *= Ak;
    }
  }
  float Si[4], Snext[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) Si[q] = fmaf(A_, Sc[q], Bv[q]);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    Snext[q] = shfl_down(Si[q], 1);
    if (lane == WAVE - 1) Snext[q] = Sc[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) Sc[q] = __shfl(Si[q], 0, WAVE);
  float g_ap = gout[3] * Ti * (1.f - Snext[3]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g_ap += gout[k] * Ti * (c[k] - Snext[k]);
    g_o[k] = gout[k] * Ti * ap * c[k] * (1.f - c[k]);
  }
  const float g_sigma = g_ap * mL * delta * (1.f - alpha);
  g_o[3] = out[3] > 0.f ? g_sigma : 0.f;
  g_L = (L < 1.f) ? g_ap * alpha : 0.f;
  if (!live) g_o[0] = g_o[1] = g_o[2] = g_o[3] = 0.f;
}

// Ray slot r of a split-adjoint kernel: waves take slots in turn.
__device__ __forceinline__ bool split_ray(const RenderArgs& a, int slot, int& orow, RaySetup& rs, int& n_done,
                                          int nchunks) {
  const int row = ray_row(a.r, slot);
  const int pix = ray_pixel(a.r, row);
  if (!a.r.pixel_ids && pix < 0) return false;
  orow = a.r.pixel_ids ? row : pix;
  if (!(pix >= 0 && pix < a.r.H * a.r.W && setup_ray(a.r, pix, rs))) return false;
  n_done = (int)a.t_chunks[(size_t)orow * (nchunks + 1) + nchunks];
  return true;
}

// ---- BF16 MLP adjoint helpers of the split kernels ---------------------------

constexpr int RES_TB_BYTES = 2 * 64 * 16 * 2;  // a wave's transpose buffer (2 x 64 x 16 bf16)

// Stage W^T of a layer W [M][K] (BF16 fragments) as the A operand of
// dX = W^T dY, its output dimension padded to Kpad.
template <typename WT>
__device__ void stage_t(char* lds, const WT* __restrict__ w, int M, int K, int Kpad) {
  for (int e = threadIdx.x; e < K * Kpad; e += blockDim.x) {
    const int m = e / Kpad, k = e - m * Kpad;  // element (m, k) of W^T = W[k][m]
    const float v = (k < M) ? (float)w[(size_t)k * K + m] : 0.0f;
    *(__bf16*)(lds + frag_offset<MNR_BF16>(m, k, Kpad / 32)) = (__bf16)v;
  }
}

__device__ __forceinline__ f4 relu_mask4(f4 d, f4 h) {
  return f4{h[0] > 0.f ? d[0] : 0.f, h[1] > 0.f ? d[1] : 0.f, h[2] > 0.f ? d[2] : 0.f, h[3] > 0.f ? d[3] : 0.f};
}

// Weight-gradient products of one 16-sample tile, dW += d h^T: MT 16-row
// tiles of d (the wave's rows) times NT tiles of h, both transposed through
// the wave's buffer tb (2 x 64 x 16 bf16) into MFMA operands (K = the
// tile's samples), added to MFMA accumulators acc[mt][KT0 + kt] (16 x 16
// blocks, D layout: lane c + 16 g holds rows 16 mt + 4 g + j of column
// 16 (KT0 + kt) + c).  The accumulators stay in registers over all of a
// block's tiles and reach LDS once, at the kernel's end (add_dw): LDS float
// atomics on this GPU cost far more than the products, and even plain
// read-add-write per tile costs more than keeping the sums in registers.
template <int MT, int NT, int KT0 = 0, int NTA>
__device__ __forceinline__ void dw_acc(__bf16* tb, const f4* d, const f4* h, f4 (&acc)[MT][NTA], int lane) {
  static_assert(MT <= 4 && NT <= 4 && KT0 + NT <= NTA, "tile counts");
  __bf16* td = tb;            // [16 MT rows][16 samples]
  __bf16* th = tb + 64 * 16;  // [16 NT columns][16 samples]
  const int c = lane & 15, g = lane >> 4;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) td[(16 * t + 4 * g + j) * 16 + c] = (__bf16)d[t][j];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) th[(16 * t + 4 * g + j) * 16 + c] = (__bf16)h[t][j];
  wave_sync_lds();
  bf16x8 bv[NT];
#pragma unroll
  for (int kt = 0; kt < NT; ++kt) {
    if (g < 2) {
      bv[kt] = *(const bf16x8*)(th + (16 * kt + c) * 16 + 8 * g);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) bv[kt][e] = (__bf16)0.0f;
    }
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    bf16x8 av;
    if (g < 2) {
      av = *(const bf16x8*)(td + (16 * mt + c) * 16 + 8 * g);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) av[e] = (__bf16)0.0f;
    }
#pragma unroll
    for (int kt = 0; kt < NT; ++kt)
      acc[mt][KT0 + kt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[kt], acc[mt][KT0 + kt], 0, 0, 0);
  }
  wave_sync_lds();
}

// The wave's accumulated rows (the first `rows` of its 16 MT) added into the
// block's LDS sums (row stride ld); the caller keeps two waves from adding
// to the same rows at once.
template <int MT, int NT>
__device__ __forceinline__ void add_dw(const f4 (&acc)[MT][NT], float* dw, int rows, int ld, int lane) {
  const int c = lane & 15, g = lane >> 4;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int kt = 0; kt < NT; ++kt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 16 * mt + 4 * g + j;
        if (row < rows) dw[row * ld + 16 * kt + c] += acc[mt][kt][j];
      }
}

// out[mt] = W^T-fragments (MT m-tiles, KS 32-wide k steps) x x (2 KS tiles).
template <int MT, int KS>
__device__ __forceinline__ void mm_t(const char* wl, const f4* x, f4* out, int lane) {
  const bf16x8* W = (const bf16x8*)wl;
  bf16x8 b[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) b[s] = pack_bf16(x[2 * s], x[2 * s + 1]);
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[(mt * KS + s) * 64 + lane], b[s], acc, 0, 0, 0);
    out[mt] = acc;
  }
}

}  // namespace mnr
