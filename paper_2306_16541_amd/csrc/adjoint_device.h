// Device helpers of the adjoint kernels (training, Sec. 5.2): segmented
// run sums that cut the number of gradient atomics, and the skinning
// adjoint of one sample per lane (Eq. 7 and 9), shared by the fused adjoint
// and the split one used with the residual motion network.
#pragma once
#include "field_device.h"

namespace mnr {

// Gradient scatter with fewer atomics.  The 64 lanes of a wave are 64
// consecutive samples of one ray, so at coarse grid levels (and in the
// blend-weight volume) neighbouring lanes often fall in the same cell and
// would add to the same addresses.  Such runs are summed across the wave
// first and only the first lane of a run issues the atomics.  Global float
// atomics are executed at the memory side on this GPU (its eight L2s are
// not coherent with each other), so their count bounds the adjoint.
struct CellRuns {
  int seg;    // run index of the lane (number of run starts at lanes <= lane)
  int steps;  // suffix-scan steps needed to sum the longest run
  bool head;  // first lane of its run
};

__device__ __forceinline__ CellRuns cell_runs(bool live, int x, int y, int z) {
  const int lane = lane_id();
  const int px = __shfl_up(x, 1, WAVE), py = __shfl_up(y, 1, WAVE), pz = __shfl_up(z, 1, WAVE);
  const int plive = __shfl_up(live ? 1 : 0, 1, WAVE);
  CellRuns r;
  r.head = !live || lane == 0 || !plive || px != x || py != y || pz != z;
  const uint64_t heads = __ballot(r.head);
  r.seg = (int)__popcll(heads & (~0ull >> (63 - lane)));
  // Longest run: a run of length >= 2^j + 1 needs 2^j non-start lanes in a
  // row after its start; count the doublings (bits past lane 63 are starts).
  uint64_t z0 = ~heads;
  int steps = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    if (z0 == 0) break;
    ++steps;
    z0 &= z0 >> (1 << j);
  }
  r.steps = steps;
  return r;
}

// In-run suffix sums: afterwards the first lane of every run holds the sum
// of the run's values (segmented Hillis-Steele scan over the wave).
template <int NV>
__device__ __forceinline__ void run_sums(const CellRuns& r, float (&v)[NV]) {
  const int lane = lane_id();
#pragma unroll 1
  for (int j = 0; j < r.steps; ++j) {
    const int d = 1 << j;
    const int seg_d = __shfl_down(r.seg, d, WAVE);
    const bool same = lane + d < WAVE && seg_d == r.seg;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const float o = __shfl_down(v[k], d, WAVE);
      v[k] += same ? o : 0.f;
    }
  }
}

// Skinning adjoint (Eq. 7, 9) of one sample per lane.  x: observed point,
// xs: x_skel, L: the weight sum, g_xs: dL/dx_skel, g_L: dL/dL (the
// likelihood factor alpha' = alpha min(L, 1)).  Per bone i:
// dL/dw_i = dL/dx_skel . (y_i - x_skel) / L + dL/dL, scattered through the
// trilinear weights into dL/dW^c (runs of lanes in one cell summed first);
// optionally dL/dG_i into the block's LDS sums dg[n_bones][12].  Every lane
// of the wave takes part (the run detection shuffles across it); lanes that
// are not live contribute nothing.
__device__ __forceinline__ void skin_adjoint(const RenderArgs& a, const float x[3], const float xs[3], float L,
                                             const float g_xs[3], float g_L, bool live, float* dg) {
  const int lane = lane_id();
  const int R = a.m.res;
  const size_t plane = (size_t)R * R * R;
  const bool above = L > EPS_L;
  const float invL = 1.f / (above ? L : EPS_L);
  const float gL = live ? g_L : 0.f;
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
    if (live && cr.head) {
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

}  // namespace mnr
