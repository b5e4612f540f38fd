// Per-sample stages of the posed-body renderer, as device functions shared by
// the forward and adjoint kernels:
//   warp_sample   inverse linear blend skinning (Sec. 4.2, Eq. 7-9)
//   encode_all    the multiresolution grid encoding of the canonical
//                 field's input (Sec. 4.4, Eq. 13)
//   stage_weights / mlp_tile  the bias-free MLP of Eq. 13 on MFMA
#pragma once
#include <utility>
#include "device_common.h"

namespace mnr {

// ---------------------------------------------------------------------------
// Inverse LBS: y_i = G_i x, w_i = trilinear(W^c_i, y_i) (zero outside the
// volume), L = sum_i w_i, x_skel = sum_i w_i y_i / max(L, eps).
// ---------------------------------------------------------------------------

struct Tri {  // trilinear cell of one point in a zero-padded volume
  int i0[3];
  float f[3];
};

__device__ __forceinline__ Tri tri_cell(float qx, float qy, float qz) {
  Tri t;
  const float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
  t.i0[0] = (int)fx; t.i0[1] = (int)fy; t.i0[2] = (int)fz;
  t.f[0] = qx - fx; t.f[1] = qy - fy; t.f[2] = qz - fz;
  return t;
}

// Raw buffer resources (gfx9 family: dword3 = 0x00020000, stride 0).  A
// read whose byte offset is >= num_records returns 0; OOB_OFFSET is used
// for trilinear corners that lie outside the volume, which gives the
// zero padding without a branch.
constexpr uint32_t OOB_OFFSET = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// Byte offsets of the 8 corners of a trilinear cell in an R^3 plane; corners
// outside [0, R-1]^3 get OOB_OFFSET.
__device__ __forceinline__ void tri_offsets(const Tri& t, int R, uint32_t off[8]) {
  const bool okx0 = (unsigned)t.i0[0] < (unsigned)R, okx1 = (unsigned)(t.i0[0] + 1) < (unsigned)R;
  const bool oky0 = (unsigned)t.i0[1] < (unsigned)R, oky1 = (unsigned)(t.i0[1] + 1) < (unsigned)R;
  const bool okz0 = (unsigned)t.i0[2] < (unsigned)R, okz1 = (unsigned)(t.i0[2] + 1) < (unsigned)R;
  const uint32_t base = (((uint32_t)t.i0[2] * R + (uint32_t)t.i0[1]) * R + (uint32_t)t.i0[0]) * 4u;
  const uint32_t sy = (uint32_t)R * 4u, sz = (uint32_t)(R * R) * 4u;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const bool ok = ((c & 1) ? okx1 : okx0) && ((c & 2) ? oky1 : oky0) && ((c & 4) ? okz1 : okz0);
    const uint32_t o = base + ((c & 1) ? 4u : 0u) + ((c & 2) ? sy : 0u) + ((c & 4) ? sz : 0u);
    off[c] = ok ? o : OOB_OFFSET;
  }
}

__device__ __forceinline__ float trilerp(const float v[8], const float f[3]) {
  const float x00 = __builtin_fmaf(f[0], v[1] - v[0], v[0]), x10 = __builtin_fmaf(f[0], v[3] - v[2], v[2]);
  const float x01 = __builtin_fmaf(f[0], v[5] - v[4], v[4]), x11 = __builtin_fmaf(f[0], v[7] - v[6], v[6]);
  const float y0 = __builtin_fmaf(f[1], x10 - x00, x00), y1 = __builtin_fmaf(f[1], x11 - x01, x01);
  return __builtin_fmaf(f[2], y1 - y0, y0);
}

__device__ __forceinline__ void bone_apply(const float* __restrict__ g, const float x[3], float y[3]) {
  y[0] = fmaf(g[0], x[0], fmaf(g[1], x[1], fmaf(g[2], x[2], g[3])));
  y[1] = fmaf(g[4], x[0], fmaf(g[5], x[1], fmaf(g[6], x[2], g[7])));
  y[2] = fmaf(g[8], x[0], fmaf(g[9], x[1], fmaf(g[10], x[2], g[11])));
}

// Cell of a canonical point in the weight volume.  Grid coordinates are
// clamped to [-2, R+1] first (every corner of such a cell is outside the
// volume anyway), so the float-to-int conversion is always in range.
__device__ __forceinline__ Tri bone_cell(const MotionArgs& m, const float y[3]) {
  const float hi = (float)(m.res + 1);
  return tri_cell(fminf(fmaxf((y[0] - m.mmin[0]) * m.mscale[0], -2.f), hi),
                  fminf(fmaxf((y[1] - m.mmin[1]) * m.mscale[1], -2.f), hi),
                  fminf(fmaxf((y[2] - m.mmin[2]) * m.mscale[2], -2.f), hi));
}

// The 8 corner weights of bone b's trilinear cell, corner c at
// (x0 + (c&1), y0 + (c>>1 & 1), z0 + (c>>2)).  Plain volume: eight 4-byte
// gathers.  Packed copy (float4 of the 2x2 x-y corners at [b][z][y0+1][x0+1]):
// two 16-byte loads, planes z0 and z0+1.  Corners outside the volume read 0
// through out-of-range offsets in both layouts, so the values are identical.
__device__ __forceinline__ void bone_corners(const MotionArgs& m, int b, const Tri& t, float v[8]) {
  const int R = m.res;
  if (m.packed) {
    const uint32_t R1 = (uint32_t)R + 1u, zstride = R1 * R1 * 16u;
    const uint32_t cx = (uint32_t)(t.i0[0] + 1), cy = (uint32_t)(t.i0[1] + 1), z = (uint32_t)t.i0[2];
    const bool okxy = cx <= (uint32_t)R && cy <= (uint32_t)R;
    const uint32_t o = ((z * R1 + cy) * R1 + cx) * 16u;  // modulo 2^32; only used when z or z+1 is in range
    const uint32_t o0 = (okxy && z < (uint32_t)R) ? o : OOB_OFFSET;
    const uint32_t o1 = (okxy && z + 1u < (uint32_t)R) ? o + zstride : OOB_OFFSET;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(m.packed + (size_t)b * R * R1 * R1, (uint32_t)R * zstride);
    const f4 lo = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, o0, 0, 0));
    const f4 hi = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, o1, 0, 0));
#pragma unroll
    for (int c = 0; c < 4; ++c) { v[c] = lo[c]; v[4 + c] = hi[c]; }
  } else {
    const uint32_t plane = (uint32_t)(R * R * R);
    uint32_t off[8];
    tri_offsets(t, R, off);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(m.weights + (size_t)b * plane, plane * 4u);
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off[c], 0, 0));
  }
}

// Bones are processed BG at a time so that all their corner loads are in
// flight before the first one is consumed.
constexpr int BG = 4;

// The layout test is a uniform branch per bone rather than two copies of
// this loop: with two loops the compiler copied the kernel's argument block
// to scratch memory.
__device__ __forceinline__ void warp_sample(const MotionArgs& m, const float (*G)[12], const float x[3], float xs[3],
                                            float& L) {
  float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, sum = 0.f;
#pragma unroll 1
  for (int b0 = 0; b0 < m.n_bones; b0 += BG) {
    float v[BG][8], y[BG][3];
    Tri t[BG];
#pragma unroll
    for (int u = 0; u < BG; ++u) {
      const int b = b0 + u < m.n_bones ? b0 + u : m.n_bones - 1;
      bone_apply(G[b], x, y[u]);
      t[u] = bone_cell(m, y[u]);
      bone_corners(m, b, t[u], v[u]);
    }
#pragma unroll
    for (int u = 0; u < BG; ++u) {
      if (b0 + u < m.n_bones) {
        const float w = trilerp(v[u], t[u].f);
        sum += w;
        acc0 = fmaf(w, y[u][0], acc0);
        acc1 = fmaf(w, y[u][1], acc1);
        acc2 = fmaf(w, y[u][2], acc2);
      }
    }
  }
  L = sum;
  const float inv = 1.0f / fmaxf(sum, EPS_L);
  xs[0] = acc0 * inv; xs[1] = acc1 * inv; xs[2] = acc2 * inv;
}

// ---------------------------------------------------------------------------
// Grid encoding of one level.
// ---------------------------------------------------------------------------

// One table row (n_feat = 2 features) through a per-level buffer resource.
template <typename TableT>
__device__ __forceinline__ f2 load_row(__amdgpu_buffer_rsrc_t rs, uint32_t row);
template <>
__device__ __forceinline__ f2 load_row<float>(__amdgpu_buffer_rsrc_t rs, uint32_t row) {
  return __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(rs, row * 8u, 0, 0));
}
template <>
__device__ __forceinline__ f2 load_row<_Float16>(__amdgpu_buffer_rsrc_t rs, uint32_t row) {
  const h2 v = __builtin_bit_cast(h2, __builtin_amdgcn_raw_buffer_load_b32(rs, row * 4u, 0, 0));
  return f2{(float)v[0], (float)v[1]};
}

template <typename TableT>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t level_rsrc(const FieldArgs& f, int l) {
  const uint32_t T = 1u << f.log2_T;
  return make_rsrc((const TableT*)f.table + (size_t)l * T * 2, T * 2u * (uint32_t)sizeof(TableT));
}

// Cell of point u (in [0,1]^3) at resolution N: i0 = min(floor(uN), N-1).
struct GridCell {
  int i0[3];
  float f[3];
};

__device__ __forceinline__ GridCell grid_cell(const float u[3], int N) {
  // p is rounded before the fractional part is taken: left to itself the
  // compiler fuses u*N - floor(p) into an FMA at some call sites only.
#pragma clang fp contract(off)
  GridCell c;
  const float Nf = (float)N;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float p = u[a] * Nf;
    const float fl = fminf(floorf(p), Nf - 1.0f);
    c.i0[a] = (int)fl;
    c.f[a] = p - fl;
  }
  return c;
}

// Row of corner (dx,dy,dz) of the cell, dense or spatially hashed.
__device__ __forceinline__ uint32_t grid_row(const GridCell& c, int N, bool dense, uint32_t mask, int k) {
  const uint32_t x = c.i0[0] + (k & 1), y = c.i0[1] + ((k >> 1) & 1), z = c.i0[2] + (k >> 2);
  if (dense) {
    const uint32_t s = (uint32_t)N + 1u;
    return x + s * (y + s * z);
  }
  return (x * 1u ^ y * 2654435761u ^ z * 805459861u) & mask;
}

// Explicit fused multiply-adds: the result must not depend on which code
// path (gathered rows or packed groups) supplied the corners.
__device__ __forceinline__ float lerp1(float a, float b, float t) { return __builtin_fmaf(t, b - a, a); }

__device__ __forceinline__ f2 trilerp2(const f2 v[8], const float f[3]) {
  f2 r;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const float x00 = lerp1(v[0][c], v[1][c], f[0]), x10 = lerp1(v[2][c], v[3][c], f[0]);
    const float x01 = lerp1(v[4][c], v[5][c], f[0]), x11 = lerp1(v[6][c], v[7][c], f[0]);
    r[c] = lerp1(lerp1(x00, x10, f[1]), lerp1(x01, x11, f[1]), f[2]);
  }
  return r;
}

// The 8 corner rows of a dense level's cell from the packed copy: groups of
// the 4 x-y corners (2 features each) at [z][y0][x0], planes z0 and z0+1,
// corner k at (x0 + (k&1), y0 + (k>>1 & 1), z0 + (k>>2)) as in grid_row.
template <typename TableT>
__device__ __forceinline__ void load_cell_packed(const FieldArgs& f, int l, const GridCell& c, int N, f2 v[8]) {
  constexpr uint32_t EB = 8u * sizeof(TableT);  // bytes of one group
  const uint32_t n = (uint32_t)N, zs = n * n * EB;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(f.dpk + f.dpk_off[l], (n + 1u) * zs);
  const uint32_t o = (((uint32_t)c.i0[2] * n + (uint32_t)c.i0[1]) * n + (uint32_t)c.i0[0]) * EB;
  if constexpr (sizeof(TableT) == 2) {
    typedef _Float16 h8 __attribute__((ext_vector_type(8)));
    const h8 lo = __builtin_bit_cast(h8, __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 0));
    const h8 hi = __builtin_bit_cast(h8, __builtin_amdgcn_raw_buffer_load_b128(rs, o + zs, 0, 0));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = f2{(float)lo[2 * k], (float)lo[2 * k + 1]};
      v[4 + k] = f2{(float)hi[2 * k], (float)hi[2 * k + 1]};
    }
  } else {
    const f4 a = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 0));
    const f4 b = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, o + 16u, 0, 0));
    const f4 d = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, o + zs, 0, 0));
    const f4 e = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, o + zs + 16u, 0, 0));
    v[0] = f2{a[0], a[1]}; v[1] = f2{a[2], a[3]}; v[2] = f2{b[0], b[1]}; v[3] = f2{b[2], b[3]};
    v[4] = f2{d[0], d[1]}; v[5] = f2{d[2], d[3]}; v[6] = f2{e[0], e[1]}; v[7] = f2{e[2], e[3]};
  }
}

// Levels are encoded in groups whose loads are all in flight before the
// first is consumed: the leading dense levels from the packed copy (when
// present) PG at a time, then the remaining levels' row gathers LG at a
// time.  Calls store(l, feature pair) for every level.
constexpr int LG = 4;
template <typename TableT>
constexpr int packed_group() { return sizeof(TableT) == 2 ? 4 : 2; }  // 32 VGPRs of loads either way

template <typename TableT, typename Store>
__device__ __forceinline__ void encode_all(const FieldArgs& f, const float u[3], bool live, Store store) {
  constexpr int PG = packed_group<TableT>();
  const uint32_t mask = (1u << f.log2_T) - 1u;
#pragma unroll 1
  for (int l0 = 0; l0 < f.n_packed; l0 += PG) {
    f2 v[PG][8];
    GridCell c[PG];
#pragma unroll
    for (int q = 0; q < PG; ++q) {
      const int l = l0 + q;
      if (l < f.n_packed) {  // uniform
        const int N = f.level_res[l];
        c[q] = grid_cell(u, N);
        if (live) load_cell_packed<TableT>(f, l, c[q], N, v[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < PG; ++q)
      if (l0 + q < f.n_packed) store(l0 + q, live ? trilerp2(v[q], c[q].f) : f2{0.f, 0.f});
  }
#pragma unroll 1
  for (int l0 = f.n_packed; l0 < f.n_levels; l0 += LG) {
    f2 v[LG][8];
    GridCell c[LG];
#pragma unroll
    for (int q = 0; q < LG; ++q) {
      const int l = l0 + q;
      if (l < f.n_levels) {  // uniform
        const int N = f.level_res[l];
        const bool dense = (f.dense_mask >> l) & 1u;
        c[q] = grid_cell(u, N);
        const __amdgpu_buffer_rsrc_t rs = level_rsrc<TableT>(f, l);
        if (live) {  // one exec-masked region: dead lanes issue no gathers
#pragma unroll
          for (int k = 0; k < 8; ++k) v[q][k] = load_row<TableT>(rs, grid_row(c[q], N, dense, mask, k));
        }
      }
    }
#pragma unroll
    for (int q = 0; q < LG; ++q)
      if (l0 + q < f.n_levels) store(l0 + q, live ? trilerp2(v[q], c[q].f) : f2{0.f, 0.f});
  }
}

__device__ __forceinline__ void unit_coords(const FieldArgs& f, const float xs[3], float u[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = fminf(fmaxf((xs[a] - f.gmin[a]) * f.gscale[a], 0.0f), 1.0f);
}

// ---------------------------------------------------------------------------
// MLP on MFMA.
//
// LDS weight layout, per layer: fragments [mt][kg][lane] of 16 bytes.
//   F32 : kg = 16-input tile t; element j = input 16t + 4g + j (g = lane/16)
//   BF16: kg = 32-input step s; element e = input 16(2s + e/4) + 4g + e%4
// Row m of the fragment is output 16mt + lane%16; the output layer is padded
// to 16 rows with zeros.
// Per-wave feature layout (B operand of layer 1), F32: [nt][t][lane] x 4
// floats; BF16: [nt][lane] x 8 bf16; sample = 16nt + lane%16, same K order.
// ---------------------------------------------------------------------------

template <int P>
struct MlpShape {
  static constexpr int KG_IN = (P == MNR_F32) ? IN_FEAT / 16 : IN_FEAT / 32;
  static constexpr int KG_HID = (P == MNR_F32) ? HIDDEN / 16 : HIDDEN / 32;
  static constexpr int FRAG = 64 * 16;  // bytes per fragment
  static constexpr int bytes_first() { return 4 * KG_IN * FRAG; }
  static constexpr int bytes_hidden() { return 4 * KG_HID * FRAG; }
  static constexpr int bytes_out() { return KG_HID * FRAG; }
  static constexpr int bytes_total(int nhh) { return bytes_first() + nhh * bytes_hidden() + bytes_out(); }
  static constexpr int feat_bytes_per_wave() { return 64 * IN_FEAT * (P == MNR_F32 ? 4 : 2); }
};

// Position of weight (m, k) of a layer inside its fragments.
template <int P>
__device__ __forceinline__ int frag_offset(int m, int k, int kgroups) {
  const int mt = m >> 4, t = k >> 4, g = (k & 15) >> 2, j = k & 3;
  const int lane = (m & 15) + 16 * g;
  if (P == MNR_F32) return (((mt * kgroups + t) * 64 + lane) * 4 + j) * 4;                 // bytes
  return (((mt * kgroups + (t >> 1)) * 64 + lane) * 8 + (t & 1) * 4 + j) * 2;              // bytes
}

template <int P, typename WT>
__device__ void stage_layer(char* lds, const WT* __restrict__ w, int M, int K, int Mpad) {
  const int kg = (P == MNR_F32) ? K / 16 : K / 32;
  for (int e = threadIdx.x; e < Mpad * K; e += blockDim.x) {
    const int m = e / K, k = e - m * K;
    const float v = (m < M) ? (float)w[(size_t)m * K + k] : 0.0f;
    if (P == MNR_F32)
      *(float*)(lds + frag_offset<P>(m, k, kg)) = v;
    else
      *(__bf16*)(lds + frag_offset<P>(m, k, kg)) = (__bf16)v;
  }
}

// Stage all layers: first (IN_FEAT -> 64), nhh x (64 -> 64), out (64 -> 4).
template <int P, int NHH>
__device__ void stage_weights(char* lds, const FieldArgs& f) {
  typedef typename std::conditional<P == MNR_F32, float, __bf16>::type WT;
  using S = MlpShape<P>;
  stage_layer<P>(lds, (const WT*)f.w[0], HIDDEN, IN_FEAT, HIDDEN);
  for (int l = 0; l < NHH; ++l)
    stage_layer<P>(lds + S::bytes_first() + l * S::bytes_hidden(), (const WT*)f.w[1 + l], HIDDEN, HIDDEN,
                   HIDDEN);
  stage_layer<P>(lds + S::bytes_first() + NHH * S::bytes_hidden(), (const WT*)f.w[1 + NHH], 4, HIDDEN, 16);
}

// Feature store (lane = sample s, features k, k+1 of the 32).
template <int P>
__device__ __forceinline__ void store_feat2(char* feat, int s, int k, f2 v) {
  const int nt = s >> 4, c = s & 15, t = k >> 4, g = (k & 15) >> 2, j = k & 3;
  const int lane = c + 16 * g;
  if (P == MNR_F32) {
    *(f2*)(feat + (((nt * 2 + t) * 64 + lane) * 4 + j) * 4) = v;
  } else {
    bf16x2 b = {(__bf16)v[0], (__bf16)v[1]};
    *(bf16x2*)(feat + ((nt * 64 + lane) * 8 + t * 4 + j) * 2) = b;
  }
}

// ReLU as a signed-integer max on the bit pattern: one instruction (fmaxf
// costs two on MFMA results, a canonicalisation and the max).  Equal to
// max(x, 0) for every non-NaN x, with -0 mapped to +0.
__device__ __forceinline__ float relu1(float x) {
  const int i = __builtin_bit_cast(int, x);
  return __builtin_bit_cast(float, i > 0 ? i : 0);
}

__device__ __forceinline__ f4 relu4(f4 v) { return f4{relu1(v[0]), relu1(v[1]), relu1(v[2]), relu1(v[3])}; }

__device__ __forceinline__ bf16x8 pack_bf16(f4 lo, f4 hi) {
  bf16x8 b;
  b[0] = (__bf16)lo[0]; b[1] = (__bf16)lo[1]; b[2] = (__bf16)lo[2]; b[3] = (__bf16)lo[3];
  b[4] = (__bf16)hi[0]; b[5] = (__bf16)hi[1]; b[6] = (__bf16)hi[2]; b[7] = (__bf16)hi[3];
  return b;
}

// BF16 layer on operands already packed: b[s] holds input rows 32 s ..
// 32 s + 31 of the lane's sample column (the layout of pack_bf16 over two
// F32 input tiles).
template <int MT, int KS>
__device__ __forceinline__ void mma_layer_bf16(const char* wl, const bf16x8 (&b)[KS], f4 (&out)[4], int lane,
                                               const float* bias = nullptr) {
  const bf16x8* W = (const bf16x8*)wl;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    f4 acc = bias ? *(const f4*)(bias + 16 * mt + 4 * (lane >> 4)) : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[(mt * KS + s) * 64 + lane], b[s], acc, 0, 0, 0);
    out[mt] = acc;
  }
}

// One dense layer: out[mt] = W x (+ bias), K = 16 * KT input tiles.  The
// optional bias (LDS floats, one per output row) initialises the
// accumulators: lane j + 16g, element e of tile mt is row 16 mt + 4 g + e.
template <int P, int MT, int KT, int NX>
__device__ __forceinline__ void mma_layer(const char* wl, const f4 (&x)[NX], f4 (&out)[4], int lane,
                                          const float* bias = nullptr) {
  static_assert(KT <= NX, "input tiles");
  auto acc0 = [&](int mt) {
    return bias ? *(const f4*)(bias + 16 * mt + 4 * (lane >> 4)) : f4{0.f, 0.f, 0.f, 0.f};
  };
  if constexpr (P == MNR_F32) {
    const f4* W = (const f4*)wl;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      f4 acc = acc0(mt);
#pragma unroll
      for (int t = 0; t < KT; ++t) {
        const f4 a = W[(mt * KT + t) * 64 + lane];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], x[t][j], acc, 0, 0, 0);
      }
      out[mt] = acc;
    }
  } else {
    constexpr int KS = KT / 2;
    bf16x8 b[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) b[s] = pack_bf16(x[2 * s], x[2 * s + 1]);
    mma_layer_bf16<MT, KS>(wl, b, out, lane, bias);
  }
}

// Layer-1 input of sample tile nt from the wave's feature buffer, as the
// activation registers x[t] (t = 0, 1) of the F32 layout.
template <int P>
__device__ __forceinline__ void load_input(const char* feat, int nt, int lane, f4 (&x)[4]) {
  if constexpr (P == MNR_F32) {
    x[0] = ((const f4*)feat)[(nt * 2 + 0) * 64 + lane];
    x[1] = ((const f4*)feat)[(nt * 2 + 1) * 64 + lane];
  } else {
    const bf16x8 b = ((const bf16x8*)feat)[nt * 64 + lane];
    x[0] = f4{(float)b[0], (float)b[1], (float)b[2], (float)b[3]};
    x[1] = f4{(float)b[4], (float)b[5], (float)b[6], (float)b[7]};
  }
  x[2] = x[3] = f4{0.f, 0.f, 0.f, 0.f};
}

// Whole MLP for the 16 samples of tile nt.  Returns the output fragment:
// lanes 0..15 hold (o0, o1, o2, o3) of sample 16nt + lane.  If `hidden` is
// non-null, the post-ReLU activations of every hidden layer are stored
// there ([layer][mt] fragments, for the adjoint).
template <int P, int NHH>
__device__ __forceinline__ f4 mlp_tile(const char* wl, const char* feat, int nt, int lane,
                                       f4 (*hidden)[4] = nullptr) {
  using S = MlpShape<P>;
  f4 h[4];
  if constexpr (P == MNR_BF16) {  // the stored features are already the packed B operand
    const bf16x8 b[1] = {((const bf16x8*)feat)[nt * 64 + lane]};
    mma_layer_bf16<4, 1>(wl, b, h, lane);
  } else {
    f4 x[4];
    load_input<P>(feat, nt, lane, x);
    mma_layer<P, 4, 2>(wl, x, h, lane);
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) h[mt] = relu4(h[mt]);
  if (hidden) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) hidden[0][mt] = h[mt];
  }
#pragma unroll
  for (int l = 0; l < NHH; ++l) {
    f4 nh[4];
    mma_layer<P, 4, 4>(wl + S::bytes_first() + l * S::bytes_hidden(), h, nh, lane);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) h[mt] = relu4(nh[mt]);
    if (hidden) {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) hidden[l + 1][mt] = h[mt];
    }
  }
  f4 o[4];
  mma_layer<P, 1, 4>(wl + S::bytes_first() + NHH * S::bytes_hidden(), h, o, lane);
  return o[0];
}

// ---------------------------------------------------------------------------
// Field evaluation of one sample per lane: inverse LBS, encoding (into the
// wave's LDS feature buffer) and the MLP.  Lanes with valid == false (or
// L == 0) are not live.  Returns the ballot of live lanes; when it is zero
// nothing else was computed.  On return lane i holds its sample's raw MLP
// outputs in `out` (the per-wave scratch `obuf`, 64 x f4, carries the lane
// transpose).  MLP tiles (16 lanes) without a live lane are skipped.
// ---------------------------------------------------------------------------

struct SampleState {
  float x[3], xs[3], L;
  bool live;
};

// Stratified offset of sample i of ray b: SplitMix64 output b*spp + i of the
// stream seeded with `seed`, top 24 bits as a fraction; 0.5 (stratum
// midpoint) when jitter is off.
__device__ __forceinline__ float sample_jitter(const RayArgs& r, int ray_index, int i) {
  if (!r.stratified) return 0.5f;
  return (float)(splitmix64(r.seed, (uint64_t)ray_index * r.spp + i) >> 40) * 0x1p-24f;
}

// ---------------------------------------------------------------------------
// Residual non-rigid motion (Sec. 4.3, Eq. 11-12) on BF16 MFMA: the same
// fragment layouts as the field's MLP.  LDS: W1 (64x32), W2, W3 (64x64),
// W4 (64x96: the skip connection appends gamma's two input tiles to h3's
// four), W5 (3 rows padded to 16), then the per-frame pose term W_omega
// Omega as 64 floats (the first layer's bias).
// ---------------------------------------------------------------------------

struct ResShape {
  static constexpr int FRAG = 64 * 16;
  static constexpr int W1 = 4 * 1 * FRAG, W2 = 4 * 2 * FRAG, W3 = 4 * 2 * FRAG, W4 = 4 * 3 * FRAG, W5 = 2 * FRAG;
  static constexpr int o2 = W1, o3 = o2 + W2, o4 = o3 + W3, o5 = o4 + W4, obias = o5 + W5;
  static constexpr int bytes() { return obias + 64 * 4; }
};

__device__ void stage_residual(char* lds, const ResArgs& r) {
  stage_layer<MNR_BF16>(lds, r.w[0], HIDDEN, 32, HIDDEN);
  stage_layer<MNR_BF16>(lds + ResShape::o2, r.w[1], HIDDEN, HIDDEN, HIDDEN);
  stage_layer<MNR_BF16>(lds + ResShape::o3, r.w[2], HIDDEN, HIDDEN, HIDDEN);
  stage_layer<MNR_BF16>(lds + ResShape::o4, r.w[3], HIDDEN, HIDDEN + 32, HIDDEN);
  stage_layer<MNR_BF16>(lds + ResShape::o5, r.w[4], 3, HIDDEN, 16);
  float* bias = (float*)(lds + ResShape::obias);
  for (int i = threadIdx.x; i < HIDDEN; i += blockDim.x) {
    float b = 0.f;
    for (int j = 0; j < r.n_omega; ++j) b = fmaf((float)r.w[5][i * r.n_omega + j], r.omega[j], b);
    bias[i] = b;
  }
}

// x_skel += x_res for the live lanes of the wave.  gamma goes through the
// wave's feature buffer (layer-1 input layout, read again by the skip
// layer); tile nt's outputs are carried back to their lanes through obuf.
__device__ __forceinline__ void residual_step(const ResArgs& r, const char* rl, char* feat, f4* obuf, SampleState& st,
                                              uint64_t live_mask, int lane) {
  float g[32];
#pragma unroll
  for (int c = 0; c < 3; ++c) g[c] = st.xs[c];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float sv, cv;
      sincospif((float)(1 << k) * st.xs[c], &sv, &cv);  // sin, cos of 2^k pi x_c
      g[3 + 6 * k + c] = r.win[k] * sv;
      g[6 + 6 * k + c] = r.win[k] * cv;
    }
  }
#pragma unroll
  for (int i = 27; i < 32; ++i) g[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i)
    store_feat2<MNR_BF16>(feat, lane, 2 * i, st.live ? f2{g[2 * i], g[2 * i + 1]} : f2{0.f, 0.f});
  wave_sync_lds();
  const float* bias = (const float*)(rl + ResShape::obias);
#pragma unroll 1
  for (int nt = 0; nt < 4; ++nt) {
    f4 o = {0.f, 0.f, 0.f, 0.f};
    if ((live_mask >> (16 * nt)) & 0xFFFFull) {
      f4 x[4], h[4], h2[4];
      load_input<MNR_BF16>(feat, nt, lane, x);
      mma_layer<MNR_BF16, 4, 2>(rl, x, h, lane, bias);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) h[mt] = relu4(h[mt]);
      mma_layer<MNR_BF16, 4, 4>(rl + ResShape::o2, h, h2, lane);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) h2[mt] = relu4(h2[mt]);
      mma_layer<MNR_BF16, 4, 4>(rl + ResShape::o3, h2, h, lane);
      const f4 cat[6] = {relu4(h[0]), relu4(h[1]), relu4(h[2]), relu4(h[3]), x[0], x[1]};
      mma_layer<MNR_BF16, 4, 6>(rl + ResShape::o4, cat, h2, lane);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) h2[mt] = relu4(h2[mt]);
      f4 oo[4];
      mma_layer<MNR_BF16, 1, 4>(rl + ResShape::o5, h2, oo, lane);
      o = oo[0];
    }
    wave_sync_lds();
    if (lane < 16) obuf[nt * 16 + lane] = o;
  }
  wave_sync_lds();
  const f4 d = obuf[lane];
  wave_sync_lds();
  if (st.live) {
    st.xs[0] += d[0];
    st.xs[1] += d[1];
    st.xs[2] += d[2];
  }
}

// ---------------------------------------------------------------------------
// The paper's own field (Sec. 4.4, Eq. 13, Fig. 9): 10-band positional
// encoding (64 values) and a 64-wide skip MLP on BF16 MFMA.  LDS: W1
// (64x64), W2, W3 (64x64), W4 (64x128: h3's four input tiles, then
// gamma's four), W5 (4 rows padded to 16).  gamma lives in the wave's
// feature buffer as two 32-feature halves in the layer-1 input layout.
// ---------------------------------------------------------------------------

struct FreqShape {
  static constexpr int FRAG = 64 * 16;
  static constexpr int W1 = 4 * 2 * FRAG, W2 = 4 * 2 * FRAG, W3 = 4 * 2 * FRAG, W4 = 4 * 4 * FRAG, W5 = 2 * FRAG;
  static constexpr int o2 = W1, o3 = o2 + W2, o4 = o3 + W3, o5 = o4 + W4;
  static constexpr int bytes() { return o5 + W5; }
  static constexpr int feat_bytes_per_wave() { return 64 * 64 * 2; }
};

__device__ void stage_freq(char* lds, const FieldArgs& f) {
  stage_layer<MNR_BF16>(lds, (const __bf16*)f.w[0], HIDDEN, 64, HIDDEN);
  stage_layer<MNR_BF16>(lds + FreqShape::o2, (const __bf16*)f.w[1], HIDDEN, HIDDEN, HIDDEN);
  stage_layer<MNR_BF16>(lds + FreqShape::o3, (const __bf16*)f.w[2], HIDDEN, HIDDEN, HIDDEN);
  stage_layer<MNR_BF16>(lds + FreqShape::o4, (const __bf16*)f.w[3], HIDDEN, 2 * HIDDEN, HIDDEN);
  stage_layer<MNR_BF16>(lds + FreqShape::o5, (const __bf16*)f.w[4], 4, HIDDEN, 16);
}

// gamma(x) of the lane's sample into the feature buffer (zeros for lanes
// that are not live); value k goes to half k / 32, feature k % 32.
__device__ __forceinline__ void store_posenc10(char* feat, int lane, const float x[3], bool live) {
  float prev = 0.f;
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    float v;
    if (k < 3) {
      v = x[k];
    } else if (k < 63) {
      const int band = (k - 3) / 6, r = (k - 3) % 6, c = r % 3;
      float sv, cv;
      sincospif((float)(1 << band) * x[c], &sv, &cv);
      v = r < 3 ? sv : cv;
    } else {
      v = 0.f;
    }
    if (k & 1) store_feat2<MNR_BF16>(feat + (k >> 5) * 4096, lane, (k - 1) & 31, live ? f2{prev, v} : f2{0.f, 0.f});
    prev = v;
  }
}

// Hidden activation h (four D-layout tiles) of layer `layer`, tile nt, as
// the BF16 operands the next layer consumes, into a chunk's save area.
__device__ __forceinline__ void save_act(bf16x8* save, int layer, int nt, int lane, const f4* h) {
  save[(layer * 4 + nt) * 128 + lane] = pack_bf16(h[0], h[1]);
  save[(layer * 4 + nt) * 128 + 64 + lane] = pack_bf16(h[2], h[3]);
}

// Raw outputs (o0..o3) of the 16 samples of tile nt, lanes 0..15.  SAVE:
// also store the four hidden activations for the adjoint.
template <bool SAVE = false>
__device__ __forceinline__ f4 freq_tile(const char* wl, const char* feat, int nt, int lane, bf16x8* save = nullptr) {
  f4 xa[4], xb[4], h[4], h2[4];
  load_input<MNR_BF16>(feat, nt, lane, xa);
  load_input<MNR_BF16>(feat + 4096, nt, lane, xb);
  const f4 g[4] = {xa[0], xa[1], xb[0], xb[1]};
  mma_layer<MNR_BF16, 4, 4>(wl, g, h, lane);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) h[mt] = relu4(h[mt]);
  if constexpr (SAVE) save_act(save, 0, nt, lane, h);
  mma_layer<MNR_BF16, 4, 4>(wl + FreqShape::o2, h, h2, lane);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) h2[mt] = relu4(h2[mt]);
  if constexpr (SAVE) save_act(save, 1, nt, lane, h2);
  mma_layer<MNR_BF16, 4, 4>(wl + FreqShape::o3, h2, h, lane);
  const f4 cat[8] = {relu4(h[0]), relu4(h[1]), relu4(h[2]), relu4(h[3]), g[0], g[1], g[2], g[3]};
  if constexpr (SAVE) save_act(save, 2, nt, lane, cat);
  mma_layer<MNR_BF16, 4, 8>(wl + FreqShape::o4, cat, h2, lane);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) h2[mt] = relu4(h2[mt]);
  if constexpr (SAVE) save_act(save, 3, nt, lane, h2);
  f4 o[4];
  mma_layer<MNR_BF16, 1, 4>(wl + FreqShape::o5, h2, o, lane);
  return o[0];
}

// LDS bytes in front of the per-wave feature buffers: the field's MLP
// weights, then (RES) the residual motion network's.
template <int P, int NHH, bool RES, bool FREQ = false>
constexpr int weight_lds_bytes() {
  return (FREQ ? FreqShape::bytes() : MlpShape<P>::bytes_total(NHH)) + (RES ? ResShape::bytes() : 0);
}

// Per-wave feature buffer: the grid's 32 features, or gamma's 64 (FREQ).
template <int P, bool FREQ>
constexpr int feat_bytes() { return FREQ ? FreqShape::feat_bytes_per_wave() : MlpShape<P>::feat_bytes_per_wave(); }

template <int P, int NHH, bool RES, bool FREQ = false>
__device__ __forceinline__ void stage_all(char* wl, const RenderArgs& a) {
  if constexpr (FREQ) stage_freq(wl, a.f);
  else stage_weights<P, NHH>(wl, a.f);
  if constexpr (RES) stage_residual(wl + (FREQ ? FreqShape::bytes() : MlpShape<P>::bytes_total(NHH)), a.res);
}

// PRE: the caller has already set st.xs (the point the field is queried at)
// and st.L (0 for samples that are not live); the warp is skipped.
template <typename TableT, int P, int NHH, bool RES = false, bool FREQ = false, bool PRE = false>
__device__ __forceinline__ uint64_t field_eval(const RenderArgs& a, bool valid, int lane, const char* wl, char* feat,
                                               f4* obuf, SampleState& st, f4& out) {
  if constexpr (!PRE) {
    st.L = 0.f;
    st.xs[0] = st.xs[1] = st.xs[2] = 0.f;
    if (valid) warp_sample(a.m, a.G, st.x, st.xs, st.L);
  }
  st.live = valid && st.L > 0.f;
  const uint64_t live_mask = __ballot(st.live);
  if (live_mask == 0) return 0;
  if constexpr (RES) {
    static_assert(P == MNR_BF16, "the residual motion network runs on the BF16 path");
    residual_step(a.res, wl + (FREQ ? FreqShape::bytes() : MlpShape<P>::bytes_total(NHH)), feat, obuf, st, live_mask,
                  lane);
  }

  if constexpr (FREQ) {
    static_assert(P == MNR_BF16, "the frequency-encoded field runs on the BF16 path");
    store_posenc10(feat, lane, st.xs, st.live);
  } else {
    float u[3];
    unit_coords(a.f, st.xs, u);
    encode_all<TableT>(a.f, u, st.live, [&](int l, f2 v) { store_feat2<P>(feat, lane, 2 * l, v); });
  }
  wave_sync_lds();
  // Tile nt's outputs go to obuf[16 nt ..]; when obuf aliases the feature
  // buffer those bytes belong to tile 0, whose features are already consumed.
#pragma unroll 1
  for (int nt = 0; nt < 4; ++nt) {
    f4 o = {0.f, 0.f, 0.f, 0.f};
    if ((live_mask >> (16 * nt)) & 0xFFFFull) {
      if constexpr (FREQ) o = freq_tile(wl, feat, nt, lane);
      else o = mlp_tile<P, NHH>(wl, feat, nt, lane);
    }
    wave_sync_lds();
    if (lane < 16) obuf[nt * 16 + lane] = o;
  }
  wave_sync_lds();
  out = obuf[lane];
  wave_sync_lds();
  return live_mask;
}

// One 64-sample chunk of a ray (lane i: sample 64 ch + i).
template <typename TableT, int P, int NHH, bool RES = false, bool FREQ = false>
__device__ __forceinline__ uint64_t chunk_eval(const RenderArgs& a, const RaySetup& rs, int ray_index, int ch,
                                               int lane, const char* wl, char* feat, f4* obuf, SampleState& st,
                                               f4& out) {
  const int i = ch * 64 + lane;
  const bool valid = i < a.r.spp;
  const float s = ((float)i + sample_jitter(a.r, ray_index, i)) * rs.delta;
  st.x[0] = fmaf(s, rs.d[0], rs.p0[0]);
  st.x[1] = fmaf(s, rs.d[1], rs.p0[1]);
  st.x[2] = fmaf(s, rs.d[2], rs.p0[2]);
  return field_eval<TableT, P, NHH, RES, FREQ>(a, valid, lane, wl, feat, obuf, st, out);
}

// ---------------------------------------------------------------------------
// Full-frame ray blocks.  Compositing is the per-ray recurrence
//   alpha = 1 - exp(-sigma delta), alpha' = alpha min(L, 1),
//   C += T alpha' c, T *= 1 - alpha'
// sample after sample, and a ray stops once T < ert_tau.  A block writes
// RGBA, optionally the adjoint's saved state, and counts evaluated samples.
// ---------------------------------------------------------------------------
// Value held by lane Q of the caller's group of G lanes (G = 4: DPP quad
// permutation; G = 8 or 16: swizzle inside each 32-lane half, lane
// (l & (32 - G)) | Q).  Every lane of the wave must be active.
template <int G, int Q>
__device__ __forceinline__ float group_bcast(float v) {
  static_assert(G == 4 || G == 8 || G == 16, "groups of 4, 8 or 16 lanes");
  const int b = __builtin_bit_cast(int, v);
  if constexpr (G == 4) return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(b, Q * 0x55, 0xF, 0xF, false));
  else return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(b, (Q << 5) | (32 - G)));
}

// Compositing (Sec. 2.1 Eq. 3 with the Sec. 4.4 likelihood factor) of
// sample j + Q of the ray held by this group of G lanes, whose opacity and
// colour lane Q computed.  Every lane of the group applies the same update,
// so the ray's state stays replicated; the order and the expressions are
// those of one sample per step, and so is early termination (after the
// sample that takes T below ert_tau).  The broadcast values reach the
// update as plain operands, so the compiler cannot fuse 1 - alpha' with the
// product that formed alpha'.
template <int G, int Q>
__device__ __forceinline__ void composite_q(const RenderArgs& a, int j, int pix, int nchunks, int k, float ap, float c0,
                                            float c1, float c2, float lv, bool& ray_act, float& Tr, float& C0,
                                            float& C1, float& C2, int& n_done, unsigned& cnt) {
  const float apq = group_bcast<G, Q>(ap), c0q = group_bcast<G, Q>(c0), c1q = group_bcast<G, Q>(c1);
  const float c2q = group_bcast<G, Q>(c2), lq = group_bcast<G, Q>(lv);
  const int i = j + Q;
  if (ray_act && i < a.r.spp) {
    if (a.t_chunks && (i & 63) == 0 && k == 0) a.t_chunks[(size_t)pix * (nchunks + 1) + (i >> 6)] = Tr;
    if (lq != 0.f) {
      const float w = Tr * apq;
      C0 = fmaf(w, c0q, C0);
      C1 = fmaf(w, c1q, C1);
      C2 = fmaf(w, c2q, C2);
      Tr *= 1.f - apq;
      ++cnt;
    }
    n_done = i + 1;
    if (Tr < a.r.ert_tau || i + 1 >= a.r.spp) ray_act = false;
  }
}

template <int G, int... Q>
__device__ __forceinline__ void composite_group(std::integer_sequence<int, Q...>, const RenderArgs& a, int j, int pix,
                                                int nchunks, int k, float ap, float c0, float c1, float c2, float lv,
                                                bool& ray_act, float& Tr, float& C0, float& C1, float& C2, int& n_done,
                                                unsigned& cnt) {
  (composite_q<G, Q>(a, j, pix, nchunks, k, ap, c0, c1, c2, lv, ray_act, Tr, C0, C1, C2, n_done, cnt), ...);
}

// One block of 64 / G rays, 4 wide and 16 / G tall (sub = 0 .. 4G - 1, raster
// order inside the 16x16 tile), marched G samples per step: lane G r + k
// evaluates sample j + k of ray r.  A block of 64 / G rays is 1 / G of the
// serial work of a wave holding 64 rays, so a frame splits into G times as
// many units and the last units to finish are short.  A ray's recurrence,
// its order and its stopping rule are those of marching it one sample per
// step; samples that follow the terminating one inside its group of G are
// evaluated and discarded (at most G - 1 per ray), and are not counted in
// n_eval.
template <typename TableT, int P, int NHH, bool RES, bool FREQ, int G>
__device__ __forceinline__ void render_tile_rays(const RenderArgs& a, int tile, int sub, int lane, const char* wl,
                                                 char* feat) {
  constexpr int RH = 16 / G;  // rows of the block
  const int S_ = a.r.spp;
  const int nchunks = (S_ + 63) >> 6;
  const int r = lane / G, k = lane % G;
  const int u = (tile % a.r.tiles_x) * 16 + (sub & 3) * 4 + (r & 3);
  const int v = (tile / a.r.tiles_x) * 16 + (sub >> 2) * RH + (r >> 2);
  const bool in_image = u < a.r.W && v < a.r.H;
  const int pix = in_image ? v * a.r.W + u : 0;
  RaySetup rs;
  bool ray_act = in_image && setup_ray(a.r, pix, rs);
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, Tr = 1.f;
  int n_done = 0;
  unsigned cnt = 0;
  for (int j = 0;; j += G) {
    if (__ballot(ray_act) == 0) break;
    const int i = j + k;
    const bool act = ray_act && i < S_;
    SampleState st;
    if (act) {
      const float s = ((float)i + sample_jitter(a.r, pix, i)) * rs.delta;
      st.x[0] = fmaf(s, rs.d[0], rs.p0[0]);
      st.x[1] = fmaf(s, rs.d[1], rs.p0[1]);
      st.x[2] = fmaf(s, rs.d[2], rs.p0[2]);
    }
    f4 out;
    const uint64_t live_mask = field_eval<TableT, P, NHH, RES, FREQ>(a, act, lane, wl, feat, (f4*)feat, st, out);
    float ap = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f, lv = 0.f;
    if (live_mask && st.live) {
      const float sigma = fmaxf(out[3], 0.f);
      ap = -expm1f(-sigma * rs.delta) * fminf(st.L, 1.f);
      c0 = 1.f / (1.f + expf(-out[0]));
      c1 = 1.f / (1.f + expf(-out[1]));
      c2 = 1.f / (1.f + expf(-out[2]));
      lv = 1.f;
    }
    composite_group<G>(std::make_integer_sequence<int, G>{}, a, j, pix, nchunks, k, ap, c0, c1, c2, lv, ray_act, Tr,
                       C0, C1, C2, n_done, cnt);
  }
  if (in_image && k == 0) {
    *(f4*)(a.out + (size_t)pix * 4) = f4{C0 + Tr * a.r.bg[0], C1 + Tr * a.r.bg[1], C2 + Tr * a.r.bg[2], 1.f - Tr};
    if (a.t_chunks) {
      float* tc = a.t_chunks + (size_t)pix * (nchunks + 1);
      for (int ch = (n_done + 63) >> 6; ch < nchunks; ++ch) tc[ch] = -1.f;
      tc[nchunks] = (float)n_done;
    }
  }
  if (a.n_eval) {
    const float tot = wave_sum(k == 0 ? (float)cnt : 0.f);  // exact: at most 16 x 1024
    if (lane == 0 && tot > 0.f) atomicAdd(a.n_eval, (unsigned long long)tot);
  }
}

// Quadrant `quad` (0..3) of a 16x16 tile: its four 4x4 ray blocks in turn.
template <typename TableT, int P, int NHH, bool RES = false, bool FREQ = false>
__device__ __forceinline__ void render_tile_packet(const RenderArgs& a, int tile, int quad, int lane, const char* wl,
                                                   char* feat) {
#pragma unroll 1
  for (int s = 0; s < 4; ++s) {
    const int sx = (quad & 1) * 2 + (s & 1), sy = (quad >> 1) * 2 + (s >> 1);
    render_tile_rays<TableT, P, NHH, RES, FREQ, 4>(a, tile, sy * 4 + sx, lane, wl, feat);
  }
}

}  // namespace mnr
