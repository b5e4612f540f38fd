// Machine-ceiling probes: a random-gather kernel, scattered float atomics
// and a dense MFMA loop (declared in metanerf_probe.h), which share nothing
// with the renderer but the buffer-resource helper; and the renderer's own
// MLP code run unfused, over features read from memory.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "../../include/metanerf_probe.h"
#include "field_device.h"  // make_rsrc
#include "host_common.h"
#include "kernels.h"  // persistent_blocks

namespace mnr {

__device__ __forceinline__ uint32_t mix32(uint32_t a, uint32_t b, uint32_t seed) {
  uint32_t h = a * 0x9E3779B9u + b * 0x85EBCA6Bu + seed;
  h ^= h >> 16; h *= 0x7FEB352Du;
  h ^= h >> 15; h *= 0x846CA68Bu;
  h ^= h >> 16;
  return h;
}

template <int RB>
__device__ __forceinline__ float load_sum(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  if constexpr (RB == 4) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
  } else if constexpr (RB == 8) {
    const f2 v = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
    return v[0] + v[1];
  } else {
    const f4 v = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    return (v[0] + v[1]) + (v[2] + v[3]);
  }
}

template <int RB>
__global__ void __launch_bounds__(256) probe_gather_kernel(const void* table, uint32_t n_rows, uint32_t win_rows,
                                                           int G, uint32_t seed, float* __restrict__ out) {
  const uint32_t gid = blockIdx.x * 256u + threadIdx.x, wave = gid >> 6;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(table, n_rows * (uint32_t)RB);
  const uint32_t span = win_rows ? n_rows - win_rows + 1u : 0u;
  float acc = 0.f;
  for (int k0 = 0; k0 < G; k0 += 8) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t k = (uint32_t)(k0 + j);
      uint32_t row;
      if (win_rows) {
        const uint32_t base = __umulhi(mix32(wave, k, seed ^ 0xA511E9B3u), span);
        row = base + __umulhi(mix32(gid, k, seed), win_rows);
      } else {
        row = __umulhi(mix32(gid, k, seed), n_rows);
      }
      v[j] = load_sum<RB>(rs, row * (uint32_t)RB);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += v[j];
  }
  out[gid] = acc;
}

__global__ void __launch_bounds__(256) probe_atomic_kernel(float* __restrict__ acc, uint32_t n_words, int K, int run,
                                                           uint32_t seed) {
  const uint32_t gid = blockIdx.x * 256u + threadIdx.x, key = gid / (uint32_t)run;
  for (int k = 0; k < K; ++k) unsafeAtomicAdd(acc + __umulhi(mix32(key, (uint32_t)k, seed), n_words), 1.0f);
}

template <bool BF16>
__global__ void __launch_bounds__(256) probe_mfma_kernel(int iters, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  f4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = c0, c2 = c0, c3 = c0;
  if constexpr (BF16) {
    bf16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      a[i] = (__bf16)(1e-3f * (float)(lane + i));
      b[i] = (__bf16)(1e-3f * (float)(lane - i));
    }
    for (int it = 0; it < iters; ++it) {
      c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, a, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, b, c3, 0, 0, 0);
    }
  } else {
    const float a = 1e-3f * (float)lane, b = 1e-3f * (float)(63 - lane);
    for (int it = 0; it < iters; ++it) {
      c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(b, a, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, a, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(b, b, c3, 0, 0, 0);
    }
  }
  out[blockIdx.x * 256u + threadIdx.x] = (c0[0] + c1[1]) + (c2[2] + c3[3]);
}

// The renderer's MLP (weights staged once per block in LDS in MFMA
// fragment order, the layer chain of mlp_tile) over features read from
// memory, one 64-sample chunk per wave at a time; the heads are the
// renderer's: rgb = sigmoid(o0..2), sigma = ReLU(o3).
template <int P, int NHH>
__global__ void __launch_bounds__(256) probe_mlp_kernel(const FieldArgs f, const void* __restrict__ feat_in, int64_t n,
                                                        float* __restrict__ out) {
  using S = MlpShape<P>;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  char* feat = lds + S::bytes_total(NHH) + wave * S::feat_bytes_per_wave();
  stage_weights<P, NHH>(lds, f);
  __syncthreads();
  const int64_t nchunks = (n + 63) >> 6;
  for (int64_t c = (int64_t)blockIdx.x * 4 + wave; c < nchunks; c += (int64_t)gridDim.x * 4) {
    const int64_t s = c * 64 + lane;
    if constexpr (P == MNR_F32) {
      float v[IN_FEAT];
#pragma unroll
      for (int k = 0; k < IN_FEAT; ++k) v[k] = 0.f;
      if (s < n) {
        const f4* src = (const f4*)((const float*)feat_in + s * IN_FEAT);
#pragma unroll
        for (int q = 0; q < IN_FEAT / 4; ++q) {
          const f4 t = src[q];
          v[4 * q] = t[0]; v[4 * q + 1] = t[1]; v[4 * q + 2] = t[2]; v[4 * q + 3] = t[3];
        }
      }
#pragma unroll
      for (int k = 0; k < IN_FEAT / 2; ++k) store_feat2<P>(feat, lane, 2 * k, f2{v[2 * k], v[2 * k + 1]});
    } else {  // BF16 features go to their LDS slots as they are (store_feat2's layout, no conversion)
      const bf16x8* src = (const bf16x8*)((const __bf16*)feat_in + s * IN_FEAT);
#pragma unroll
      for (int q = 0; q < IN_FEAT / 8; ++q) {
        bf16x8 t = {};
        if (s < n) t = src[q];
#pragma unroll
        for (int j = 0; j < 4; ++j) {  // features 8q + 2j, 8q + 2j + 1
          const int k = 8 * q + 2 * j, nt = lane >> 4, ln = (lane & 15) + 16 * ((k & 15) >> 2);
          *(bf16x2*)(feat + ((nt * 64 + ln) * 8 + (k >> 4) * 4 + (k & 3)) * 2) = bf16x2{t[2 * j], t[2 * j + 1]};
        }
      }
    }
    wave_sync_lds();
#pragma unroll 1
    for (int nt = 0; nt < 4; ++nt) {
      const f4 o = mlp_tile<P, NHH>(lds, feat, nt, lane);
      const int64_t r = c * 64 + nt * 16 + lane;
      if (lane < 16 && r < n)
        *(f4*)(out + r * 4) = f4{1.f / (1.f + expf(-o[0])), 1.f / (1.f + expf(-o[1])), 1.f / (1.f + expf(-o[2])),
                                 fmaxf(o[3], 0.f)};
    }
    wave_sync_lds();  // the next chunk rewrites the feature buffer
  }
}

template <int P, int NHH>
static hipError_t launch_probe_mlp(const FieldArgs& F, const void* feat, int64_t n, float* out, hipStream_t st) {
  using S = MlpShape<P>;
  const int lds = S::bytes_total(NHH) + 4 * S::feat_bytes_per_wave();
  auto kern = probe_mlp_kernel<P, NHH>;
  static PersistentGrid pg;
  const int max_blocks = persistent_blocks(kern, 256, lds, pg);
  const int64_t need = ((n + 63) / 64 + 3) / 4;
  const int grid = need < max_blocks ? (int)need : max_blocks;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, st, F, feat, n, out);
  return hipGetLastError();
}

}  // namespace mnr

using namespace mnr;

extern "C" mnr_status mnr_probe_gather(const void* table, uint64_t table_bytes, int32_t row_bytes,
                                       uint32_t window_bytes, int32_t gathers_per_lane, int32_t n_lanes,
                                       uint32_t seed, float* out, void* stream) {
  clear_error();
  if (!table || !out) return fail(MNR_E_INVALID, "probe_gather: null pointer");
  if (row_bytes != 4 && row_bytes != 8 && row_bytes != 16) return fail(MNR_E_SHAPE, "probe_gather: row_bytes 4, 8 or 16");
  if (table_bytes < (uint64_t)row_bytes || table_bytes > 0x7FFFFFFFull)
    return fail(MNR_E_SHAPE, "probe_gather: table_bytes out of range");
  if (gathers_per_lane < 8 || gathers_per_lane % 8 || n_lanes < 256 || n_lanes % 256)
    return fail(MNR_E_SHAPE, "probe_gather: gathers_per_lane must be a multiple of 8, n_lanes of 256");
  const uint32_t n_rows = (uint32_t)(table_bytes / (uint64_t)row_bytes);
  const uint32_t win_rows = window_bytes ? window_bytes / (uint32_t)row_bytes : 0u;
  if (window_bytes && (win_rows < 1 || win_rows > n_rows)) return fail(MNR_E_SHAPE, "probe_gather: bad window");
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid(n_lanes / 256), block(256);
  if (row_bytes == 4) hipLaunchKernelGGL(probe_gather_kernel<4>, grid, block, 0, st, table, n_rows, win_rows, gathers_per_lane, seed, out);
  else if (row_bytes == 8) hipLaunchKernelGGL(probe_gather_kernel<8>, grid, block, 0, st, table, n_rows, win_rows, gathers_per_lane, seed, out);
  else hipLaunchKernelGGL(probe_gather_kernel<16>, grid, block, 0, st, table, n_rows, win_rows, gathers_per_lane, seed, out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MNR_OK : fail(MNR_E_HIP, "probe_gather launch: %s", hipGetErrorString(e));
}

extern "C" mnr_status mnr_probe_atomic(float* acc, uint32_t n_words, int32_t atomics_per_lane, int32_t n_lanes,
                                       int32_t run, uint32_t seed, void* stream) {
  clear_error();
  if (!acc) return fail(MNR_E_INVALID, "probe_atomic: null pointer");
  if (n_words < 1 || atomics_per_lane < 1 || n_lanes < 256 || n_lanes % 256 || run < 1 || run > 64)
    return fail(MNR_E_SHAPE, "probe_atomic: bad sizes");
  hipLaunchKernelGGL(probe_atomic_kernel, dim3(n_lanes / 256), dim3(256), 0, (hipStream_t)stream, acc, n_words,
                     atomics_per_lane, run, seed);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MNR_OK : fail(MNR_E_HIP, "probe_atomic launch: %s", hipGetErrorString(e));
}

// LDS operation throughput (the adjoint's block sums): one op per thread
// per iteration on word (thread + 97 k) mod 8192.
template <int OP>
__global__ void __launch_bounds__(1024) probe_lds_kernel(int iters, float* __restrict__ out) {
  __shared__ float sf[8192];
  __shared__ uint32_t su[8192];
  __shared__ unsigned long long s64[4096];
  for (int i = threadIdx.x; i < 8192; i += blockDim.x) {
    sf[i] = 0.f;
    su[i] = 0u;
  }
  for (int i = threadIdx.x; i < 4096; i += blockDim.x) s64[i] = 0ull;
  __syncthreads();
  const float v = 1.0f + (float)threadIdx.x * 1e-7f;
  for (int k = 0; k < iters; ++k) {
    const uint32_t w = (threadIdx.x + 97u * (uint32_t)k) & 8191u;
    if constexpr (OP == 0) atomicAdd(&sf[w], v);
    if constexpr (OP == 1) atomicAdd(&su[w], 1u);
    if constexpr (OP == 2) atomicAdd(&s64[w & 4095u], 1ull);
    if constexpr (OP == 3) sf[w] += v;
    if constexpr (OP == 4) sf[w] = v;
  }
  __syncthreads();
  out[(size_t)blockIdx.x * 1024 + threadIdx.x] = sf[threadIdx.x] + (float)su[threadIdx.x] + (float)s64[threadIdx.x];
}

extern "C" mnr_status mnr_probe_lds(int32_t op, int32_t iters, int32_t n_blocks, float* out, void* stream) {
  clear_error();
  if (!out) return fail(MNR_E_INVALID, "probe_lds: null pointer");
  if (op < 0 || op > 4) return fail(MNR_E_INVALID, "probe_lds: op must be 0..4");
  if (iters < 1 || iters > 100000 || n_blocks < 4 || n_blocks > 4096) return fail(MNR_E_SHAPE, "probe_lds: bad sizes");
  hipStream_t st = (hipStream_t)stream;
  switch (op) {
    case 0: hipLaunchKernelGGL(probe_lds_kernel<0>, dim3(n_blocks), dim3(1024), 0, st, iters, out); break;
    case 1: hipLaunchKernelGGL(probe_lds_kernel<1>, dim3(n_blocks), dim3(1024), 0, st, iters, out); break;
    case 2: hipLaunchKernelGGL(probe_lds_kernel<2>, dim3(n_blocks), dim3(1024), 0, st, iters, out); break;
    case 3: hipLaunchKernelGGL(probe_lds_kernel<3>, dim3(n_blocks), dim3(1024), 0, st, iters, out); break;
    default: hipLaunchKernelGGL(probe_lds_kernel<4>, dim3(n_blocks), dim3(1024), 0, st, iters, out); break;
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MNR_OK : fail(MNR_E_HIP, "probe_lds launch: %s", hipGetErrorString(e));
}

extern "C" mnr_status mnr_probe_mfma(mnr_dtype dtype, int32_t iters, int32_t n_blocks, float* out, void* stream) {
  clear_error();
  if (!out) return fail(MNR_E_INVALID, "probe_mfma: null pointer");
  if (dtype != MNR_F32 && dtype != MNR_BF16) return fail(MNR_E_DTYPE, "probe_mfma: F32 or BF16");
  if (iters < 1 || n_blocks < 1) return fail(MNR_E_SHAPE, "probe_mfma: iters and n_blocks must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  if (dtype == MNR_BF16) hipLaunchKernelGGL(probe_mfma_kernel<true>, dim3(n_blocks), dim3(256), 0, st, iters, out);
  else hipLaunchKernelGGL(probe_mfma_kernel<false>, dim3(n_blocks), dim3(256), 0, st, iters, out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MNR_OK : fail(MNR_E_HIP, "probe_mfma launch: %s", hipGetErrorString(e));
}

extern "C" mnr_status mnr_probe_mlp(const mnr_field* field, const void* feat, int64_t n, float* out, void* stream) {
  clear_error();
  if (!field) return fail(MNR_E_INVALID, "probe_mlp: null field");
  if (n < 0 || n > ((int64_t)1 << 40)) return fail(MNR_E_SHAPE, "probe_mlp: n out of range");
  if (n > 0 && (!feat || !out)) return fail(MNR_E_INVALID, "probe_mlp: null pointer");
  if (((uintptr_t)feat | (uintptr_t)out) & 15) return fail(MNR_E_INVALID, "probe_mlp: feat and out must be 16-byte aligned");
  if (field->encoding != MNR_ENC_GRID) return fail(MNR_E_UNSUPPORTED, "probe_mlp: the grid-encoded field's MLP only");
  if (field->mlp_dtype != MNR_F32 && field->mlp_dtype != MNR_BF16) return fail(MNR_E_DTYPE, "probe_mlp: F32 or BF16 MLP");
  const int nl = field->n_layers;
  if (nl < 2 || nl > 4) return fail(MNR_E_SHAPE, "probe_mlp: 2..4 layers");
  if (field->width[0] != IN_FEAT || field->width[nl] != 4) return fail(MNR_E_SHAPE, "probe_mlp: widths 32 -> ... -> 4");
  for (int k = 1; k < nl; ++k)
    if (field->width[k] != HIDDEN) return fail(MNR_E_SHAPE, "probe_mlp: hidden width must be 64");
  for (int k = 0; k < nl; ++k)
    if (!field->w[k]) return fail(MNR_E_INVALID, "probe_mlp: null weight %d", k);
  if (n == 0) return MNR_OK;
  FieldArgs F;
  std::memset(&F, 0, sizeof(F));  // only the weights are read
  for (int k = 0; k < nl; ++k) F.w[k] = field->w[k];
  F.n_layers = nl;
  hipStream_t st = (hipStream_t)stream;
  const int nhh = nl - 2;
  hipError_t e;
  if (field->mlp_dtype == MNR_BF16)
    e = nhh == 0 ? launch_probe_mlp<MNR_BF16, 0>(F, feat, n, out, st)
      : nhh == 1 ? launch_probe_mlp<MNR_BF16, 1>(F, feat, n, out, st)
                 : launch_probe_mlp<MNR_BF16, 2>(F, feat, n, out, st);
  else
    e = nhh == 0 ? launch_probe_mlp<MNR_F32, 0>(F, feat, n, out, st)
      : nhh == 1 ? launch_probe_mlp<MNR_F32, 1>(F, feat, n, out, st)
                 : launch_probe_mlp<MNR_F32, 2>(F, feat, n, out, st);
  return e == hipSuccess ? MNR_OK : fail(MNR_E_HIP, "probe_mlp launch: %s", hipGetErrorString(e));
}
