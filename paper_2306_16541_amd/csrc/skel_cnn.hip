// Skeleton-motion CNN (Sec. 4.2, Eq. 10, Fig. 7): fully connected layer,
// then five 3-D transposed convolutions (kernel 4, stride 2, padding 1)
// from one voxel to the 32^3 logit volume of the blend weights, and its
// adjoint.  It runs once per training step (about 1.5 GFLOP with the
// adjoint).  The kernels are direct, weights and activations read through
// the caches; each output element belongs to a group of R lanes that split
// its reduction and meet by xor shuffles.  R is chosen per layer so that
// every launch has about 512 K lanes (the chip's wave slots): the coarse
// layers have few outputs and long reductions (2,048 terms per output in
// the first layer, 8,192 in its adjoint), the fine ones many outputs and
// short reductions.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "host_common.h"

namespace mnr {

constexpr float SLOPE = 0.2f;  // LeakyReLU

__device__ __forceinline__ float lrelu(float x) { return x > 0.f ? x : SLOPE * x; }

// Sum over the R lanes of the caller's group (R divides 64; a group is
// either fully active or fully idle).
template <int R>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int m = R / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, WAVE);
  return v;
}

// out[o][X] = sum_i sum_taps w[i][o][k] in[i][v], X = 2 v - 1 + k per axis.
// For each output coordinate two input positions contribute:
// v = (X + 1) / 2 - t, k = X + 1 - 2 v, t = 0, 1.  Lane r of a group takes
// the input channels i = r, r + R, ...
template <int R>
__global__ void tconv_fwd_kernel(const float* __restrict__ in, const float* __restrict__ w, float* __restrict__ out,
                                 int ci, int co, int D, int act) {
  const int D2 = 2 * D;
  const int64_t n = (int64_t)co * D2 * D2 * D2;
  const int r = threadIdx.x % R;
  const int64_t groups = (int64_t)gridDim.x * blockDim.x / R;
  for (int64_t e = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / R; e < n; e += groups) {
    const int X = (int)(e % D2), Y = (int)((e / D2) % D2), Z = (int)((e / D2 / D2) % D2);
    const int o = (int)(e / ((int64_t)D2 * D2 * D2));
    float acc = 0.f;
    for (int tz = 0; tz < 2; ++tz) {
      const int vz = (Z + 1) / 2 - tz, kz = Z + 1 - 2 * vz;
      if (vz < 0 || vz >= D || kz > 3) continue;
      for (int ty = 0; ty < 2; ++ty) {
        const int vy = (Y + 1) / 2 - ty, ky = Y + 1 - 2 * vy;
        if (vy < 0 || vy >= D || ky > 3) continue;
        for (int tx = 0; tx < 2; ++tx) {
          const int vx = (X + 1) / 2 - tx, kx = X + 1 - 2 * vx;
          if (vx < 0 || vx >= D || kx > 3) continue;
          const int64_t vi = ((int64_t)vz * D + vy) * D + vx, ki = (kz * 4 + ky) * 4 + kx;
          for (int i = r; i < ci; i += R)
            acc = fmaf(w[((int64_t)i * co + o) * 64 + ki], in[(int64_t)i * D * D * D + vi], acc);
        }
      }
    }
    acc = group_sum<R>(acc);
    if (r == 0) out[e] = act ? lrelu(acc) : acc;
  }
}

// gin[i][v] = lrelu'(a_in[i][v]) sum_o sum_k w[i][o][k] gout[o][2 v - 1 + k];
// lane r of a group takes the output channels o = r, r + R, ...
template <int R>
__global__ void tconv_dgrad_kernel(const float* __restrict__ gout, const float* __restrict__ w,
                                   const float* __restrict__ a_in, float* __restrict__ gin, int ci, int co, int D) {
  const int D2 = 2 * D;
  const int64_t n = (int64_t)ci * D * D * D;
  const int r = threadIdx.x % R;
  const int64_t groups = (int64_t)gridDim.x * blockDim.x / R;
  for (int64_t e = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / R; e < n; e += groups) {
    const int vx = (int)(e % D), vy = (int)((e / D) % D), vz = (int)((e / D / D) % D);
    const int i = (int)(e / ((int64_t)D * D * D));
    float acc = 0.f;
    for (int kz = 0; kz < 4; ++kz) {
      const int Z = 2 * vz - 1 + kz;
      if (Z < 0 || Z >= D2) continue;
      for (int ky = 0; ky < 4; ++ky) {
        const int Y = 2 * vy - 1 + ky;
        if (Y < 0 || Y >= D2) continue;
        for (int kx = 0; kx < 4; ++kx) {
          const int X = 2 * vx - 1 + kx;
          if (X < 0 || X >= D2) continue;
          const int64_t oi = ((int64_t)Z * D2 + Y) * D2 + X;
          const int ki = (kz * 4 + ky) * 4 + kx;
          for (int o = r; o < co; o += R)
            acc = fmaf(w[((int64_t)i * co + o) * 64 + ki], gout[(int64_t)o * D2 * D2 * D2 + oi], acc);
        }
      }
    }
    acc = group_sum<R>(acc);
    if (r == 0) gin[e] = a_in[e] > 0.f ? acc : SLOPE * acc;
  }
}

// gw[i][o][k] += sum_v in[i][v] gout[o][2 v - 1 + k]; lane r of a group
// takes the input positions v = r, r + R, ... (flattened).
template <int R>
__global__ void tconv_wgrad_kernel(const float* __restrict__ in, const float* __restrict__ gout,
                                   float* __restrict__ gw, int ci, int co, int D) {
  const int D2 = 2 * D, DDD = D * D * D;
  const int64_t n = (int64_t)ci * co * 64;
  const int r = threadIdx.x % R;
  const int64_t groups = (int64_t)gridDim.x * blockDim.x / R;
  for (int64_t e = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / R; e < n; e += groups) {
    const int ki = (int)(e % 64), kx = ki & 3, ky = (ki >> 2) & 3, kz = ki >> 4;
    const int o = (int)((e / 64) % co), i = (int)(e / 64 / co);
    const float* src = in + (int64_t)i * DDD;
    const float* g = gout + (int64_t)o * D2 * D2 * D2;
    float acc = 0.f;
    for (int v = r; v < DDD; v += R) {
      const int vx = v % D, vy = (v / D) % D, vz = v / (D * D);
      const int Z = 2 * vz - 1 + kz, Y = 2 * vy - 1 + ky, X = 2 * vx - 1 + kx;
      if (Z < 0 || Z >= D2 || Y < 0 || Y >= D2 || X < 0 || X >= D2) continue;
      acc = fmaf(src[v], g[((int64_t)Z * D2 + Y) * D2 + X], acc);
    }
    acc = group_sum<R>(acc);
    if (r == 0) gw[e] += acc;
  }
}

__global__ void fc_fwd_kernel(const float* __restrict__ w, const float* __restrict__ z, float* __restrict__ out,
                              int c0, int L) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < c0; c += gridDim.x * blockDim.x) {
    float acc = 0.f;
    for (int j = 0; j < L; ++j) acc = fmaf(w[(int64_t)c * L + j], z[j], acc);
    out[c] = lrelu(acc);
  }
}

// gw[c][j] += g[c] z[j] (g already carries the LeakyReLU derivative).
__global__ void fc_wgrad_kernel(const float* __restrict__ g, const float* __restrict__ z, float* __restrict__ gw,
                                int c0, int L) {
  const int64_t n = (int64_t)c0 * L;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    gw[e] += g[e / L] * z[e % L];
}

static int grid_of(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

// Lanes per output element: about 512 K lanes in all, at most `terms`
// (the reduction length) and at most a wave.
static int lanes_per_output(int64_t n, int64_t terms) {
  int R = 1;
  while (R < 64 && n * R * 2 <= (int64_t)1 << 19 && R * 2 <= terms) R *= 2;
  return R;
}

// Launches kernel template K<R> for the R that lanes_per_output picks.
template <template <int> class K, typename... Args>
static void launch_grouped(int64_t n, int64_t terms, hipStream_t st, Args... args) {
  const int R = lanes_per_output(n, terms);
  const dim3 grid(grid_of(n * R)), block(256);
  switch (R) {
    case 1: hipLaunchKernelGGL(K<1>::fn, grid, block, 0, st, args...); break;
    case 2: hipLaunchKernelGGL(K<2>::fn, grid, block, 0, st, args...); break;
    case 4: hipLaunchKernelGGL(K<4>::fn, grid, block, 0, st, args...); break;
    case 8: hipLaunchKernelGGL(K<8>::fn, grid, block, 0, st, args...); break;
    case 16: hipLaunchKernelGGL(K<16>::fn, grid, block, 0, st, args...); break;
    case 32: hipLaunchKernelGGL(K<32>::fn, grid, block, 0, st, args...); break;
    default: hipLaunchKernelGGL(K<64>::fn, grid, block, 0, st, args...); break;
  }
}

template <int R> struct TconvFwd { static constexpr auto fn = tconv_fwd_kernel<R>; };
template <int R> struct TconvDgrad { static constexpr auto fn = tconv_dgrad_kernel<R>; };
template <int R> struct TconvWgrad { static constexpr auto fn = tconv_wgrad_kernel<R>; };

// Activation k (k = 0..4) has channels[k] channels on a (2^k)^3 grid.
static int64_t act_size(const mnr_skel_cnn* c, int k) { return (int64_t)c->channels[k] << (3 * k); }
static int64_t act_offset(const mnr_skel_cnn* c, int k) {
  int64_t off = 0;
  for (int j = 0; j < k; ++j) off += act_size(c, j);
  return off;
}

static mnr_status validate_cnn(const mnr_skel_cnn* c) {
  if (!c || !c->z || !c->w_fc) return fail(MNR_E_INVALID, "skel_cnn: null pointer");
  for (int k = 0; k < 5; ++k)
    if (!c->w[k]) return fail(MNR_E_INVALID, "skel_cnn: null weight %d", k);
  if (c->latent < 1 || c->latent > 4096) return fail(MNR_E_SHAPE, "skel_cnn: latent must be in [1, 4096]");
  for (int k = 0; k < 6; ++k)
    if (c->channels[k] < 1 || c->channels[k] > 1024) return fail(MNR_E_SHAPE, "skel_cnn: channels must be in [1, 1024]");
  return MNR_OK;
}

}  // namespace mnr

using namespace mnr;

extern "C" uint64_t mnr_skel_cnn_act_floats(const mnr_skel_cnn* c) {
  clear_error();
  if (validate_cnn(c) != MNR_OK) return 0;
  return (uint64_t)act_offset(c, 5);
}

extern "C" uint64_t mnr_skel_cnn_scratch_floats(const mnr_skel_cnn* c) {
  clear_error();
  if (validate_cnn(c) != MNR_OK) return 0;
  int64_t mx = 0;
  for (int k = 0; k < 5; ++k) mx = act_size(c, k) > mx ? act_size(c, k) : mx;
  return 2 * (uint64_t)mx;
}

extern "C" mnr_status mnr_skel_cnn_forward(const mnr_skel_cnn* c, float* act, float* logits, void* stream) {
  clear_error();
  if (mnr_status s = validate_cnn(c)) return s;
  if (!act || !logits) return fail(MNR_E_INVALID, "skel_cnn: null output");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(fc_fwd_kernel, dim3(grid_of(c->channels[0])), dim3(256), 0, st, c->w_fc, c->z, act,
                     c->channels[0], c->latent);
  for (int k = 1; k <= 5; ++k) {
    const float* in = act + act_offset(c, k - 1);
    float* out = k < 5 ? act + act_offset(c, k) : logits;
    const int64_t n = (int64_t)c->channels[k] << (3 * k);
    launch_grouped<TconvFwd>(n, c->channels[k - 1], st, in, (const float*)c->w[k - 1], out, c->channels[k - 1],
                             c->channels[k], 1 << (k - 1), k < 5 ? 1 : 0);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MNR_OK : fail(MNR_E_HIP, "skel_cnn forward: %s", hipGetErrorString(e));
}

extern "C" mnr_status mnr_skel_cnn_backward(const mnr_skel_cnn* c, const float* act, const float* grad_logits,
                                            float* grad_w_fc, float* const* grad_w, float* scratch, void* stream) {
  clear_error();
  if (mnr_status s = validate_cnn(c)) return s;
  if (!act || !grad_logits || !grad_w_fc || !grad_w || !scratch) return fail(MNR_E_INVALID, "skel_cnn: null pointer");
  for (int k = 0; k < 5; ++k)
    if (!grad_w[k]) return fail(MNR_E_INVALID, "skel_cnn: null gradient %d", k);
  hipStream_t st = (hipStream_t)stream;
  int64_t mx = 0;
  for (int k = 0; k < 5; ++k) mx = act_size(c, k) > mx ? act_size(c, k) : mx;
  float* buf[2] = {scratch, scratch + mx};
  const float* g = grad_logits;  // dL/d(output of convolution k)
  for (int k = 5; k >= 1; --k) {
    const float* in = act + act_offset(c, k - 1);
    const int D = 1 << (k - 1), ci = c->channels[k - 1], co = c->channels[k];
    launch_grouped<TconvWgrad>((int64_t)ci * co * 64, (int64_t)D * D * D, st, in, g, grad_w[k - 1], ci, co, D);
    float* gin = buf[k & 1];
    launch_grouped<TconvDgrad>((int64_t)ci * D * D * D, co, st, g, (const float*)c->w[k - 1], in, gin, ci, co, D);
    g = gin;
  }
  hipLaunchKernelGGL(fc_wgrad_kernel, dim3(grid_of((int64_t)c->channels[0] * c->latent)), dim3(256), 0, st, g, c->z,
                     grad_w_fc, c->channels[0], c->latent);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MNR_OK : fail(MNR_E_HIP, "skel_cnn backward: %s", hipGetErrorString(e));
}
