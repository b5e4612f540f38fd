// Elementwise and small-reduction kernels of the training step (Sec. 5.2):
// the squared-error loss (MSE term of Eq. 14), the per-voxel softmax that
// turns free logits into canonical blend weights W^c (Sec. 4.2) and its
// adjoint, Adam (beta1 = 0.9, beta2 = 0.99 in the paper), precision
// conversion of parameter copies, the packed copies of the blend-weight
// volume and of the dense grid levels read by the renderer, and a kernel
// fill.
#include "device_common.h"
#include "kernels.h"

namespace mnr {

static inline int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (int)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

// Single block: deterministic reduction order.
__global__ void __launch_bounds__(1024) mse_kernel(const float* __restrict__ rgba, const float* __restrict__ tgt, int n,
                                                   float* __restrict__ grad, float* __restrict__ loss) {
  __shared__ float part[1024 / 64];
  const float scale = 1.0f / (3.0f * (float)n);
  float acc = 0.f;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    const f4 c = *(const f4*)(rgba + 4 * (size_t)r);
    const float e0 = c[0] - tgt[3 * (size_t)r], e1 = c[1] - tgt[3 * (size_t)r + 1], e2 = c[2] - tgt[3 * (size_t)r + 2];
    acc += e0 * e0 + e1 * e1 + e2 * e2;
    *(f4*)(grad + 4 * (size_t)r) = f4{2.f * scale * e0, 2.f * scale * e1, 2.f * scale * e2, 0.f};
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && loss) {
    float s = 0.f;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += part[i];
    loss[0] = s * scale;
  }
}

hipError_t launch_mse(const float* rgba, const float* target, int n, float* grad, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(1024), 0, st, rgba, target, n, grad, loss);
  return hipGetLastError();
}

__global__ void softmax_fwd_kernel(const float* __restrict__ x, float* __restrict__ w, int C, int64_t V) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < V; v += (int64_t)gridDim.x * blockDim.x) {
    float mx = -INFINITY;
    for (int c = 0; c < C; ++c) mx = fmaxf(mx, x[c * V + v]);
    float s = 0.f;
    for (int c = 0; c < C; ++c) s += expf(x[c * V + v] - mx);
    const float inv = 1.0f / s;
    for (int c = 0; c < C; ++c) w[c * V + v] = expf(x[c * V + v] - mx) * inv;
  }
}

hipError_t launch_softmax_fwd(const float* logits, float* w, int C, int64_t V, hipStream_t st) {
  hipLaunchKernelGGL(softmax_fwd_kernel, dim3(grid_for(V, 256)), dim3(256), 0, st, logits, w, C, V);
  return hipGetLastError();
}

__global__ void softmax_bwd_kernel(const float* __restrict__ w, const float* __restrict__ g, float* __restrict__ gl,
                                   int C, int64_t V) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < V; v += (int64_t)gridDim.x * blockDim.x) {
    float dot = 0.f;
    for (int c = 0; c < C; ++c) dot += w[c * V + v] * g[c * V + v];
    for (int c = 0; c < C; ++c) gl[c * V + v] += w[c * V + v] * (g[c * V + v] - dot);
  }
}

hipError_t launch_softmax_bwd(const float* w, const float* g, float* gl, int C, int64_t V, hipStream_t st) {
  hipLaunchKernelGGL(softmax_bwd_kernel, dim3(grid_for(V, 256)), dim3(256), 0, st, w, g, gl, C, V);
  return hipGetLastError();
}

// The blend-weight logits' whole update in one pass per voxel (free logits,
// Sec. 4.2 as trained here): the softmax adjoint dL/dlogit_c =
// w_c (g_c - sum_k w_k g_k), written to gl; Adam on the logits (the same
// arithmetic as adam_kernel); the softmax of the new logits into w: the
// work of the three separate kernels in one pass over the volume.
__global__ void motion_step_kernel(float* __restrict__ logits, float* __restrict__ w, const float* __restrict__ g,
                                   float* __restrict__ gl, float* __restrict__ m, float* __restrict__ v, int C,
                                   int64_t V, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < V; x += (int64_t)gridDim.x * blockDim.x) {
    float dot = 0.f;
    for (int c = 0; c < C; ++c) dot += w[c * V + x] * g[c * V + x];
    float mx = -INFINITY;
    for (int c = 0; c < C; ++c) {
      const int64_t i = c * V + x;
      const float gi = 0.f + w[i] * (g[i] - dot);
      gl[i] = gi;
      const float mi = b1 * m[i] + (1.f - b1) * gi;
      const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
      m[i] = mi;
      v[i] = vi;
      const float pi = logits[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
      logits[i] = pi;
      mx = fmaxf(mx, pi);
    }
    float s = 0.f;
    for (int c = 0; c < C; ++c) s += expf(logits[c * V + x] - mx);
    const float inv = 1.0f / s;
    for (int c = 0; c < C; ++c) w[c * V + x] = expf(logits[c * V + x] - mx) * inv;
  }
}

hipError_t launch_motion_step(float* logits, float* w, const float* g, float* gl, float* m, float* v, int C,
                              int64_t V, float lr, float b1, float b2, float eps, int step, hipStream_t st) {
  const float bc1 = 1.f - (float)std::pow((double)b1, (double)step);
  const float bc2 = 1.f - (float)std::pow((double)b2, (double)step);
  hipLaunchKernelGGL(motion_step_kernel, dim3(grid_for(V, 256)), dim3(256), 0, st, logits, w, g, gl, m, v, C, V, lr,
                     b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

template <typename LowT>
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                            float bc2, LowT* __restrict__ low) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    if (low) low[i] = (LowT)pi;
  }
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                       int step, void* lowp, mnr_dtype dt, hipStream_t st) {
  const float bc1 = 1.f - (float)std::pow((double)b1, (double)step);
  const float bc2 = 1.f - (float)std::pow((double)b2, (double)step);
  const dim3 grid(grid_for(n, 256));
  if (lowp && dt == MNR_BF16)
    hipLaunchKernelGGL(adam_kernel<__bf16>, grid, dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, bc1, bc2,
                       (__bf16*)lowp);
  else
    hipLaunchKernelGGL(adam_kernel<_Float16>, grid, dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, bc1, bc2,
                       (_Float16*)lowp);
  return hipGetLastError();
}

// Tensor blockIdx.y of the list; the x blocks stride over it.
template <typename LowT>
__global__ void adam_list_kernel(const AdamList l, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  const int k = blockIdx.y;
  float* __restrict__ p = l.p[k];
  const float* __restrict__ g = l.g[k];
  float* __restrict__ m = l.m[k];
  float* __restrict__ v = l.v[k];
  LowT* __restrict__ low = (LowT*)l.low[k];
  const int64_t n = l.n[k];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    if (low) low[i] = (LowT)pi;
  }
}

hipError_t launch_adam_list(const AdamList& l, float lr, float b1, float b2, float eps, int step, mnr_dtype low_dt,
                            hipStream_t st) {
  if (l.count <= 0) return hipSuccess;
  if (l.count > MAX_LIST) return hipErrorInvalidValue;
  const float bc1 = 1.f - (float)std::pow((double)b1, (double)step);
  const float bc2 = 1.f - (float)std::pow((double)b2, (double)step);
  int64_t most = 0;
  for (int k = 0; k < l.count; ++k) most = l.n[k] > most ? l.n[k] : most;
  const dim3 grid(grid_for(most, 256), l.count);
  if (low_dt == MNR_BF16)
    hipLaunchKernelGGL(adam_list_kernel<__bf16>, grid, dim3(256), 0, st, l, lr, b1, b2, eps, bc1, bc2);
  else
    hipLaunchKernelGGL(adam_list_kernel<_Float16>, grid, dim3(256), 0, st, l, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

template <typename LowT>
__global__ void convert_kernel(const float* __restrict__ s, LowT* __restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = (LowT)s[i];
}

hipError_t launch_convert(const float* src, void* dst, mnr_dtype dt, int64_t n, hipStream_t st) {
  if (dt == MNR_BF16)
    hipLaunchKernelGGL(convert_kernel<__bf16>, dim3(grid_for(n, 256)), dim3(256), 0, st, src, (__bf16*)dst, n);
  else
    hipLaunchKernelGGL(convert_kernel<_Float16>, dim3(grid_for(n, 256)), dim3(256), 0, st, src, (_Float16*)dst, n);
  return hipGetLastError();
}

__global__ void zero_kernel(uint32_t* __restrict__ d, int64_t n_words) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_words; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = 0u;
}

// Processing order of a ray list: a counting sort of the rays by the
// Morton index of their pixel's cell in a 64 x 64 grid over the image (one
// block; not stable).  Rays that are close on the image sample close points,
// so neighbouring slots then gather from the same table and blend-weight
// lines.
constexpr int ORDER_THREADS = 1024;
constexpr int ORDER_CELLS = 4096;

__device__ __forceinline__ uint32_t order_cell(int pix, int H, int W) {
  if (pix < 0 || pix >= H * W) return 0u;
  const uint32_t x = (uint32_t)(pix % W) * 64u / (uint32_t)W, y = (uint32_t)(pix / W) * 64u / (uint32_t)H;
  uint32_t m = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b) m |= (((x >> b) & 1u) << (2 * b)) | (((y >> b) & 1u) << (2 * b + 1));
  return m;
}

__global__ void __launch_bounds__(ORDER_THREADS) ray_order_kernel(const int32_t* __restrict__ pixel_ids, int n, int H,
                                                                 int W, int32_t* __restrict__ order) {
  __shared__ uint32_t cnt[ORDER_CELLS];
  __shared__ uint32_t red[ORDER_THREADS / WAVE];
  const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x >> 6;
  for (int c = threadIdx.x; c < ORDER_CELLS; c += ORDER_THREADS) cnt[c] = 0u;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += ORDER_THREADS) atomicAdd(&cnt[order_cell(pixel_ids[i], H, W)], 1u);
  __syncthreads();
  constexpr int PER = ORDER_CELLS / ORDER_THREADS;  // consecutive cells per thread
  uint32_t loc[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    loc[j] = cnt[threadIdx.x * PER + j];
    sum += loc[j];
  }
  uint32_t incl = sum;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t o = __shfl_up(incl, d, WAVE);
    if (lane >= d) incl += o;
  }
  if (lane == WAVE - 1) red[wave] = incl;
  __syncthreads();
  uint32_t run = incl - sum;
  for (int w = 0; w < wave; ++w) run += red[w];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    cnt[threadIdx.x * PER + j] = run;
    run += loc[j];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += ORDER_THREADS) order[atomicAdd(&cnt[order_cell(pixel_ids[i], H, W)], 1u)] = i;
}

hipError_t launch_ray_order(const int32_t* pixel_ids, int n, int H, int W, int32_t* order, hipStream_t st) {
  hipLaunchKernelGGL(ray_order_kernel, dim3(1), dim3(ORDER_THREADS), 0, st, pixel_ids, n, H, W, order);
  return hipGetLastError();
}

// Buffer blockIdx.y of the list (byte counts that are multiples of 4).
__global__ void zero_list_kernel(const ZeroList z) {
  const int k = blockIdx.y;
  uint32_t* __restrict__ d = (uint32_t*)z.p[k];
  const int64_t n = z.bytes[k] / 4;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = 0u;
}

hipError_t launch_zero_list(const ZeroList& z, hipStream_t st) {
  if (z.n <= 0) return hipSuccess;
  if (z.n > MAX_LIST) return hipErrorInvalidValue;
  int64_t most = 0;
  for (int k = 0; k < z.n; ++k) most = z.bytes[k] / 4 > most ? z.bytes[k] / 4 : most;
  hipLaunchKernelGGL(zero_list_kernel, dim3(grid_for(most, 256), z.n), dim3(256), 0, st, z);
  return hipGetLastError();
}

// One float4 per (bone, z, y+1, x+1): the blend weights of the cell's four
// x-y corners in plane z, zero for corners outside the volume.
__global__ void pack_motion_kernel(const float* __restrict__ w, f4* __restrict__ packed, int R, int64_t n) {
  const int64_t R1 = R + 1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int x0 = (int)(e % R1) - 1, y0 = (int)((e / R1) % R1) - 1;
    const int64_t zb = e / (R1 * R1);  // bone * R + z
    const float* plane = w + zb * R * R;  // plane z of bone b: channels are contiguous R^3 blocks
    auto at = [&](int x, int y) { return ((unsigned)x < (unsigned)R && (unsigned)y < (unsigned)R) ? plane[y * R + x] : 0.f; };
    packed[e] = f4{at(x0, y0), at(x0 + 1, y0), at(x0, y0 + 1), at(x0 + 1, y0 + 1)};
  }
}

hipError_t launch_pack_motion(const float* w, f4* packed, int n_bones, int R, hipStream_t st) {
  const int64_t n = (int64_t)n_bones * R * (R + 1) * (R + 1);
  hipLaunchKernelGGL(pack_motion_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, w, packed, R, n);
  return hipGetLastError();
}

// One group per (z, y, x) cell base of a dense level: the rows of its four
// x-y corners in plane z, 2 features each, copied in the table's dtype.
// Dense level blockIdx.y of the list, all levels in one launch.
struct DenseList {
  const void* level[MNR_MAX_LEVELS];
  void* out[MNR_MAX_LEVELS];
  int N[MNR_MAX_LEVELS];
  int n;
};

template <typename TableT>
__global__ void pack_dense_kernel(const DenseList d) {
  const int k = blockIdx.y;
  const TableT* __restrict__ level = (const TableT*)d.level[k];
  TableT* __restrict__ out = (TableT*)d.out[k];
  const int N = d.N[k];
  const int64_t s = N + 1, n = (int64_t)(N + 1) * N * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = e % N, y = (e / N) % N, z = e / ((int64_t)N * N);
    const int64_t r0 = x + s * (y + s * z);
    const int64_t rows[4] = {r0, r0 + 1, r0 + s, r0 + s + 1};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      out[e * 8 + 2 * c] = level[rows[c] * 2];
      out[e * 8 + 2 * c + 1] = level[rows[c] * 2 + 1];
    }
  }
}

hipError_t launch_pack_dense(const FieldArgs& f, mnr_dtype dt, hipStream_t st) {
  const size_t T = (size_t)1 << f.log2_T;
  const size_t esz = dt == MNR_F32 ? 4 : 2;
  DenseList d{};
  int64_t most = 0;
  for (int l = 0; l < f.n_levels; ++l) {
    if (!((f.dense_mask >> l) & 1u)) continue;
    const int N = f.level_res[l];
    d.level[d.n] = (const char*)f.table + (size_t)l * T * 2 * esz;
    d.out[d.n] = (char*)f.dpk + f.dpk_off[l];  // (a byte offset)
    d.N[d.n++] = N;
    const int64_t n = (int64_t)(N + 1) * N * N;
    most = n > most ? n : most;
  }
  if (d.n == 0) return hipSuccess;
  if (dt == MNR_F32)
    hipLaunchKernelGGL(pack_dense_kernel<float>, dim3(grid_for(most, 256), d.n), dim3(256), 0, st, d);
  else
    hipLaunchKernelGGL(pack_dense_kernel<_Float16>, dim3(grid_for(most, 256), d.n), dim3(256), 0, st, d);
  return hipGetLastError();
}
hipError_t launch_zero(void* dst, size_t bytes, hipStream_t st) {
  const int64_t n = (int64_t)(bytes / 4);
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, (uint32_t*)dst, n);
  return hipGetLastError();
}

}  // namespace mnr
