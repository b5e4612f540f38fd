// Binned scatter-add of the grid-table gradient (training, Sec. 5.2).
//
// The adjoint's gradient with respect to the grid table is a scatter-add:
// every evaluated sample adds to 8 rows of each level.  On the hashed levels
// the rows are spread over the whole table by the spatial hash, so
// consecutive samples of a ray almost never share one; on the dense levels
// the adjoint first sums runs of consecutive samples in one cell.  Done with
// global float atomics, which this GPU executes at the memory side at
// ~20 G/s, the scatter costs more than the rest of the adjoint.  Instead the
// adjoint writes one record (key, two feature gradients) per sample (per run
// on a dense level), level and corner, and the records are summed here
// without global float atomics:
//   1. bin_histogram: per tile of records, a histogram of the key bins
//      (a bin = 2^shift consecutive keys, up to a 128 KiB slice of the table
//      gradient), written tile-major to H[tile][bin] (one contiguous row per
//      tile: thousands of bins make a bin-major layout's column writes and
//      reads the slowest part of the pipeline);
//   2. bin_segsum / bin_total / bin_scan / bin_offsets: exclusive scan of H in (bin,
//      tile) order, per bin over BIN_SEGS segments of tiles in parallel,
//      giving every (bin, tile) pair its place in bin order, and the list of
//      summing items (a bin of t records is ceil(t / ACC_PART_RECORDS)
//      items: the coarse dense levels pack millions of records into a few
//      bins);
//   3. bin_scatter: each tile sorts its records by bin in LDS and writes
//      them to their places, bin run by bin run;
//   4. bin_accumulate: one block per item sums its records into an LDS copy
//      of the bin's slice (64-bit fixed point, integer LDS atomics), then
//      adds the slice to the table gradient (a bin of one item has one
//      owner: plain read-add-write; the items of a split bin add with float
//      atomics, a few thousand per item).
// The key map (KeyMap) numbers the hashed levels' rows (T keys per level),
// then the dense levels' ((N+1)^3 keys per level), so no bin is spent on
// rows a dense level does not have; then, from a bin-aligned start, the
// elements of the blend-weight gradient dL/dW^c (Eq. 7), whose records carry
// two x-adjacent cell corners each.  Traffic is a few passes over the
// records (12 bytes each) instead of two memory-side atomics per record.
#include <cfloat>

#include "kernels.h"

namespace mnr {

constexpr int BIN_THREADS = 1024;
constexpr int BIN_TILE = BIN_TILE_RECORDS;  // records per tile
constexpr int BIN_PER_THREAD = BIN_TILE / BIN_THREADS;
constexpr int ACC_THREADS = 1024;           // the per-bin sums
constexpr int ACC_SHIFT = 12;               // rows per summing block: 2^12 x 2 features x 8 bytes = 64 KiB of LDS

int scatter_bin_shift(int64_t n_keys) {
  // bins of 2^12 keys (one summing block each, 64 KiB of fixed-point sums
  // in LDS: two blocks per CU), larger only when that would make more than
  // MAX_BINS of them (their blocks then sum 2^12-row parts)
  int shift = ACC_SHIFT;
  while ((n_keys + ((int64_t)1 << shift) - 1) >> shift > MAX_BINS) ++shift;
  return shift;
}

// Records written: the adjoint reserves space with the cursor and writes
// nothing past the capacity, so the count is clamped to it.
__device__ __forceinline__ uint32_t record_count(const uint32_t* cursor, uint32_t cap) {
  const uint32_t c = *cursor;
  return c < cap ? c : cap;
}

__global__ void __launch_bounds__(BIN_THREADS) bin_histogram_kernel(const uint32_t* __restrict__ cursor, uint32_t cap,
                                                                    const uint32_t* __restrict__ keys, int shift,
                                                                    int n_bins, uint32_t* __restrict__ H) {
  __shared__ uint32_t hist[MAX_BINS];
  const uint32_t count = record_count(cursor, cap);
  const int tile = blockIdx.x;
  if ((int64_t)tile * BIN_TILE >= count) return;
  for (int b = threadIdx.x; b < n_bins; b += BIN_THREADS) hist[b] = 0;
  __syncthreads();
  const uint32_t t0 = (uint32_t)tile * BIN_TILE;
  uint32_t k[BIN_PER_THREAD];
  // loads from clamped places, then the range test: all of a thread's
  // loads are in flight together instead of one branch and wait per load
#pragma unroll
  for (int j = 0; j < BIN_PER_THREAD; ++j) {
    const uint32_t i = t0 + j * BIN_THREADS + threadIdx.x;
    k[j] = keys[i < count ? i : count - 1];
  }
#pragma unroll
  for (int j = 0; j < BIN_PER_THREAD; ++j) {
    const uint32_t i = t0 + j * BIN_THREADS + threadIdx.x;
    k[j] = i < count ? k[j] >> shift : 0xFFFFFFFFu;
  }
  // The dense levels' records come in long stretches of one bin: the lanes
  // that share the first lane's bin add once, through one lane.
  const int lane = (int)(threadIdx.x & (WAVE - 1));
#pragma unroll
  for (int j = 0; j < BIN_PER_THREAD; ++j) {
    const uint32_t b0 = __builtin_amdgcn_readfirstlane(k[j]);
    const bool same = k[j] == b0;
    const uint64_t m = __ballot(same);
    if (k[j] < (uint32_t)n_bins) {  // keys are < n_keys by construction
      if (!same)
        atomicAdd(&hist[k[j]], 1u);
      else if (lane == __ffsll((unsigned long long)m) - 1)
        atomicAdd(&hist[b0], (uint32_t)__popcll(m));
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < n_bins; b += BIN_THREADS) H[(size_t)tile * n_bins + b] = hist[b];
}

// Summing items of a bin of n records.
__device__ __forceinline__ uint32_t bin_items(uint32_t n) {
  return (n + ACC_PART_RECORDS - 1) / ACC_PART_RECORDS;
}

// Tiles of segment s (the per-bin scans over tiles run in BIN_SEGS
// segments, one block per segment and BIN_SCAN_BINS bins).
__device__ __forceinline__ void segment_tiles(uint32_t count, int s, int& t0, int& t1) {
  const int n_tiles = (int)((count + BIN_TILE - 1) / BIN_TILE);
  const int per = (n_tiles + BIN_SEGS - 1) / BIN_SEGS;
  t0 = min(n_tiles, s * per);
  t1 = min(n_tiles, t0 + per);
}

// seg[s][b] = records of bin b in the tiles of segment s.
__global__ void __launch_bounds__(BIN_SCAN_BINS) bin_segsum_kernel(const uint32_t* __restrict__ cursor, uint32_t cap,
                                                                  const uint32_t* __restrict__ H, int n_bins,
                                                                  uint32_t* __restrict__ seg) {
  const int b = blockIdx.x * BIN_SCAN_BINS + threadIdx.x, s = blockIdx.y;
  if (b >= n_bins) return;
  int t0, t1;
  segment_tiles(record_count(cursor, cap), s, t0, t1);
  uint32_t sum = 0;
#pragma unroll 8
  for (int t = t0; t < t1; ++t) sum += H[(size_t)t * n_bins + b];
  seg[(size_t)s * n_bins + b] = sum;
}

// total[b] = records of bin b (the sum of its segments' counts).
__global__ void __launch_bounds__(BIN_SCAN_BINS) bin_total_kernel(const uint32_t* __restrict__ seg, int n_bins,
                                                                 uint32_t* __restrict__ total) {
  const int b = blockIdx.x * BIN_SCAN_BINS + threadIdx.x;
  if (b >= n_bins) return;
  uint32_t sum = 0;
#pragma unroll
  for (int s = 0; s < BIN_SEGS; ++s) sum += seg[(size_t)s * n_bins + b];
  total[b] = sum;
}

// One block: base[b] = records of the bins before b; the summing items:
// item_base[b] = items of the bins before b, item_bin[item_base[b] + j] = b
// for the bin's items j, and their count.
constexpr int BIN_SCAN_THREADS = 1024;
__global__ void __launch_bounds__(BIN_SCAN_THREADS) bin_scan_kernel(const uint32_t* __restrict__ total, int n_bins,
                                                                   uint32_t* __restrict__ base,
                                                                   uint32_t* __restrict__ item_base,
                                                                   uint32_t* __restrict__ item_bin,
                                                                   uint32_t* __restrict__ n_items) {
  __shared__ uint32_t red[2][BIN_SCAN_THREADS / WAVE];
  constexpr int PER = MAX_BINS / BIN_SCAN_THREADS;  // consecutive bins per thread
  const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x >> 6;
  uint32_t tot[PER], rec = 0, items = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int b = threadIdx.x * PER + j;
    tot[j] = b < n_bins ? total[b] : 0u;
    rec += tot[j];
    items += bin_items(tot[j]);
  }
  // exclusive scans of (records, items) over the threads' bin groups
  uint32_t ir = rec, ii = items;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t o1 = __shfl_up(ir, d, WAVE), o2 = __shfl_up(ii, d, WAVE);
    if (lane >= d) { ir += o1; ii += o2; }
  }
  if (lane == WAVE - 1) { red[0][wave] = ir; red[1][wave] = ii; }
  __syncthreads();
  uint32_t r0 = ir - rec, i0 = ii - items;
  for (int w = 0; w < wave; ++w) { r0 += red[0][w]; i0 += red[1][w]; }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int b = threadIdx.x * PER + j;
    if (b >= n_bins) break;
    base[b] = r0;
    item_base[b] = i0;
    const uint32_t nb = bin_items(tot[j]);
    for (uint32_t k = 0; k < nb; ++k) item_bin[i0 + k] = (uint32_t)b;
    r0 += tot[j];
    i0 += nb;
    if (b == n_bins - 1) *n_items = i0;
  }
}

// H[t][b] becomes the place of tile t's first record of bin b (records in
// (bin, tile) order).
__global__ void __launch_bounds__(BIN_SCAN_BINS) bin_offsets_kernel(const uint32_t* __restrict__ cursor, uint32_t cap,
                                                                   uint32_t* __restrict__ H, int n_bins,
                                                                   const uint32_t* __restrict__ seg,
                                                                   const uint32_t* __restrict__ base) {
  const int b = blockIdx.x * BIN_SCAN_BINS + threadIdx.x, s = blockIdx.y;
  if (b >= n_bins) return;
  int t0, t1;
  segment_tiles(record_count(cursor, cap), s, t0, t1);
  uint32_t run = base[b];
  for (int q = 0; q < s; ++q) run += seg[(size_t)q * n_bins + b];  // the bin's records in earlier segments
#pragma unroll 8
  for (int t = t0; t < t1; ++t) {
    const uint32_t v = H[(size_t)t * n_bins + b];
    H[(size_t)t * n_bins + b] = run;
    run += v;
  }
}

// Tile of scatter block i: the 8 XCDs take contiguous ranges of tiles
// (block i runs on XCD i mod 8), so that a bin's records from neighbouring
// tiles, which land next to each other, are written through one L2.
__device__ __forceinline__ int scatter_tile(uint32_t count) {
  const int n_tiles = (int)((count + BIN_TILE - 1) / BIN_TILE);
  const int per = (n_tiles + 7) / 8;
  const int j = (int)(blockIdx.x >> 3);
  return j < per ? (int)(blockIdx.x & 7) * per + j : n_tiles;
}

// Each tile's records are first sorted by bin in LDS (a counting sort), then
// written out bin run by bin run, so that consecutive lanes write
// consecutive places (about BIN_TILE / n_bins records per run).
constexpr int SCATTER_LDS = MAX_BINS * 4 * 2 + BIN_TILE * (4 + 8);

__global__ void __launch_bounds__(BIN_THREADS) bin_scatter_kernel(const uint32_t* __restrict__ cursor, uint32_t cap,
                                                                  const uint32_t* __restrict__ keys,
                                                                  const f2* __restrict__ vals, int shift, int n_bins,
                                                                  const uint32_t* __restrict__ H,
                                                                  uint32_t* __restrict__ skeys,
                                                                  f2* __restrict__ svals) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  uint32_t* start = (uint32_t*)lds;            // [n_bins] first local place of each bin
  uint32_t* cur = start + MAX_BINS;            // [n_bins] counts, then global places
  uint32_t* lkeys = cur + MAX_BINS;            // [BIN_TILE] records in bin order
  f2* lvals = (f2*)(lkeys + BIN_TILE);
  __shared__ uint32_t red[BIN_THREADS / WAVE];
  const uint32_t count = record_count(cursor, cap);
  const int tile = scatter_tile(count);
  if ((int64_t)tile * BIN_TILE >= count) return;
  const uint32_t t0 = (uint32_t)tile * BIN_TILE;
  const int n_here = (int)min((uint32_t)BIN_TILE, count - t0);
  for (int b = threadIdx.x; b < n_bins; b += BIN_THREADS) cur[b] = 0;
  __syncthreads();
  uint32_t k[BIN_PER_THREAD], rank[BIN_PER_THREAD];
  f2 v[BIN_PER_THREAD];
#pragma unroll
  for (int j = 0; j < BIN_PER_THREAD; ++j) {
    const int i = j * BIN_THREADS + threadIdx.x;
    k[j] = i < n_here ? keys[t0 + i] : 0xFFFFFFFFu;
    v[j] = i < n_here ? vals[t0 + i] : f2{0.f, 0.f};
  }
  // ranks within the bin; the lanes that share the first lane's bin take
  // one block of consecutive ranks through one lane (in lane order)
  const int lane = (int)(threadIdx.x & (WAVE - 1));
#pragma unroll
  for (int j = 0; j < BIN_PER_THREAD; ++j) {
    const uint32_t b = k[j] >> shift;
    const uint32_t b0 = __builtin_amdgcn_readfirstlane(b);
    const bool same = b == b0;
    const uint64_t m = __ballot(same);
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t got = 0;
    if (b < (uint32_t)n_bins) {
      if (!same)
        got = atomicAdd(&cur[b], 1u);
      else if (lane == leader)
        got = atomicAdd(&cur[b], (uint32_t)__popcll(m));
    }
    const uint32_t first = __shfl(got, leader, WAVE);
    rank[j] = same ? first + (uint32_t)__popcll(m & ((1ull << lane) - 1ull)) : got;
  }
  __syncthreads();
  // exclusive scan of the counts: start[b]
  const int per = (n_bins + BIN_THREADS - 1) / BIN_THREADS;
  const int b0 = threadIdx.x * per;
  uint32_t local = 0;
  for (int b = b0; b < b0 + per && b < n_bins; ++b) local += cur[b];
  uint32_t incl = local;  // inclusive scan of the per-thread sums across the block
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t o = __shfl_up(incl, d, WAVE);
    if ((int)(threadIdx.x & 63) >= d) incl += o;
  }
  if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = incl;
  __syncthreads();
  uint32_t wave_base = 0;
  for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wave_base += red[w];
  uint32_t run = wave_base + incl - local;
  for (int b = b0; b < b0 + per && b < n_bins; ++b) {
    start[b] = run;
    run += cur[b];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < BIN_PER_THREAD; ++j) {
    const uint32_t b = k[j] >> shift;
    if (b < (uint32_t)n_bins) {
      const uint32_t p = start[b] + rank[j];
      lkeys[p] = k[j];
      lvals[p] = v[j];
    }
  }
  __shared__ uint32_t n_sorted;
  if (threadIdx.x == 0) n_sorted = start[n_bins - 1] + cur[n_bins - 1];
  __syncthreads();
  for (int b = threadIdx.x; b < n_bins; b += BIN_THREADS) cur[b] = H[(size_t)tile * n_bins + b];
  __syncthreads();
  for (int p = threadIdx.x; p < (int)n_sorted; p += BIN_THREADS) {
    const uint32_t kk = lkeys[p];
    const uint32_t b = kk >> shift;
    if (b < (uint32_t)n_bins) {
      const uint32_t g = cur[b] + ((uint32_t)p - start[b]);
      skeys[g] = kk;
      svals[g] = lvals[p];
    }
  }
}

// One block per item of a bin (and per 2^ACC_SHIFT-row part of the bin when
// bins are larger): the slice's sums in LDS as 64-bit fixed point.  LDS
// float atomics on this GPU are ~40x slower than integer ones, so every
// value is scaled by a power of two chosen from a bound M on the values'
// magnitudes (the adjoint's largest table or blend-weight record value) and
// the item's record count (n M < 2^62: no sum can overflow), rounded to an
// integer and added with integer atomics.  The integer sums are exact, so a
// bin summed by one item does not depend on the order of its records; each
// value is rounded once, by at most n M 2^-63 (for n = 2^16 records, 1e-14
// of the largest value).  The items of a split bin add their (exact) sums to
// the gradient with float atomics.  If M is not finite the values are summed
// in floats instead.  Keys map to table rows or dL/dW^c elements through
// the key map.
__global__ void __launch_bounds__(ACC_THREADS) bin_accumulate_kernel(const uint32_t* __restrict__ skeys,
                                                                     const f2* __restrict__ svals, int shift,
                                                                     const uint32_t* __restrict__ total,
                                                                     const uint32_t* __restrict__ base,
                                                                     const uint32_t* __restrict__ item_base,
                                                                     const uint32_t* __restrict__ item_bin,
                                                                     const uint32_t* __restrict__ n_items,
                                                                     const uint32_t* __restrict__ vmax,
                                                                     const KeyMap map, float* __restrict__ grad,
                                                                     float* __restrict__ grad_w) {
  extern __shared__ unsigned long long acc[];  // [2][rows]: the two features in separate planes
  const int parts_log2 = shift > ACC_SHIFT ? shift - ACC_SHIFT : 0;
  const uint32_t item = blockIdx.x >> parts_log2;
  const int part = blockIdx.x & ((1 << parts_log2) - 1);
  if (item >= *n_items) return;
  const uint32_t b = item_bin[item];
  const uint32_t n_bin = total[b];
  const uint32_t r0 = (item - item_base[b]) * (uint32_t)ACC_PART_RECORDS;  // the item's first record in the bin
  const uint32_t n = min(n_bin - r0, (uint32_t)ACC_PART_RECORDS);
  const bool shared = n_bin > (uint32_t)ACC_PART_RECORDS;  // other items add to the same rows
  const int rows = 1 << (shift - parts_log2);
  const uint32_t lo = (uint32_t)part * rows, kmask = (1u << shift) - 1u;
  const uint32_t s0 = base[b] + r0;
  const int64_t k0 = ((int64_t)b << shift) + lo;
  const bool wc_slice = k0 >= (int64_t)map.wc_start && k0 < (int64_t)map.wc_end;
  const float M = __uint_as_float(vmax[wc_slice ? 1 : 0]);
  if (M == 0.f) return;  // every value is zero
  for (int i = threadIdx.x; i < 2 * rows; i += ACC_THREADS) acc[i] = 0ull;
  __syncthreads();
  const bool fixed = M <= FLT_MAX;
  int e = 0;
  frexp((double)M * (double)n, &e);  // M n < 2^e
  const double scale = ldexp(1.0, 62 - e);
  float* accf = (float*)acc;  // float sums (a non-finite value in the item)
  constexpr int U = 8;  // records in flight per thread
  for (uint32_t i0 = 0; i0 < n; i0 += U * ACC_THREADS) {
    uint32_t r[U];
    f2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {  // clamped places: the U loads are in flight together
      const uint32_t i = i0 + u * ACC_THREADS + threadIdx.x;
      const uint32_t ic = s0 + (i < n ? i : n - 1);
      r[u] = skeys[ic];
      v[u] = svals[ic];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = i0 + u * ACC_THREADS + threadIdx.x;
      const uint32_t row = (r[u] & kmask) - lo;
      if (i >= n || row >= (uint32_t)rows) continue;
      if (fixed) {
        atomicAdd(&acc[row], (unsigned long long)(long long)rint((double)v[u][0] * scale));
        atomicAdd(&acc[rows + row], (unsigned long long)(long long)rint((double)v[u][1] * scale));
      } else {
        atomicAdd(&accf[row], v[u][0]);
        atomicAdd(&accf[rows + row], v[u][1]);
      }
    }
  }
  __syncthreads();
  if (wc_slice) {
    // dL/dW^c: element k0 + r takes plane 0 of its own key and plane 1 of
    // the key before (the pair's second corner); pairs never cross slices
    for (int r = threadIdx.x; r < rows; r += ACC_THREADS) {
      const int64_t key = k0 + r;
      float v;
      if (fixed) {
        const long long s = (long long)acc[r] + (r > 0 ? (long long)acc[rows + r - 1] : 0ll);
        v = (float)((double)s / scale);
      } else {
        v = accf[r] + (r > 0 ? accf[rows + r - 1] : 0.f);
      }
      if (v != 0.f && key < (int64_t)map.wc_end) {
        float* g = grad_w + (key - map.wc_start);
        if (shared) unsafeAtomicAdd(g, v);
        else *g += v;
      }
    }
    return;
  }
  for (int r = threadIdx.x; r < rows; r += ACC_THREADS) {
    const f2 v = fixed ? f2{(float)((double)(long long)acc[r] / scale), (float)((double)(long long)acc[rows + r] / scale)}
                       : f2{accf[r], accf[rows + r]};
    const int64_t key = k0 + r;
    if ((v[0] != 0.f || v[1] != 0.f) && key < (int64_t)map.start[map.n]) {
      int j = 0;
      while (j + 1 < map.n && (uint32_t)key >= map.start[j + 1]) ++j;
      const int64_t row = ((int64_t)map.level[j] << map.log2_T) + ((uint32_t)key - map.start[j]);
      float* g = grad + 2 * row;
      if (shared) {
        unsafeAtomicAdd(g, v[0]);
        unsafeAtomicAdd(g + 1, v[1]);
      } else {
        *(f2*)g = *(f2*)g + v;
      }
    }
  }
}

hipError_t launch_binned_scatter(const ScatterPlan& p, float* grad_table, float* grad_weights, hipStream_t st) {
  const int parts_log2 = p.shift > ACC_SHIFT ? p.shift - ACC_SHIFT : 0;
  const int lds = (2 << (p.shift - parts_log2)) * (int)sizeof(unsigned long long);
  static PersistentGrid once_acc, once_sc;  // raise the LDS limits once
  persistent_blocks(bin_accumulate_kernel, ACC_THREADS, (2 << ACC_SHIFT) * (int)sizeof(unsigned long long), once_acc);
  persistent_blocks(bin_scatter_kernel, BIN_THREADS, SCATTER_LDS, once_sc);
  hipLaunchKernelGGL(bin_histogram_kernel, dim3(p.n_tiles_cap), dim3(BIN_THREADS), 0, st, p.cursor, p.cap, p.keys,
                     p.shift, p.n_bins, p.hist);
  const dim3 seg_grid((p.n_bins + BIN_SCAN_BINS - 1) / BIN_SCAN_BINS, BIN_SEGS);
  hipLaunchKernelGGL(bin_segsum_kernel, seg_grid, dim3(BIN_SCAN_BINS), 0, st, p.cursor, p.cap, p.hist, p.n_bins,
                     p.seg);
  hipLaunchKernelGGL(bin_total_kernel, dim3(seg_grid.x), dim3(BIN_SCAN_BINS), 0, st, p.seg, p.n_bins, p.total);
  hipLaunchKernelGGL(bin_scan_kernel, dim3(1), dim3(BIN_SCAN_THREADS), 0, st, p.total, p.n_bins, p.base,
                     p.item_base, p.item_bin, p.n_items);
  hipLaunchKernelGGL(bin_offsets_kernel, seg_grid, dim3(BIN_SCAN_BINS), 0, st, p.cursor, p.cap, p.hist, p.n_bins,
                     p.seg, p.base);
  hipLaunchKernelGGL(bin_scatter_kernel, dim3((p.n_tiles_cap + 7) / 8 * 8), dim3(BIN_THREADS), SCATTER_LDS, st, p.cursor, p.cap,
                     p.keys, p.vals, p.shift, p.n_bins, p.hist, p.skeys, p.svals);
  hipLaunchKernelGGL(bin_accumulate_kernel, dim3((unsigned)p.max_items << parts_log2), dim3(ACC_THREADS), lds, st,
                     p.skeys, p.svals, p.shift, p.total, p.base, p.item_base, p.item_bin, p.n_items, p.vmax, p.map,
                     grad_table, grad_weights);
  return hipGetLastError();
}

}  // namespace mnr
