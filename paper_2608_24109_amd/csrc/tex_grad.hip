// Tiled reduction of material-map gradient records (counting sort by tile; per tile, chunk by
// chunk, a counting sort of the taps by texel in LDS and one thread per texel summing its taps in
// registers; then one plain read-modify-write of the tile in dtex).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "exm_internal.h"
#include "tex_grad.h"

namespace exm {
namespace {

constexpr int kThreads = 256;
constexpr int kSortBlocks = 1024;  // grid of the histogram pass
constexpr int kTexels = kTexTileW * kTexTileH;        // texels of a tile
constexpr int kRecsPerThread = (int)(kTexChunk / kThreads);
static_assert(kTexChunk % kThreads == 0 && kTexels % kThreads == 0, "whole per-thread shares");

__global__ __launch_bounds__(kThreads) void k_tg_clear(uint32_t* counter, uint32_t* bucket_count, int32_t B) {
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i == 0) *counter = 0u;
  if (i <= B) bucket_count[i] = 0u;
}

__device__ __forceinline__ uint32_t n_records(const TexGradWs& w) {
  return (uint32_t)min((int64_t)*w.counter, w.cap);
}

__device__ __forceinline__ uint32_t bucket_of(const TexGradWs& w, uint32_t col, uint32_t row) {
  return ((row & ~kTexStepBit) / kTexTileH) * (uint32_t)w.nbx + (col & ~kTexStepBit) / kTexTileW;
}

// a record whose first tap lies outside the map (not written by the adjoints) is dropped
__device__ __forceinline__ bool valid(const TexGradWs& w, uint32_t col, uint32_t row) {
  return (col & ~kTexStepBit) < (uint32_t)w.Wt && (row & ~kTexStepBit) < (uint32_t)w.Ht;
}

// global tile sizes
__global__ __launch_bounds__(kThreads) void k_tg_hist(TexGradWs w) {
  extern __shared__ uint32_t h[];
  for (int32_t b = threadIdx.x; b < w.n_buckets; b += kThreads) h[b] = 0u;
  __syncthreads();
  const uint32_t n = n_records(w);
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const uint2 cr = *reinterpret_cast<const uint2*>(w.rec + i);
    if (valid(w, cr.x, cr.y)) atomicAdd(&h[bucket_of(w, cr.x, cr.y)], 1u);
  }
  __syncthreads();
  for (int32_t b = threadIdx.x; b < w.n_buckets; b += kThreads)
    if (h[b]) atomicAdd(&w.bucket_count[b], h[b]);
}

// exclusive scan of the tile sizes (one block)
__global__ __launch_bounds__(kThreads) void k_tg_scan(TexGradWs w) {
  __shared__ uint32_t part[kThreads];
  const int32_t B = w.n_buckets;
  const int32_t per = (B + kThreads - 1) / kThreads;
  const int32_t b0 = min(B, (int32_t)threadIdx.x * per), b1 = min(B, b0 + per);
  uint32_t s = 0;
  for (int32_t b = b0; b < b1; ++b) s += w.bucket_count[b];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int k = 0; k < kThreads; ++k) {
      const uint32_t v = part[k];
      part[k] = acc;
      acc += v;
    }
    w.bucket_off[B] = acc;
  }
  __syncthreads();
  uint32_t acc = part[threadIdx.x];
  for (int32_t b = b0; b < b1; ++b) {
    w.bucket_off[b] = acc;
    w.bucket_cur[b] = acc;
    acc += w.bucket_count[b];
  }
}

// Each block owns one contiguous range of the records: it counts its range per tile, reserves
// its share of every tile with one atomic per tile, and places its records in range order (a
// tile's records from one block land in consecutive slots).
__global__ __launch_bounds__(kThreads) void k_tg_scatter(TexGradWs w) {
  extern __shared__ uint32_t h[];
  const int32_t B = w.n_buckets;
  const uint32_t n = n_records(w);
  const uint32_t per = (uint32_t)(((uint64_t)n + gridDim.x - 1) / gridDim.x);
  const uint32_t r0 = (uint32_t)min((uint64_t)blockIdx.x * per, (uint64_t)n);
  const uint32_t r1 = (uint32_t)min((uint64_t)r0 + per, (uint64_t)n);
  for (int32_t b = threadIdx.x; b < B; b += kThreads) h[b] = 0u;
  __syncthreads();
  for (uint32_t i = r0 + threadIdx.x; i < r1; i += kThreads) {
    const uint2 cr = *reinterpret_cast<const uint2*>(w.rec + i);
    if (valid(w, cr.x, cr.y)) atomicAdd(&h[bucket_of(w, cr.x, cr.y)], 1u);
  }
  __syncthreads();
  for (int32_t b = threadIdx.x; b < B; b += kThreads)
    if (h[b]) h[b] = atomicAdd(&w.bucket_cur[b], h[b]);
  __syncthreads();
  for (uint32_t i = r0 + threadIdx.x; i < r1; i += kThreads) {
    const uint4* src = reinterpret_cast<const uint4*>(w.rec + i);
    const uint4 q0 = src[0], q1 = src[1], q2 = src[2], q3 = src[3];
    if (!valid(w, q0.x, q0.y)) continue;
    const uint32_t slot = atomicAdd(&h[bucket_of(w, q0.x, q0.y)], 1u);
    uint4* dst = reinterpret_cast<uint4*>(w.sorted + slot);
    dst[0] = q0;
    dst[1] = q1;
    dst[2] = q2;
    dst[3] = q3;
  }
}

// One block per tile (LDS: a chunk's weights and gradients 48 KB, per-texel counts and offsets
// 16 KB, the (record, tap) lists 8 KB). The tile's records are taken kTexChunk at a time; each
// thread owns kTexels / kThreads texels and keeps their sums in registers across the chunks, so
// the block ends with one plain read-modify-write of the tile in dtex (no other block's records
// reach it; device-scope float atomics into dtex cost six times the whole reduction).
__global__ __launch_bounds__(kThreads) void k_tg_reduce(TexGradWs w, float* __restrict__ dtex) {
  __shared__ float4 lw[kTexChunk];        // weights of the chunk's records
  __shared__ float4 lg[2 * kTexChunk];    // gradients of the chunk's records
  __shared__ uint32_t cnt[kTexels], off[kTexels];
  __shared__ uint16_t list[4 * kTexChunk];  // record index * 4 + tap, grouped by texel
  __shared__ uint32_t wsum[kThreads / 64];
  constexpr int kOwn = kTexels / kThreads;  // texels per thread: threadIdx.x + v * kThreads
  const int32_t b = blockIdx.x;
  const uint32_t rb0 = w.bucket_off[b], rb1 = w.bucket_off[b + 1];
  if (rb0 == rb1) return;
  const int32_t x0 = (b % w.nbx) * kTexTileW, y0 = (b / w.nbx) * kTexTileH;
  float a[kOwn][8];
#pragma unroll
  for (int v = 0; v < kOwn; ++v)
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) a[v][ch] = 0.0f;
  for (uint32_t r0 = rb0; r0 < rb1; r0 += (uint32_t)kTexChunk) {
    const uint32_t n = min(rb1 - r0, (uint32_t)kTexChunk);
    for (int32_t t = threadIdx.x; t < kTexels; t += kThreads) cnt[t] = 0u;
    __syncthreads();
    // stage the records; count each tap inside the tile at its texel (rank = its place there)
    uint32_t tr[kRecsPerThread][4];  // texel << 16 | rank, or 0xFFFFFFFF
#pragma unroll
    for (int u = 0; u < kRecsPerThread; ++u) {
      const uint32_t i = threadIdx.x + (uint32_t)(u * kThreads);
#pragma unroll
      for (int k = 0; k < 4; ++k) tr[u][k] = 0xFFFFFFFFu;
      if (i >= n) continue;
      const uint4* src = reinterpret_cast<const uint4*>(w.sorted + r0 + i);
      const uint4 q0 = src[0], q1 = src[1], q2 = src[2], q3 = src[3];
      const float wt[4] = {__uint_as_float(q0.z), __uint_as_float(q0.w), __uint_as_float(q1.x),
                           __uint_as_float(q1.y)};
      lw[i] = make_float4(wt[0], wt[1], wt[2], wt[3]);
      lg[2 * i] =
          make_float4(__uint_as_float(q1.z), __uint_as_float(q1.w), __uint_as_float(q2.x), __uint_as_float(q2.y));
      lg[2 * i + 1] =
          make_float4(__uint_as_float(q2.z), __uint_as_float(q2.w), __uint_as_float(q3.x), __uint_as_float(q3.y));
      const uint32_t col = q0.x & ~kTexStepBit, row = q0.y & ~kTexStepBit;
      const bool dx = (q0.x & kTexStepBit) != 0u, dy = (q0.y & kTexStepBit) != 0u;
      const int32_t lx = (int32_t)col - x0, ly = (int32_t)row - y0;  // in the tile by the bucket
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (wt[k] == 0.0f || !tex_tap_in_tile(k, col, row, dx, dy)) continue;
        const uint32_t t = (uint32_t)((ly + ((k & 2) && dy ? 1 : 0)) * kTexTileW + lx + ((k & 1) && dx ? 1 : 0));
        tr[u][k] = t << 16 | atomicAdd(&cnt[t], 1u);
      }
    }
    __syncthreads();
    // exclusive scan of the counts (kTexels / kThreads consecutive texels per thread)
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < kOwn; ++q) sum += cnt[threadIdx.x * kOwn + q];
    uint32_t x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if ((int)__lane_id() >= o) x += y;
    }
    if (__lane_id() == 63) wsum[threadIdx.x >> 6] = x;
    __syncthreads();
    uint32_t acc0 = x - sum;
    for (uint32_t q = 0; q < (threadIdx.x >> 6); ++q) acc0 += wsum[q];
#pragma unroll
    for (int q = 0; q < kOwn; ++q) {
      off[threadIdx.x * kOwn + q] = acc0;
      acc0 += cnt[threadIdx.x * kOwn + q];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kRecsPerThread; ++u)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (tr[u][k] != 0xFFFFFFFFu)
          list[off[tr[u][k] >> 16] + (tr[u][k] & 0xFFFFu)] =
              (uint16_t)(((threadIdx.x + (uint32_t)(u * kThreads)) << 2) | (uint32_t)k);
    __syncthreads();
    // each thread adds the listed taps of its texels to their sums
#pragma unroll
    for (int v = 0; v < kOwn; ++v) {
      const int32_t t = threadIdx.x + v * kThreads;
      const uint32_t e0 = off[t], e1 = e0 + cnt[t];
      for (uint32_t e = e0; e < e1; ++e) {
        const uint32_t code = list[e], i = code >> 2;
        const float wk = reinterpret_cast<const float*>(lw)[4 * i + (code & 3u)];
        const float4 g0 = lg[2 * i], g1 = lg[2 * i + 1];
        a[v][0] += wk * g0.x;
        a[v][1] += wk * g0.y;
        a[v][2] += wk * g0.z;
        a[v][3] += wk * g0.w;
        a[v][4] += wk * g1.x;
        a[v][5] += wk * g1.y;
        a[v][6] += wk * g1.z;
        a[v][7] += wk * g1.w;
      }
    }
    __syncthreads();  // before the next chunk reuses the staging arrays
  }
  // dtex += the tile's sums (texels outside the map get no taps: the taps are clamped to it)
#pragma unroll
  for (int v = 0; v < kOwn; ++v) {
    const int32_t t = threadIdx.x + v * kThreads;
    const int32_t xx = x0 + t % kTexTileW, yy = y0 + t / kTexTileW;
    bool any = false;
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) any |= a[v][ch] != 0.0f;
    if (!any || xx >= w.Wt || yy >= w.Ht) continue;
    float4* d = reinterpret_cast<float4*>(dtex + ((int64_t)yy * w.Wt + xx) * 8);
    const float4 d0 = d[0], d1 = d[1];
    d[0] = make_float4(d0.x + a[v][0], d0.y + a[v][1], d0.z + a[v][2], d0.w + a[v][3]);
    d[1] = make_float4(d1.x + a[v][4], d1.y + a[v][5], d1.z + a[v][6], d1.w + a[v][7]);
  }
}

}  // namespace

hipError_t launch_tex_grad_clear(const TexGradWs& w, hipStream_t s) {
  const int32_t n = w.n_buckets + 1;
  k_tg_clear<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(w.counter, w.bucket_count, w.n_buckets);
  return hipGetLastError();
}

hipError_t launch_tex_grad_reduce(const TexGradWs& w, float* dtex, hipStream_t s) {
  if (w.n_buckets > kTexMaxBuckets || w.n_buckets < 1) return hipErrorInvalidValue;
  const size_t lds = (size_t)w.n_buckets * 4;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(kSortBlocks, (w.cap + kThreads - 1) / kThreads));
  {
    EXM_TIMED("tex_grad_sort", s);
    k_tg_hist<<<grid, kThreads, lds, s>>>(w);
    k_tg_scan<<<1, kThreads, 0, s>>>(w);
    int dev = 0, cus = 256, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipGetLastError();
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return hipGetLastError();
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_tg_scatter, kThreads, lds) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    const unsigned sg = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((int64_t)cus * per_cu, (w.cap + kThreads - 1) / kThreads));
    k_tg_scatter<<<sg, kThreads, lds, s>>>(w);
  }
  {
    EXM_TIMED("tex_grad_reduce", s);
    k_tg_reduce<<<(unsigned)w.n_buckets, kThreads, 0, s>>>(w, dtex);
  }
  return hipGetLastError();
}

}  // namespace exm
