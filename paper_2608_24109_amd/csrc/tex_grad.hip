// Tiled reduction of material-map gradient records (counting sort by tile, LDS sums per chunk of
// a tile, then dtex += the sums: plain read-modify-writes for a tile's only chunk, else atomics).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "exm_internal.h"
#include "tex_grad.h"

namespace exm {
namespace {

constexpr int kThreads = 256;
constexpr int kSortBlocks = 1024;  // grid of the histogram pass
constexpr int kTileFloats = kTexTileW * kTexTileH * 8;  // 64 KB of LDS

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

__device__ __forceinline__ uint32_t n_chunks(uint32_t count) {
  return (uint32_t)((count + kTexChunk - 1) / kTexChunk);
}

// exclusive scans of the tile sizes and of their reduction chunks (one block)
__global__ __launch_bounds__(kThreads) void k_tg_scan(TexGradWs w) {
  __shared__ uint32_t part[kThreads], partc[kThreads];
  const int32_t B = w.n_buckets;
  const int32_t per = (B + kThreads - 1) / kThreads;
  const int32_t b0 = min(B, (int32_t)threadIdx.x * per), b1 = min(B, b0 + per);
  uint32_t s = 0, sc = 0;
  for (int32_t b = b0; b < b1; ++b) {
    s += w.bucket_count[b];
    sc += n_chunks(w.bucket_count[b]);
  }
  part[threadIdx.x] = s;
  partc[threadIdx.x] = sc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0, accc = 0;
    for (int k = 0; k < kThreads; ++k) {
      const uint32_t v = part[k], vc = partc[k];
      part[k] = acc;
      partc[k] = accc;
      acc += v;
      accc += vc;
    }
    w.bucket_off[B] = acc;
    w.chunk_off[B] = accc;
  }
  __syncthreads();
  uint32_t acc = part[threadIdx.x], accc = partc[threadIdx.x];
  for (int32_t b = b0; b < b1; ++b) {
    w.bucket_off[b] = acc;
    w.bucket_cur[b] = acc;
    w.chunk_off[b] = accc;
    const uint32_t nc = n_chunks(w.bucket_count[b]);
    for (uint32_t k = 0; k < nc; ++k) w.chunk_bucket[accc + k] = (uint32_t)b;
    acc += w.bucket_count[b];
    accc += nc;
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

// One block per chunk of a tile's records: w_k * g_c of the taps inside the tile added into LDS,
// then dtex += the nonzero sums (no other tile's records reach these texels). Blocks past the last
// chunk exit at once (the grid is sized for the largest possible chunk count).
__global__ __launch_bounds__(kThreads) void k_tg_reduce(TexGradWs w, float* __restrict__ dtex) {
  __shared__ float acc[kTileFloats];
  const uint32_t c = blockIdx.x;
  const int32_t B = w.n_buckets;
  if (c >= w.chunk_off[B]) return;
  const int32_t b = (int32_t)w.chunk_bucket[c];
  const bool alone = w.chunk_off[b + 1] - w.chunk_off[b] == 1u;
  const uint32_t r0 = w.bucket_off[b] + (uint32_t)((int64_t)(c - w.chunk_off[b]) * kTexChunk);
  const uint32_t r1 = (uint32_t)min((int64_t)w.bucket_off[b + 1], (int64_t)r0 + kTexChunk);
  const int32_t x0 = (b % w.nbx) * kTexTileW, y0 = (b / w.nbx) * kTexTileH;
  for (int32_t k = threadIdx.x; k < kTileFloats / 4; k += kThreads)
    reinterpret_cast<float4*>(acc)[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  __syncthreads();
  for (uint32_t i = r0 + threadIdx.x; i < r1; i += kThreads) {
    const uint4* src = reinterpret_cast<const uint4*>(w.sorted + i);
    const uint4 q0 = src[0], q1 = src[1], q2 = src[2], q3 = src[3];
    const uint32_t col = q0.x & ~kTexStepBit, row = q0.y & ~kTexStepBit;
    const bool dx = (q0.x & kTexStepBit) != 0u, dy = (q0.y & kTexStepBit) != 0u;
    const int32_t lx = (int32_t)col - x0, ly = (int32_t)row - y0;  // in the tile by the bucket
    const float wt[4] = {__uint_as_float(q0.z), __uint_as_float(q0.w), __uint_as_float(q1.x), __uint_as_float(q1.y)};
    const float g[8] = {__uint_as_float(q1.z), __uint_as_float(q1.w), __uint_as_float(q2.x), __uint_as_float(q2.y),
                        __uint_as_float(q2.z), __uint_as_float(q2.w), __uint_as_float(q3.x), __uint_as_float(q3.y)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (wt[k] == 0.0f || !tex_tap_in_tile(k, col, row, dx, dy)) continue;
      const int32_t e = ((ly + ((k & 2) && dy ? 1 : 0)) * kTexTileW + lx + ((k & 1) && dx ? 1 : 0)) * 8;
#pragma unroll
      for (int ch = 0; ch < 8; ++ch)
        if (g[ch] != 0.0f) atomicAdd(&acc[e + ch], wt[k] * g[ch]);
    }
  }
  __syncthreads();
  // dtex += the sums, four floats (half a texel) per lane and kWb of them in flight per thread
  constexpr int kWb = 4;
  static_assert(kTileFloats % (4 * kThreads * kWb) == 0, "whole write-back rounds");
  for (int32_t k0 = threadIdx.x; k0 < kTileFloats / 4; k0 += kThreads * kWb) {
    float4 v[kWb], d[kWb];
    bool in[kWb];
    float4* p[kWb];
#pragma unroll
    for (int u = 0; u < kWb; ++u) {
      const int32_t k = k0 + u * kThreads;  // float4 index: texel k / 2, channels 4 (k & 1) ..
      v[u] = reinterpret_cast<const float4*>(acc)[k];
      const int32_t t = k >> 1, x = x0 + t % kTexTileW, y = y0 + t / kTexTileW;
      in[u] = x < w.Wt && y < w.Ht && (v[u].x != 0.0f || v[u].y != 0.0f || v[u].z != 0.0f || v[u].w != 0.0f);
      p[u] = reinterpret_cast<float4*>(dtex + ((int64_t)y * w.Wt + x) * 8 + 4 * (k & 1));
      if (in[u] && alone) d[u] = *p[u];
    }
#pragma unroll
    for (int u = 0; u < kWb; ++u) {
      if (!in[u]) continue;
      if (alone) {
        *p[u] = make_float4(d[u].x + v[u].x, d[u].y + v[u].y, d[u].z + v[u].z, d[u].w + v[u].w);
      } else {
        float* q = reinterpret_cast<float*>(p[u]);
        if (v[u].x != 0.0f) unsafeAtomicAdd(q, v[u].x);
        if (v[u].y != 0.0f) unsafeAtomicAdd(q + 1, v[u].y);
        if (v[u].z != 0.0f) unsafeAtomicAdd(q + 2, v[u].z);
        if (v[u].w != 0.0f) unsafeAtomicAdd(q + 3, v[u].w);
      }
    }
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
    const int64_t max_chunks = (w.cap + kTexChunk - 1) / kTexChunk + w.n_buckets;  // <= tex_grad_max_chunks
    k_tg_reduce<<<(unsigned)max_chunks, kThreads, 0, s>>>(w, dtex);
  }
  return hipGetLastError();
}

}  // namespace exm
