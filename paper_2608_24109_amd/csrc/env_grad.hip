// Binned reduction of env-gradient records (counting sort by bucket, LDS sums per chunk of a bucket).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "env_grad.h"
#include "exm_internal.h"

namespace exm {
namespace {

constexpr int kThreads = 256;
constexpr int kSortBlocks = 1024;     // grid of the histogram and scatter passes
constexpr int kMaxLdsBuckets = 8192;  // He * We <= 2^24 texels

__global__ __launch_bounds__(kThreads) void k_eg_clear(uint32_t* counter, uint32_t* bucket_count, int32_t B) {
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i == 0) *counter = 0u;
  if (i <= B) bucket_count[i] = 0u;
}

// unused slots carry kNoTexel; any other texel outside the buckets is dropped as well
__device__ __forceinline__ bool valid(const EnvGradWs& w, uint32_t t) {
  return (t >> kBucketShift) < (uint32_t)w.n_buckets;
}

__device__ __forceinline__ uint32_t n_records(const EnvGradWs& w) {
  return (uint32_t)min((int64_t)*w.counter, w.cap);
}

// global bucket sizes
__global__ __launch_bounds__(kThreads) void k_eg_hist(EnvGradWs w) {
  __shared__ uint32_t h[kMaxLdsBuckets];
  for (int32_t b = threadIdx.x; b < w.n_buckets; b += kThreads) h[b] = 0u;
  __syncthreads();
  const uint32_t n = n_records(w);
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const uint32_t t = w.rec[i].texel;
    if (valid(w, t)) atomicAdd(&h[t >> kBucketShift], 1u);
  }
  __syncthreads();
  for (int32_t b = threadIdx.x; b < w.n_buckets; b += kThreads)
    if (h[b]) atomicAdd(&w.bucket_count[b], h[b]);
}

// records in flight per thread in the histogram and reduction loops (indices stay below 2^32:
// a chunk holds fewer than 2^31 records)
constexpr int kLoads = 8;

// Contiguous record range of block g of a G-block tiled pass (the histogram and the scatter split
// the records the same way).
__device__ __forceinline__ void block_range(uint32_t n, uint32_t g, uint32_t G, uint32_t* r0, uint32_t* r1) {
  const uint32_t per = (uint32_t)(((uint64_t)n + G - 1) / G);
  *r0 = (uint32_t)min((uint64_t)g * per, (uint64_t)n);
  *r1 = (uint32_t)min((uint64_t)*r0 + per, (uint64_t)n);
}

// bucket sizes of each block's range (all B entries of the block's row) and the global sizes
__global__ __launch_bounds__(kThreads) void k_eg_hist_blocks(EnvGradWs w) {
  __shared__ uint32_t h[kTileMaxBuckets];
  const int32_t B = w.n_buckets;
  for (int32_t b = threadIdx.x; b < B; b += kThreads) h[b] = 0u;
  __syncthreads();
  uint32_t r0, r1;
  block_range(n_records(w), blockIdx.x, gridDim.x, &r0, &r1);
  // kLoads records per thread loaded together before their LDS atomics (a load followed by its
  // atomic waits for memory once per record)
  uint32_t i = r0 + threadIdx.x;
  for (; i + (kLoads - 1) * kThreads < r1; i += kLoads * kThreads) {
    uint32_t t[kLoads];
#pragma unroll
    for (int k = 0; k < kLoads; ++k) t[k] = w.rec[i + k * kThreads].texel;
#pragma unroll
    for (int k = 0; k < kLoads; ++k)
      if (valid(w, t[k])) atomicAdd(&h[t[k] >> kBucketShift], 1u);
  }
  for (; i < r1; i += kThreads) {
    const uint32_t t = w.rec[i].texel;
    if (valid(w, t)) atomicAdd(&h[t >> kBucketShift], 1u);
  }
  __syncthreads();
  for (int32_t b = threadIdx.x; b < B; b += kThreads) {
    w.blk_off[(size_t)blockIdx.x * B + b] = h[b];
    if (h[b]) atomicAdd(&w.bucket_count[b], h[b]);
  }
}

// after k_eg_scan: each block's first slot in every bucket (one block per bucket, an exclusive
// scan over the G per-block counts; G <= kMaxScatterBlocks = 4 * kThreads)
__global__ __launch_bounds__(kThreads) void k_eg_block_offsets(EnvGradWs w, uint32_t G) {
  __shared__ uint32_t wsum[kThreads / 64];
  const int32_t b = blockIdx.x;
  const uint32_t per = (G + kThreads - 1) / kThreads;
  const uint32_t g0 = min(G, threadIdx.x * per), g1 = min(G, g0 + per);
  uint32_t v[kMaxScatterBlocks / kThreads];
  uint32_t sum = 0;
#pragma unroll
  for (uint32_t k = 0; k < kMaxScatterBlocks / kThreads; ++k) {
    v[k] = g0 + k < g1 ? w.blk_off[(size_t)(g0 + k) * w.n_buckets + b] : 0u;
    sum += v[k];
  }
  uint32_t x = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if ((int)__lane_id() >= o) x += y;
  }
  if (__lane_id() == 63) wsum[threadIdx.x >> 6] = x;
  __syncthreads();
  uint32_t acc = w.bucket_off[b] + x - sum;
  for (uint32_t q = 0; q < (threadIdx.x >> 6); ++q) acc += wsum[q];
#pragma unroll
  for (uint32_t k = 0; k < kMaxScatterBlocks / kThreads; ++k) {
    if (g0 + k < g1) w.blk_off[(size_t)(g0 + k) * w.n_buckets + b] = acc;
    acc += v[k];
  }
}

__device__ __forceinline__ uint32_t n_chunks(uint32_t count) {
  return (uint32_t)((count + kReduceChunk - 1) / kReduceChunk);
}

// exclusive scans of the bucket sizes and of their reduction chunks (one block)
__global__ __launch_bounds__(kThreads) void k_eg_scan(EnvGradWs w) {
  __shared__ uint32_t part[kThreads], partc[kThreads];
  const int32_t B = w.n_buckets;
  const int32_t per = (B + kThreads - 1) / kThreads;
  const int32_t b0 = threadIdx.x * per, b1 = min(B, b0 + per);
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
    acc += w.bucket_count[b];
    accc += n_chunks(w.bucket_count[b]);
  }
}

// each block reserves its share of every bucket with one atomic, then places its records
__global__ __launch_bounds__(kThreads) void k_eg_scatter(EnvGradWs w) {
  __shared__ uint32_t h[kMaxLdsBuckets];
  for (int32_t b = threadIdx.x; b < w.n_buckets; b += kThreads) h[b] = 0u;
  __syncthreads();
  const uint32_t n = n_records(w);
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const uint32_t t = w.rec[i].texel;
    if (valid(w, t)) atomicAdd(&h[t >> kBucketShift], 1u);
  }
  __syncthreads();
  for (int32_t b = threadIdx.x; b < w.n_buckets; b += kThreads)
    if (h[b]) h[b] = atomicAdd(&w.bucket_cur[b], h[b]);
  __syncthreads();
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const EnvRec r = w.rec[i];
    if (!valid(w, r.texel)) continue;
    const uint32_t slot = atomicAdd(&h[r.texel >> kBucketShift], 1u);
    w.sorted[slot] = r;
  }
}

constexpr int kTileRecs = 2048;                      // records per tile of the tiled scatter
constexpr int kTilePer = kTileRecs / kThreads;       // records per thread and tile
static_assert(kMaxScatterBlocks % kThreads == 0, "block-offset scan: whole per-thread groups");

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if ((int)__lane_id() >= o) x += y;
  }
  return x;
}

// Tiled scatter (n_buckets <= kTileMaxBuckets): each block owns the contiguous range of the
// records that k_eg_hist_blocks counted for it, starts from the first slots k_eg_block_offsets
// gave it in every bucket, and walks its range in tiles of kTileRecs records: a counting sort of the tile by bucket in LDS, and the sorted tile
// written out run by run behind the block's per-bucket cursors. A bucket's runs of consecutive
// tiles are adjacent in memory, so the lines they share are completed microseconds apart and
// merge in L2 instead of being written back part-filled; the stores of a run are coalesced.
__global__ __launch_bounds__(kThreads) void k_eg_scatter_tiled(EnvGradWs w) {
  __shared__ uint32_t cur[kTileMaxBuckets], cnt[kTileMaxBuckets], off[kTileMaxBuckets];
  __shared__ uint4 lrec[kTileRecs];  // records as raw 16-byte words (texel first)
  __shared__ uint32_t wsum[kThreads / 64];
  const int32_t B = w.n_buckets;
  uint32_t r0, r1;
  block_range(n_records(w), blockIdx.x, gridDim.x, &r0, &r1);
  for (int32_t b = threadIdx.x; b < B; b += kThreads) cur[b] = w.blk_off[(size_t)blockIdx.x * B + b];
  const int32_t per = (B + kThreads - 1) / kThreads;  // buckets per thread in the tile scan
  const int32_t b0 = min(B, (int32_t)threadIdx.x * per), b1 = min(B, b0 + per);
  for (uint32_t t0 = r0; t0 < r1; t0 += kTileRecs) {
    for (int32_t b = threadIdx.x; b < B; b += kThreads) cnt[b] = 0u;
    __syncthreads();
    uint4 r[kTilePer];
    int32_t bk[kTilePer];
    uint32_t rank[kTilePer];
#pragma unroll
    for (int k = 0; k < kTilePer; ++k) {
      const uint32_t i = t0 + (uint32_t)(k * kThreads) + threadIdx.x;
      r[k] = i < r1 ? reinterpret_cast<const uint4*>(w.rec)[i] : make_uint4(kNoTexel, 0u, 0u, 0u);
      const bool ok = valid(w, r[k].x);
      bk[k] = ok ? (int32_t)(r[k].x >> kBucketShift) : -1;
      rank[k] = ok ? atomicAdd(&cnt[bk[k]], 1u) : 0u;
    }
    __syncthreads();
    // exclusive scan of the tile's bucket counts
    uint32_t sum = 0;
    for (int32_t b = b0; b < b1; ++b) sum += cnt[b];
    const uint32_t incl = wave_incl_scan(sum);
    if (__lane_id() == 63) wsum[threadIdx.x >> 6] = incl;
    __syncthreads();
    uint32_t excl = incl - sum;
    for (uint32_t q = 0; q < (threadIdx.x >> 6); ++q) excl += wsum[q];
    for (int32_t b = b0; b < b1; ++b) {
      off[b] = excl;
      excl += cnt[b];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTilePer; ++k)
      if (bk[k] >= 0) lrec[off[bk[k]] + rank[k]] = r[k];
    __syncthreads();
    const uint32_t total = off[B - 1] + cnt[B - 1];
    for (uint32_t i = threadIdx.x; i < total; i += kThreads) {
      const uint4 q = lrec[i];
      const uint32_t b = q.x >> kBucketShift;
      reinterpret_cast<uint4*>(w.sorted)[cur[b] + (i - off[b])] = q;
    }
    __syncthreads();
    for (int32_t b = threadIdx.x; b < B; b += kThreads) cur[b] += cnt[b];
    __syncthreads();
  }
}

// one block per chunk of a bucket's records: FP64 sums in LDS, then denv += sums (a plain
// read-modify-write when the chunk is the bucket's only one, else FP64 atomics). Blocks past the
// last chunk exit at once (the grid is sized for the largest possible chunk count).
__global__ __launch_bounds__(kThreads) void k_eg_reduce(EnvGradWs w, int64_t n_texels, double* __restrict__ denv) {
  __shared__ double acc[3 * kBucketTexels];
  const uint32_t c = blockIdx.x;
  const int32_t B = w.n_buckets;
  if (c >= w.chunk_off[B]) return;
  // the bucket of chunk c: last b with chunk_off[b] <= c
  int32_t lo = 0, hi = B - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (w.chunk_off[mid] <= c)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int32_t b = lo;
  const bool alone = w.chunk_off[b + 1] - w.chunk_off[b] == 1u;
  const uint32_t r0 = w.bucket_off[b] + (uint32_t)((int64_t)(c - w.chunk_off[b]) * kReduceChunk);
  const uint32_t r1 = (uint32_t)min((int64_t)w.bucket_off[b + 1], (int64_t)r0 + kReduceChunk);
  for (int32_t k = threadIdx.x; k < 3 * kBucketTexels; k += kThreads) acc[k] = 0.0;
  __syncthreads();
  uint32_t i = r0 + threadIdx.x;
  for (; i + (kLoads - 1) * kThreads < r1; i += kLoads * kThreads) {
    EnvRec r[kLoads];
#pragma unroll
    for (int k = 0; k < kLoads; ++k) r[k] = w.sorted[i + k * kThreads];
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
      const uint32_t t = r[k].texel & (kBucketTexels - 1);
      atomicAdd(&acc[3 * t], (double)r[k].w[0]);
      atomicAdd(&acc[3 * t + 1], (double)r[k].w[1]);
      atomicAdd(&acc[3 * t + 2], (double)r[k].w[2]);
    }
  }
  for (; i < r1; i += kThreads) {
    const EnvRec r = w.sorted[i];
    const uint32_t t = r.texel & (kBucketTexels - 1);
    atomicAdd(&acc[3 * t], (double)r.w[0]);
    atomicAdd(&acc[3 * t + 1], (double)r.w[1]);
    atomicAdd(&acc[3 * t + 2], (double)r.w[2]);
  }
  __syncthreads();
  const int64_t base = (int64_t)b * kBucketTexels;
  for (int32_t k = threadIdx.x; k < 3 * kBucketTexels; k += kThreads) {
    const int64_t t = base + k / 3;
    if (t >= n_texels || acc[k] == 0.0) continue;
    if (alone)
      denv[3 * base + k] += acc[k];
    else
      unsafeAtomicAdd(denv + 3 * base + k, acc[k]);
  }
}

}  // namespace

hipError_t launch_env_grad_clear(const EnvGradWs& w, hipStream_t s) {
  const int32_t n = w.n_buckets + 1;
  {
    EXM_TIMED("env_grad_clear", s);
    k_eg_clear<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(w.counter, w.bucket_count, w.n_buckets);
  }
  return hipGetLastError();
}

hipError_t launch_env_grad_reduce(const EnvGradWs& w, int32_t He, int32_t We, double* denv, hipStream_t s) {
  if (w.n_buckets > kMaxLdsBuckets) return hipErrorInvalidValue;  // the ABI bounds He * We
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(kSortBlocks, (w.cap + kThreads - 1) / kThreads));
  const bool tiled = w.n_buckets <= kTileMaxBuckets;
  unsigned tg = 1;  // tiled path: one contiguous range per resident scatter block
  if (tiled) {
    int dev = 0, cus = 256, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipGetLastError();
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return hipGetLastError();
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_eg_scatter_tiled, kThreads, 0) !=
            hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    tg = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>(std::min<int64_t>((int64_t)cus * per_cu, kMaxScatterBlocks),
                             (w.cap + kTileRecs - 1) / kTileRecs));
  }
  {
    EXM_TIMED("env_grad_hist", s);
    if (tiled)
      k_eg_hist_blocks<<<tg, kThreads, 0, s>>>(w);
    else
      k_eg_hist<<<grid, kThreads, 0, s>>>(w);
  }
  {
    EXM_TIMED("env_grad_scan", s);
    k_eg_scan<<<1, kThreads, 0, s>>>(w);
    if (tiled) k_eg_block_offsets<<<(unsigned)w.n_buckets, kThreads, 0, s>>>(w, tg);
  }
  {
    EXM_TIMED("env_grad_scatter", s);
    if (tiled)
      k_eg_scatter_tiled<<<tg, kThreads, 0, s>>>(w);
    else
      k_eg_scatter<<<grid, kThreads, 0, s>>>(w);
  }
  {
    EXM_TIMED("env_grad_reduce", s);
    const int64_t max_chunks = (w.cap + kReduceChunk - 1) / kReduceChunk + w.n_buckets;
    k_eg_reduce<<<(unsigned)max_chunks, kThreads, 0, s>>>(w, (int64_t)He * We, denv);
  }
  return hipGetLastError();
}

}  // namespace exm
