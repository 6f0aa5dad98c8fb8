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
  for (uint32_t i = r0 + threadIdx.x; i < r1; i += kThreads) {
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
  {
    EXM_TIMED("env_grad_hist", s);
    k_eg_hist<<<grid, kThreads, 0, s>>>(w);
  }
  {
    EXM_TIMED("env_grad_scan", s);
    k_eg_scan<<<1, kThreads, 0, s>>>(w);
  }
  {
    EXM_TIMED("env_grad_scatter", s);
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
