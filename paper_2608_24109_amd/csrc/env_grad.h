// Environment-map gradient by binned reduction instead of per-sample atomics.
//
// The adjoint of an env sample is three FP32 weights for one texel (dLoss/dE of the sample).
// Adjoint kernels append one 16-byte record per sample into a workspace (one atomic per wave
// reserves the wave's range); then a counting sort groups the records by buckets of
// kBucketTexels texels, and one block per chunk of at most kReduceChunk records of a bucket sums
// them in LDS (FP64) and adds the sums to denv: with plain read-modify-writes when the chunk is
// its bucket's only one (no other block touches those texels), with FP64 atomics otherwise
// (importance sampling puts many records in the buckets of bright texels, which one block per
// bucket would serialise). The sums equal the per-sample atomics' up to the order of FP64
// additions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace exm {

constexpr int32_t kBucketShift = 11;
constexpr int32_t kBucketTexels = 1 << kBucketShift;  // 2048 texels x 3 x 8 B = 48 KB of LDS
constexpr uint32_t kNoTexel = 0xFFFFFFFFu;            // record slot reserved but unused
constexpr int64_t kReduceChunk = 32768;               // records summed by one block
constexpr int32_t kTileMaxBuckets = 1024;             // buckets of the tiled scatter (LDS cursors)
constexpr int32_t kMaxScatterBlocks = 1024;           // blocks of the tiled histogram and scatter

struct alignas(16) EnvRec {
  uint32_t texel;
  float w[3];
};
static_assert(sizeof(EnvRec) == 16, "record layout");

struct EnvGradWs {
  uint32_t* counter;       // records appended
  uint32_t* bucket_count;  // [B]
  uint32_t* bucket_off;    // [B + 1]
  uint32_t* bucket_cur;    // [B]
  uint32_t* chunk_off;     // [B + 1] first reduction chunk of each bucket
  uint32_t* blk_off;       // [kMaxScatterBlocks, B] per-block counts, then first slots (B <= kTileMaxBuckets)
  EnvRec* rec;             // [cap] as appended
  EnvRec* sorted;          // [cap] grouped by bucket
  int64_t cap;
  int32_t n_buckets;
};

inline int32_t env_grad_buckets(int32_t He, int32_t We) {
  return (int32_t)(((int64_t)He * We + kBucketTexels - 1) / kBucketTexels);
}

inline size_t eg_align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline size_t env_grad_blk_bytes(int32_t B) {
  return B <= kTileMaxBuckets ? eg_align256((size_t)kMaxScatterBlocks * (size_t)B * 4) : 0;
}

inline size_t env_grad_ws_bytes(int64_t cap, int32_t He, int32_t We) {
  const int32_t B = env_grad_buckets(He, We);
  return 256 + 4 * eg_align256(((size_t)B + 1) * 4) + env_grad_blk_bytes(B) +
         2 * eg_align256((size_t)cap * sizeof(EnvRec));
}

inline EnvGradWs env_grad_ws(void* ws, int64_t cap, int32_t He, int32_t We) {
  const int32_t B = env_grad_buckets(He, We);
  char* q = static_cast<char*>(ws);
  EnvGradWs w;
  w.counter = reinterpret_cast<uint32_t*>(q);
  q += 256;
  w.bucket_count = reinterpret_cast<uint32_t*>(q);
  q += eg_align256(((size_t)B + 1) * 4);
  w.bucket_off = reinterpret_cast<uint32_t*>(q);
  q += eg_align256(((size_t)B + 1) * 4);
  w.bucket_cur = reinterpret_cast<uint32_t*>(q);
  q += eg_align256(((size_t)B + 1) * 4);
  w.chunk_off = reinterpret_cast<uint32_t*>(q);
  q += eg_align256(((size_t)B + 1) * 4);
  w.blk_off = reinterpret_cast<uint32_t*>(q);
  q += env_grad_blk_bytes(B);
  w.rec = reinterpret_cast<EnvRec*>(q);
  q += eg_align256((size_t)cap * sizeof(EnvRec));
  w.sorted = reinterpret_cast<EnvRec*>(q);
  w.cap = cap;
  w.n_buckets = B;
  return w;
}

// Largest pixel chunk (multiple of 64, at most max_px) whose records (per_px per pixel) fit.
// Record slots are 32-bit: a chunk holds fewer than 2^31 records.
inline int64_t env_grad_chunk(size_t ws_bytes, int64_t per_px, int32_t He, int32_t We, int64_t max_px) {
  int64_t lo = 0, hi = (max_px + 63) / 64;
  if (per_px > 0) hi = std::min<int64_t>(hi, ((int64_t)1 << 31) / (64 * per_px));
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (env_grad_ws_bytes(mid * 64 * per_px, He, We) <= ws_bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo * 64;
}

// Reserves n consecutive record slots for each lane; one atomic per wave. Every lane of the
// wave must call it (no lane may have exited).
__device__ __forceinline__ uint32_t env_grad_reserve(uint32_t* counter, uint32_t n) {
  uint32_t x = n;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if ((int)__lane_id() >= o) x += y;
  }
  const uint32_t total = __shfl(x, 63, 64);
  uint32_t base = 0;
  if (__lane_id() == 63 && total != 0u) base = atomicAdd(counter, total);
  base = __shfl(base, 63, 64);
  return base + x - n;
}

__device__ __forceinline__ void env_grad_put(const EnvGradWs& w, uint32_t slot, uint32_t texel, float a, float b,
                                             float c) {
  if ((int64_t)slot < w.cap) {
    EnvRec r;
    r.texel = texel;
    r.w[0] = a;
    r.w[1] = b;
    r.w[2] = c;
    w.rec[slot] = r;
  }
}

// zero the counters (a fill kernel, so that the sequence stays capturable)
hipError_t launch_env_grad_clear(const EnvGradWs& w, hipStream_t s);
// denv += per-texel sums of the appended records
hipError_t launch_env_grad_reduce(const EnvGradWs& w, int32_t He, int32_t We, double* denv, hipStream_t s);

}  // namespace exm
