// Material-map gradient by a tiled reduction instead of per-tap atomics.
//
// The map adjoint of a pixel is eight channel gradients spread over the four bilinear taps of its
// texture position. An adjoint kernel appends one 64-byte record per pixel (the first tap, the
// step to the second column and row of taps, the four weights, the eight gradients; one atomic
// per wave reserves the wave's range). Taps that fall outside the tile of kTexTileW x kTexTileH
// texels holding the first tap (the second column or row of taps crossing the tile's last column
// or row: about one pixel in twenty) are added to dtex by the adjoint kernel itself, with atomics.
// A counting sort groups the records by the tile of their first tap. One block per tile takes the
// tile's records kTexChunk at a time: it stages them in LDS, lists for every texel of the tile
// the (record, tap) pairs that reach it (a counting sort of the taps by texel with integer LDS
// atomics), and lets the thread that owns the texel add w_k * g_c over its list to sums it keeps
// in registers. The block ends with one plain read-modify-write of the tile in dtex: no other
// block writes those texels, and the adjoint's atomics have completed before the reduction
// starts. The per-texel sums equal those of the per-tap atomics up to the order of FP32 additions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdlib>

#include "env_grad.h"

namespace exm {

constexpr int32_t kTexTileW = 64;               // texels per tile along a row
constexpr int32_t kTexTileH = 32;               // rows per tile
constexpr int32_t kTexMaxBuckets = 16384;       // tiles of the largest map this path handles
constexpr int64_t kTexChunk = 1024;             // records staged at a time by a tile's block
constexpr uint32_t kTexStepBit = 0x80000000u;   // in col / row: the second tap is one further

struct alignas(16) TexRec {
  uint32_t col;  // column of the first tap | kTexStepBit if taps two and four are one column on
  uint32_t row;  // row of the first tap | kTexStepBit if taps three and four are one row down
  float w[4];    // bilinear weights of the four taps
  float g[8];    // map adjoint of the eight channels
  uint32_t pad[2];
};
static_assert(sizeof(TexRec) == 64, "record layout");

struct TexGradWs {
  uint32_t* counter;       // records appended
  uint32_t* bucket_count;  // [kTexMaxBuckets + 1]
  uint32_t* bucket_off;    // [kTexMaxBuckets + 1]
  uint32_t* bucket_cur;    // [kTexMaxBuckets + 1]
  TexRec* rec;             // [cap] as appended
  TexRec* sorted;          // [cap] grouped by bucket
  int64_t cap;
  int32_t Ht, Wt, nbx, n_buckets;
};

inline int32_t tex_grad_buckets(int32_t Ht, int32_t Wt) {
  const int64_t nbx = ((int64_t)Wt + kTexTileW - 1) / kTexTileW, nby = ((int64_t)Ht + kTexTileH - 1) / kTexTileH;
  return (int32_t)std::min<int64_t>(nbx * nby, (int64_t)kTexMaxBuckets + 1);
}

// whether the tiled reduction handles a map of this size (else the adjoints scatter with atomics)
inline bool tex_grad_tiled(int32_t Ht, int32_t Wt) {
  return Ht > 0 && Wt > 0 && tex_grad_buckets(Ht, Wt) <= kTexMaxBuckets;
}


inline size_t tg_align256(size_t x) { return (x + 255) & ~(size_t)255; }

// bytes for cap records (independent of the map size: the tables are sized for kTexMaxBuckets)
inline size_t tex_grad_ws_bytes(int64_t cap) {
  return 256 + 3 * tg_align256(((size_t)kTexMaxBuckets + 1) * 4) + 2 * tg_align256((size_t)cap * sizeof(TexRec));
}

inline TexGradWs tex_grad_ws(void* ws, int64_t cap, int32_t Ht, int32_t Wt) {
  char* q = static_cast<char*>(ws);
  TexGradWs w;
  w.counter = reinterpret_cast<uint32_t*>(q);
  q += 256;
  const size_t tb = tg_align256(((size_t)kTexMaxBuckets + 1) * 4);
  w.bucket_count = reinterpret_cast<uint32_t*>(q);
  q += tb;
  w.bucket_off = reinterpret_cast<uint32_t*>(q);
  q += tb;
  w.bucket_cur = reinterpret_cast<uint32_t*>(q);
  q += tb;
  w.rec = reinterpret_cast<TexRec*>(q);
  q += tg_align256((size_t)cap * sizeof(TexRec));
  w.sorted = reinterpret_cast<TexRec*>(q);
  w.cap = cap;
  w.Ht = Ht;
  w.Wt = Wt;
  w.nbx = (int32_t)(((int64_t)Wt + kTexTileW - 1) / kTexTileW);
  w.n_buckets = tex_grad_buckets(Ht, Wt);
  return w;
}

// Reserves one record slot for each lane with `want`; one atomic per wave. Every lane of the wave
// must call it (no lane may have exited).
__device__ __forceinline__ uint32_t tex_grad_reserve(uint32_t* counter, bool want) {
  const uint64_t m = __ballot(want);
  const uint32_t total = (uint32_t)__popcll(m);
  uint32_t base = 0;
  if (__lane_id() == 0 && total != 0u) base = atomicAdd(counter, total);
  base = __shfl(base, 0, 64);
  return base + (uint32_t)__popcll(m & ((1ull << __lane_id()) - 1ull));
}

// Reserves n consecutive record slots for each lane (n may differ between lanes); one atomic per
// wave. Every lane of the wave must call it.
__device__ __forceinline__ uint32_t tex_grad_reserve_n(uint32_t* counter, uint32_t n) {
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

// A reserved record left unused: its first tap lies outside every map, so the sort drops it.
__device__ __forceinline__ void tex_grad_skip(const TexGradWs& w, uint32_t slot) {
  if ((int64_t)slot < w.cap)
    *reinterpret_cast<uint2*>(w.rec + slot) = make_uint2(~kTexStepBit, ~kTexStepBit);
}

// Whether tap k (laid out as by bilinear_taps: tap 1 = tap 0 plus the column step dx, tap 2 = tap
// 0 plus the row step dy, tap 3 = both) lies in the tile of tap 0 at (col, row).
__host__ __device__ __forceinline__ bool tex_tap_in_tile(int k, uint32_t col, uint32_t row, bool dx, bool dy) {
  const bool out_x = (k & 1) && dx && (col % kTexTileW) == (uint32_t)(kTexTileW - 1);
  const bool out_y = (k & 2) && dy && (row % kTexTileH) == (uint32_t)(kTexTileH - 1);
  return !(out_x || out_y);
}

// The record of one pixel's map adjoint; the taps outside the first tap's tile go to dtex at once.
__device__ __forceinline__ void tex_grad_put(const TexGradWs& w, uint32_t slot, const int32_t tap[4],
                                             const float wt[4], const float g8[8], float* __restrict__ dtex) {
  if ((int64_t)slot >= w.cap) return;
  const uint32_t col = (uint32_t)(tap[0] % w.Wt), row = (uint32_t)(tap[0] / w.Wt);
  const bool dx = tap[1] != tap[0], dy = tap[2] != tap[0];
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    if (wt[k] == 0.0f || tex_tap_in_tile(k, col, row, dx, dy)) continue;
    float* dst = dtex + (int64_t)tap[k] * 8;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (g8[c] != 0.0f) unsafeAtomicAdd(dst + c, wt[k] * g8[c]);
  }
  uint4* d = reinterpret_cast<uint4*>(w.rec + slot);
  d[0] = make_uint4(col | (dx ? kTexStepBit : 0u), row | (dy ? kTexStepBit : 0u),
                    __float_as_uint(wt[0]), __float_as_uint(wt[1]));
  d[1] = make_uint4(__float_as_uint(wt[2]), __float_as_uint(wt[3]), __float_as_uint(g8[0]), __float_as_uint(g8[1]));
  d[2] = make_uint4(__float_as_uint(g8[2]), __float_as_uint(g8[3]), __float_as_uint(g8[4]), __float_as_uint(g8[5]));
  d[3] = make_uint4(__float_as_uint(g8[6]), __float_as_uint(g8[7]), 0u, 0u);
}

// Largest pixel chunk (multiple of 64, at most max_px) of an adjoint whose env-gradient records
// (env_per_px per pixel) and map-gradient records (tex_per_px per pixel) fit in ws_bytes; the env
// part comes first in the workspace.
inline int64_t adjoint_chunk(size_t ws_bytes, int64_t env_per_px, int64_t tex_per_px, int32_t He, int32_t We,
                             int64_t max_px) {
  int64_t lo = 0, hi = (max_px + 63) / 64;
  const int64_t per = std::max<int64_t>(std::max<int64_t>(env_per_px, tex_per_px), 1);
  hi = std::min<int64_t>(hi, ((int64_t)1 << 31) / (64 * per));
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (env_grad_ws_bytes(mid * 64 * env_per_px, He, We) + tex_grad_ws_bytes(mid * 64 * tex_per_px) <= ws_bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo * 64;
}

// zero the counters (a fill kernel, so that the sequence stays capturable)
hipError_t launch_tex_grad_clear(const TexGradWs& w, hipStream_t s);
// dtex += per-texel sums of the appended records
hipError_t launch_tex_grad_reduce(const TexGradWs& w, float* dtex, hipStream_t s);

}  // namespace exm
