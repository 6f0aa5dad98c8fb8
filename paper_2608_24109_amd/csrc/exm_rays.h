// Ray batches between the kernels that generate rays, the persistent traversal kernel and the
// kernels that consume the results, plus the workspace layouts of the passes that use them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "exm_device.h"

namespace exm {

// 16-byte ray record: direction and the index of its origin record. The rays that leave one
// point (a pixel's shadow or secondary rays, a secondary point's light samples) share that record:
// the point and the triangle it lies on, which they skip.
struct alignas(16) RayRec {
  float d[3];
  uint32_t org;
};
static_assert(sizeof(RayRec) == 16, "ray layout");
struct alignas(16) RayOrg {
  float o[3];
  int32_t skip;
};
static_assert(sizeof(RayOrg) == 16, "origin layout");

// The wavefront records (rays, contributions) are written once and read once by a later kernel,
// after far more data than the caches hold has passed: nontemporal stores keep them from displacing
// the sampling tables and the BVH that the kernels reuse.
__device__ __forceinline__ void store_ray(RayRec* rays, int64_t slot, const float d[3], uint32_t org) {
  typedef float f4v __attribute__((ext_vector_type(4)));
  const f4v v = {d[0], d[1], d[2], __uint_as_float(org)};
  __builtin_nontemporal_store(v, reinterpret_cast<f4v*>(rays) + slot);
}
__device__ __forceinline__ void store_contrib(float* contrib, int64_t slot, float r, float g, float b) {
  __builtin_nontemporal_store(r, contrib + 3 * slot);
  __builtin_nontemporal_store(g, contrib + 3 * slot + 1);
  __builtin_nontemporal_store(b, contrib + 3 * slot + 2);
}

// Region r holds count[r] rays at slots [r * region_stride, r * region_stride + count[r]); a hit
// counts at t >= tmin (for batches over several assets, the tmin of the region's asset).
struct RayBatch {
  const RayRec* rays;
  const RayOrg* orgs;
  const uint32_t* count;
  int32_t n_regions;
  int64_t region_stride;
  float tmin;
  uint32_t* region_counter;  // workspace word, reset by the launcher
};

// A persistent traversal wave refills once fewer than kRayRefill lanes still traverse, and a
// round's node phase hands over to its leaf phase once fewer than `gate` lanes lack a postponed
// leaf: kTravLeafGateWide for batches whose regions hold at least kWideRegion ray slots (N_d >= 32
// direct samples per pixel), kTravLeafGate otherwise. Swept with the wave-wide any-hit leaf phase
// (gate 2-32 x refill 24-48): at N_d 64 gate 16 (any-hit traversal of the displaced sphere 23.8 ->
// 22.0 ms against the per-lane leaf loop at refill 32 and gate 8, tori 23.2 -> 22.9 ms), at N_d 8
// gate 8 (a 1600^2 relight 1.73 -> 1.68 ms; gate 16 took 1.86 ms).
constexpr int32_t kRayRefill = 24;
constexpr int32_t kTravLeafGate = 8;
constexpr int32_t kTravLeafGateWide = 16;
constexpr int64_t kWideRegion = 2048;
// The BVHs of a launch whose rays come from several assets (a batch of requests): region r's rays
// belong to asset f, region_start[f] <= r < region_start[f + 1].
struct BvhTable {
  BvhView b[kMaxFrames];
  float tmin[kMaxFrames];
  int32_t region_start[kMaxFrames + 1];
  int32_t n;
};

// any-hit: out[slot] = 1 if something is hit at t >= tmin (the skipped triangle excepted)
hipError_t launch_trace_any(const exm_bvh* bvh, const RayBatch& rb, uint8_t* out, unsigned long long* counters,
                            hipStream_t s);
// any-hit over the regions of a batch, each region traversing its own asset's BVH
hipError_t launch_trace_any_batch(const BvhTable& t, const RayBatch& rb, uint8_t* out, unsigned long long* counters,
                                  hipStream_t s);
// closest hit: out[slot] = {id (-1 miss), t, b1, b2}
hipError_t launch_trace_closest(const exm_bvh* bvh, const RayBatch& rb, HitRec* out, unsigned long long* counters,
                                hipStream_t s);

// ---- workspace carving ----
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Direct pass over a chunk of P pixels (P a multiple of 64; one region per 64 pixels, N_d slots
// per pixel): counter, per-region counts, per-pixel sample masks, rays, the covered pixels' origin
// records (region * 64 + the pixel's rank among the region's covered pixels), contributions, hits.
struct DirectWs {
  uint32_t* counter;
  uint32_t* count;
  uint64_t* mask;
  RayRec* rays;
  RayOrg* orgs;
  float* contrib;
  uint8_t* hit;
};

inline size_t direct_ws_bytes(int64_t P, int32_t N_d) {
  const int64_t slots = P * (int64_t)(N_d > 0 ? N_d : 1);
  return 256 + align256((size_t)(P / 64) * 4) + align256((size_t)P * 8) + align256((size_t)slots * 16) +
         align256((size_t)P * 16) + align256((size_t)slots * 12) + align256((size_t)slots);
}

inline DirectWs direct_ws(void* ws, int64_t P, int32_t N_d) {
  const int64_t slots = P * (int64_t)(N_d > 0 ? N_d : 1);
  char* q = static_cast<char*>(ws);
  DirectWs w;
  w.counter = reinterpret_cast<uint32_t*>(q);
  q += 256;
  w.count = reinterpret_cast<uint32_t*>(q);
  q += align256((size_t)(P / 64) * 4);
  w.mask = reinterpret_cast<uint64_t*>(q);
  q += align256((size_t)P * 8);
  w.rays = reinterpret_cast<RayRec*>(q);
  q += align256((size_t)slots * 16);
  w.orgs = reinterpret_cast<RayOrg*>(q);
  q += align256((size_t)P * 16);
  w.contrib = reinterpret_cast<float*>(q);
  q += align256((size_t)slots * 12);
  w.hit = reinterpret_cast<uint8_t*>(q);
  return w;
}

// largest chunk (multiple of 64 pixels, at most max_px) that fits ws_bytes; 0 if none
inline int64_t direct_chunk(size_t ws_bytes, int32_t N_d, int64_t max_px) {
  int64_t lo = 0, hi = (max_px + 63) / 64;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (direct_ws_bytes(mid * 64, N_d) <= ws_bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo * 64;
}

// Indirect pass over a chunk of P pixels (P a multiple of 64): secondary rays (N_b per pixel)
// with their closest hits and the covered pixels' origin records (as in the direct pass), then the
// light samples of valid hits (N_b * N_s per pixel) with their shadow rays, the origin records of the
// valid hits (at the secondary ray's slot), contributions and hits, and for each (pixel, light
// sample) the slot of its shadow ray in its region (sh_slot[pixel * N_b * N_s + j * N_s + s], set
// where sh_mask has the bit).
struct IndirectWs {
  uint32_t* counter;
  uint32_t* sec_count;
  RayRec* sec_rays;
  RayOrg* sec_orgs;
  HitRec* sec_hits;
  uint32_t* sh_count;
  uint64_t* sh_mask;
  RayRec* sh_rays;
  RayOrg* sh_orgs;
  float* sh_contrib;
  uint8_t* sh_hit;
  uint32_t* sh_slot;
};

inline size_t indirect_ws_bytes(int64_t P, int32_t N_b, int32_t N_s) {
  const int64_t s1 = P * (int64_t)(N_b > 0 ? N_b : 1), s2 = s1 * (N_s > 0 ? N_s : 1);
  return 256 + 2 * align256((size_t)(P / 64) * 4) + align256((size_t)s1 * 16) + align256((size_t)P * 16) +
         align256((size_t)s1 * 16) + align256((size_t)P * 8) + align256((size_t)s2 * 16) + align256((size_t)s1 * 16) +
         align256((size_t)s2 * 12) + align256((size_t)s2) + align256((size_t)s2 * 4);
}

inline IndirectWs indirect_ws(void* ws, int64_t P, int32_t N_b, int32_t N_s) {
  const int64_t s1 = P * (int64_t)(N_b > 0 ? N_b : 1), s2 = s1 * (N_s > 0 ? N_s : 1);
  char* q = static_cast<char*>(ws);
  IndirectWs w;
  w.counter = reinterpret_cast<uint32_t*>(q);
  q += 256;
  w.sec_count = reinterpret_cast<uint32_t*>(q);
  q += align256((size_t)(P / 64) * 4);
  w.sh_count = reinterpret_cast<uint32_t*>(q);
  q += align256((size_t)(P / 64) * 4);
  w.sec_rays = reinterpret_cast<RayRec*>(q);
  q += align256((size_t)s1 * 16);
  w.sec_orgs = reinterpret_cast<RayOrg*>(q);
  q += align256((size_t)P * 16);
  w.sec_hits = reinterpret_cast<HitRec*>(q);
  q += align256((size_t)s1 * 16);
  w.sh_mask = reinterpret_cast<uint64_t*>(q);
  q += align256((size_t)P * 8);
  w.sh_rays = reinterpret_cast<RayRec*>(q);
  q += align256((size_t)s2 * 16);
  w.sh_orgs = reinterpret_cast<RayOrg*>(q);
  q += align256((size_t)s1 * 16);
  w.sh_contrib = reinterpret_cast<float*>(q);
  q += align256((size_t)s2 * 12);
  w.sh_hit = reinterpret_cast<uint8_t*>(q);
  q += align256((size_t)s2);
  w.sh_slot = reinterpret_cast<uint32_t*>(q);
  return w;
}

inline int64_t indirect_chunk(size_t ws_bytes, int32_t N_b, int32_t N_s, int64_t max_px) {
  // a chunk's origin records (one per secondary ray slot) are indexed by 32-bit fields of the rays
  max_px = std::min<int64_t>(max_px, (((int64_t)1 << 31) - 64) / (N_b > 0 ? N_b : 1));
  int64_t lo = 0, hi = (max_px + 63) / 64;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (indirect_ws_bytes(mid * 64, N_b, N_s) <= ws_bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo * 64;
}

}  // namespace exm
