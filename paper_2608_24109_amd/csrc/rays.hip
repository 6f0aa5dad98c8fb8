// Batched ray queries on the BVH: any-hit (visibility) and closest-hit (secondary rays).
//
// Rays arrive in regions: region r holds count[r] rays at slots [r * region_stride, ...). The
// kernel is persistent: a wave claims a whole region with one atomic, then its lanes take the
// region's rays one at a time as they finish (wave-local bookkeeping through ballots, no
// atomics), so a wave is held neither by its longest ray nor by idle lanes. Traversal yields
// back to refilling when fewer than `refill` lanes are still traversing (24), and a round's node
// phase hands over to its leaf phase once fewer than `leaf_gate` lanes lack a postponed leaf (8,
// or 16 for regions of many rays: waiting for every lane, as in the plain while-while loop, left
// most lanes idle). Any-hit
// queries test their leaves across the whole wave (every lane of the wave runs every round, with
// or without a ray, so that the leaf phase's cross-lane reads see all lanes). Each lane keeps only
// a ray and its traversal state, so the kernel stays small and many waves are resident to hide
// the latency of node fetches.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "exm_device.h"
#include "exm_rays.h"

namespace exm {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  const uint32_t lane = __lane_id();
  return (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
}

// BATCH: the regions come from several assets; a wave looks up the BVH of each region it claims
// and every lane keeps the BVH of its own ray (lanes of one wave may hold rays of two regions).
// Six waves per SIMD (the LDS stack allows six blocks per CU): held to 80 VGPRs, with a few
// spilled bytes, the traversal ran faster than at five waves with 88-100 VGPRs (tori any-hit
// 19.0 against 18.0 ms).
template <bool ANY, bool COUNT, bool BATCH>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(6, 6))) void k_trace(BvhView B0, BvhTable bt, RayBatch rb, int32_t refill,
                                                    int32_t leaf_gate, HitRec* __restrict__ out_hit,
                                                    uint8_t* __restrict__ out_any,
                                                    unsigned long long* __restrict__ counters) {
  __shared__ int32_t stack_mem[kStackLds * kThreads];
  int32_t ovf[kStackOvf];  // private: only stacks deeper than kStackLds reach it
  const LaneStack stack{stack_mem + threadIdx.x, (private_i32*)ovf, kThreads};
  BvhView B = B0;        // the BVH of the lane's ray
  BvhView B_region = B0;  // the BVH of the region being handed out (wave-uniform)
  float tmin_region = rb.tmin;
  // wave-uniform region cursor
  int32_t region = -1;
  uint32_t next = 0, count = 0;
  int64_t base = 0;
  bool exhausted = false;
  // lane state
  bool have_ray = false;
  int64_t slot = 0;
  Ray ray;  // set below, before the first round
  float tmin = 0.0f;
  int32_t skip = -1;
  TravState ts;
  ts.ref = ts.leaf = kEmptyRef;  // no query: every lane joins the wave's leaf phases anyway
  ts.sp = 0;
  ts.rounds = 0;
  HitRec h;
  h.id = -1;
  h.t = __builtin_huge_valf();
  h.b1 = h.b2 = 0.0f;
  ray = make_ray(mk(0.f, 0.f, 0.f), mk(0.f, 0.f, 1.f));
  TraceCount tc;
  uint32_t n_rays = 0;

  while (true) {
    uint64_t need = __ballot(!have_ray);
    while (need != 0ull && !exhausted) {
      if (next >= count) {
        int32_t r = 0;
        if (__lane_id() == 0) r = (int32_t)atomicAdd(rb.region_counter, 1u);
        region = __shfl(r, 0, 64);
        if (region >= rb.n_regions) {
          exhausted = true;
          break;
        }
        count = rb.count[region];
        next = 0;
        if (BATCH) {
          int32_t f = 0;
          while (f + 1 < bt.n && region >= bt.region_start[f + 1]) ++f;
          B_region = bt.b[f];
          tmin_region = bt.tmin[f];
        }
        base = (int64_t)region * rb.region_stride;
        continue;
      }
      const uint32_t avail = count - next;
      const uint32_t rank = lanes_below(need);
      if (!have_ray && rank < avail) {
        slot = base + next + rank;
        if (BATCH) B = B_region;
        const RayRec R = rb.rays[slot];
        const RayOrg O = rb.orgs[R.org];
        ray = make_ray(mk(O.o[0], O.o[1], O.o[2]), mk(R.d[0], R.d[1], R.d[2]));
        tmin = BATCH ? tmin_region : rb.tmin;
        skip = O.skip;
        trav_begin(B, ts, h, stack);
        have_ray = true;
        if (COUNT) ++n_rays;
      }
      next += min(avail, (uint32_t)__popcll(need));
      need = __ballot(!have_ray);
    }
    if (__ballot(have_ray) == 0ull) break;
    while (true) {  // every lane of the wave calls trav_round (the any-hit leaf phase spans the wave)
      const bool fin = trav_round<ANY, COUNT, BATCH>(B, ray, tmin, skip, stack, ts, h, &tc, leaf_gate);
      if (have_ray && fin) {
        if (ANY)
          out_any[slot] = h.id >= 0 ? 1 : 0;
        else
          out_hit[slot] = h;
        have_ray = false;
        ts.ref = ts.leaf = kEmptyRef;
      }
      if (__popcll(__ballot(have_ray)) < refill) break;
    }
  }
  if (COUNT) {
    atomicAdd(counters + 0, (unsigned long long)n_rays);
    atomicAdd(counters + 1, (unsigned long long)tc.nodes);
    atomicAdd(counters + 2, (unsigned long long)tc.tris);
  }
}

__global__ void k_reset_counter(uint32_t* c) { *c = 0u; }

template <bool ANY, bool COUNT, bool BATCH>
hipError_t launch_impl(const BvhView& B0, const BvhTable& bt, const RayBatch& rb, HitRec* out_hit, uint8_t* out_any,
                       unsigned long long* counters, hipStream_t s) {
  if (rb.n_regions <= 0) return hipSuccess;
  int dev = 0, cus = 256, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipGetLastError();
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return hipGetLastError();
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_trace<ANY, COUNT, BATCH>, kThreads, 0) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int64_t waves_needed = rb.n_regions;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((waves_needed + 3) / 4, (int64_t)cus * per_cu));
  k_reset_counter<<<1, 1, 0, s>>>(rb.region_counter);
  {
    EXM_TIMED(ANY ? "trace_any" : "trace_closest", s);
    const int32_t gate = rb.region_stride >= kWideRegion ? kTravLeafGateWide : kTravLeafGate;
    k_trace<ANY, COUNT, BATCH><<<(unsigned)blocks, kThreads, 0, s>>>(B0, bt, rb, kRayRefill, gate, out_hit, out_any,
                                                                      counters);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_trace_any(const exm_bvh* bvh, const RayBatch& rb, uint8_t* out, unsigned long long* counters,
                            hipStream_t s) {
  const BvhView B{bvh->nodes, bvh->tris};
  const BvhTable none{};
  return counters ? launch_impl<true, true, false>(B, none, rb, nullptr, out, counters, s)
                  : launch_impl<true, false, false>(B, none, rb, nullptr, out, nullptr, s);
}

hipError_t launch_trace_any_batch(const BvhTable& t, const RayBatch& rb, uint8_t* out, unsigned long long* counters,
                                  hipStream_t s) {
  return counters ? launch_impl<true, true, true>(t.b[0], t, rb, nullptr, out, counters, s)
                  : launch_impl<true, false, true>(t.b[0], t, rb, nullptr, out, nullptr, s);
}

hipError_t launch_trace_closest(const exm_bvh* bvh, const RayBatch& rb, HitRec* out, unsigned long long* counters,
                                hipStream_t s) {
  const BvhView B{bvh->nodes, bvh->tris};
  const BvhTable none{};
  return counters ? launch_impl<false, true, false>(B, none, rb, out, nullptr, counters, s)
                  : launch_impl<false, false, false>(B, none, rb, out, nullptr, nullptr, s);
}

}  // namespace exm
