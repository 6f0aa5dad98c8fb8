// Direct illumination (Direct Illumination, Eq. 12-17) and its adjoint.
//
// Forward, per covered pixel: attribute query at the visible point (Eq. 10-11), then N_d
// env samples drawn from the importance-sampling tables; a sample with n_s . w > 0 traces an
// any-hit shadow ray and, if unoccluded, adds E f_r (n_s . w) / pdf (Eq. 13-16 for f_r).
// It runs as three kernels per chunk of pixels:
//   gen      one wave per 64 pixels: the attribute query one thread per pixel, then the N_d
//            samples one thread per sample (64 / N_d pixels at a time); each sample with
//            n_s . w > 0 writes its shadow ray and its contribution E f_r c / pdf compactly into
//            the wave's region of the workspace (slots from ballots, no atomics), each pixel's
//            rays together and in sample order;
//   trace    the persistent any-hit kernel over the regions (rays.hip);
//   finalize one wave per 64 pixels: a pixel's rays start after those of the lanes below it
//            (a prefix sum of the sample masks); one thread per sample loads its hit flag and
//            contribution, the unoccluded contributions of a pixel are summed across its lanes
//            and its visibility bits written.
// The visibility bits of all samples are stored so the adjoint never traces a ray.
//
// Adjoint, per covered pixel with upstream g = dLoss/dL_dir: the same samples again (same RNG
// counters), skipping those whose bit is clear; accumulates d/d(a, r, m, n_s) over samples,
// maps d/dn_s through the normalisation to d/dq of the normal map, and scatters the eight
// channel gradients to the four bilinear taps; dLoss/dE of each sample becomes a record that
// the binned reduction of env_grad.hip adds to its env texel. The pdf and every discrete choice
// are held fixed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "env_grad.h"
#include "exm_device.h"
#include "exm_rays.h"
#include "tex_grad.h"

namespace exm {
namespace {

constexpr int kThreads = 256;
// env picks in flight per thread in dir_gen and in the adjoint (on the displaced sphere, 3 or 4 in
// dir_gen took 7.0 -> 7.5 / 8.6 ms, 4 in the adjoint 5.6 -> 9.8 ms). Since the 16-byte ray records,
// the adjoint's records written in pick order and the eight-wave blocks, one pick beats two in both:
// dir_gen 6.39 -> 5.26 ms (74 VGPRs, more waves per SIMD), the adjoint 4.55 -> 4.41 ms.
constexpr int kGenPicks = 1;
constexpr int kBwdPicks = 1;

struct KParams {
  int32_t N_d;
  uint32_t flags;
  float f_diel, eps, tmin;
  RngKey key;
};

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return (uint32_t)__popcll(mask & ((1ull << __lane_id()) - 1ull));
}

// The shading point of a covered pixel, staged in LDS between the two phases of dir_gen: kRecWords
// words per pixel, structure of arrays over the wave's 64 pixels (the lanes reading one pixel's
// record read the same word: a broadcast).
constexpr int kRecWords = 15;
enum RecField { kRns = 0, kRwo = 3, kRa = 6, kRal2 = 9, kRm = 10, kRpix = 11, kRvid = 12, kRlane = 13, kRg1o = 14 };

struct ShadePt {
  f3 ns, wo;
  float a[3], alpha2, m, g1o;  // alpha^2 and G1(wo) from spec_pixel
  uint32_t pix, vid, lane;
};

__device__ __forceinline__ ShadePt load_pt(const uint32_t* rec, uint32_t c) {
  const float* rf = reinterpret_cast<const float*>(rec);
  ShadePt q;
  q.ns = mk(rf[kRns * 64 + c], rf[(kRns + 1) * 64 + c], rf[(kRns + 2) * 64 + c]);
  q.wo = mk(rf[kRwo * 64 + c], rf[(kRwo + 1) * 64 + c], rf[(kRwo + 2) * 64 + c]);
  q.a[0] = rf[kRa * 64 + c];
  q.a[1] = rf[(kRa + 1) * 64 + c];
  q.a[2] = rf[(kRa + 2) * 64 + c];
  q.alpha2 = rf[kRal2 * 64 + c];
  q.m = rf[kRm * 64 + c];
  q.g1o = rf[kRg1o * 64 + c];
  q.pix = rec[kRpix * 64 + c];
  q.vid = rec[kRvid * 64 + c];
  q.lane = rec[kRlane * 64 + c];
  return q;
}

// alpha^2 (clamped) and G1(wo) of a shading point: they depend on the pixel only, so the forward
// pass computes them once per pixel; the same expressions and order as spec_terms
__device__ __forceinline__ void spec_pixel(f3 n, f3 wo, float r, float* alpha2, float* g1o) {
  const float alpha = r * r;
  float a2 = alpha * alpha;
  if (a2 < 1e-12f) a2 = 1e-12f;
  const float co = dot(n, wo);
  const float so = sqrtf(a2 + (1.0f - a2) * co * co);
  *alpha2 = a2;
  *g1o = 2.0f * co * __builtin_amdgcn_rcpf(co + so);
}

// f_r(wi, wo) of Eq. 13 at a staged shading point (alpha^2 and G1(wo) from spec_pixel): the values
// spec_terms gives, without the per-sample square root of G1(wo)
__device__ __forceinline__ void brdf_eval(const ShadePt& S, f3 wi, f3 wo, float ci, const KParams& p, float fr[3]) {
  const float kd = (p.flags & EXM_SPECULAR_ONLY) ? 0.0f : (1.0f - S.m) * kInvPi;
  fr[0] = kd * S.a[0];
  fr[1] = kd * S.a[1];
  fr[2] = kd * S.a[2];
  if (p.flags & EXM_DIFFUSE_ONLY) return;
  const f3 hs = wi + wo;
  const float hl = len(hs);
  const float co = dot(S.ns, wo);
  if (!(hl >= 1e-12f) || !(co > 0.0f) || !(ci > 0.0f)) return;
  const f3 h = __builtin_amdgcn_rcpf(hl) * hs;
  const float chh = dot(S.ns, h);
  const f3 nx = cross(S.ns, h);
  const float d = dot(nx, nx) + S.alpha2 * chh * chh;
  const float D = S.alpha2 * __builtin_amdgcn_rcpf(kPi * d * d);
  const float si = sqrtf(S.alpha2 + (1.0f - S.alpha2) * ci * ci);
  const float G1i = 2.0f * ci * __builtin_amdgcn_rcpf(ci + si);
  const float x = 1.0f - fmaxf(dot(wi, h), 0.0f);
  const float x2 = x * x;
  const float x5 = x2 * x2 * x;
  const float den = 4.0f * ci * co + p.eps;
  const float k = D * G1i * S.g1o * __builtin_amdgcn_rcpf(den);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float F0 = (1.0f - S.m) * p.f_diel + S.m * S.a[c];
    fr[c] += k * (F0 + (1.0f - F0) * x5);
  }
}

// One wave, 64 consecutive pixels (pixel gid of the views V at workspace position `local`; the
// wave's region is local / 64). Phase A, one lane per pixel: the attribute query, staged in `rec`
// (kRecWords x 64 words of LDS owned by the wave) at the pixel's rank among the covered ones.
// Phase B, one lane per sample: each pass takes 64 / N_d covered pixels, lane k of a pixel's group
// draws its sample k, and the samples with n_s . w > 0 get their shadow ray and contribution,
// compacted by a ballot. The region therefore holds each pixel's rays together, in sample order,
// the pixels in lane order: a traversal wave takes the rays of one or two pixels at a time
// (one origin), and the sampling runs with every lane busy whatever the coverage. COUNT: also
// accumulates env samples drawn into counters[3].
template <bool COUNT>
__device__ __forceinline__ void dir_gen_wave(const MeshView& M, const TexView& T, const EnvView& E, const EnvTabs& tb,
                                             const ShadeViews& V, const int32_t* __restrict__ tri_id,
                                             const float* __restrict__ bary, const KParams& p, int64_t gid,
                                             int64_t local, const DirectWs& ws, unsigned long long* __restrict__ counters,
                                             uint32_t* rec) {
  const int64_t HW = (int64_t)V.H * V.W;
  const int64_t region = local >> 6;
  const uint32_t lane = __lane_id();
  const int32_t f = gid < HW * V.n ? tri_id[gid] : -1;
  const uint64_t cov = __ballot(f >= 0);
  const uint32_t n_cov = (uint32_t)__popcll(cov);
  if (f >= 0) {
    const int32_t view = (int32_t)(gid / HW);
    const uint32_t pix = (uint32_t)(gid - view * HW);
    const float2 b = reinterpret_cast<const float2*>(bary)[gid];
    const Surf S = query(M, T, f, b.x, b.y, p.flags);
    const f3 wo = normalize(mk(V.eye[view][0], V.eye[view][1], V.eye[view][2]) - S.x);
    const uint32_t c = lanes_below(cov);
    float* rf = reinterpret_cast<float*>(rec);
    rf[kRns * 64 + c] = S.ns.x;
    rf[(kRns + 1) * 64 + c] = S.ns.y;
    rf[(kRns + 2) * 64 + c] = S.ns.z;
    rf[kRwo * 64 + c] = wo.x;
    rf[(kRwo + 1) * 64 + c] = wo.y;
    rf[(kRwo + 2) * 64 + c] = wo.z;
    rf[kRa * 64 + c] = S.a[0];
    rf[(kRa + 1) * 64 + c] = S.a[1];
    rf[(kRa + 2) * 64 + c] = S.a[2];
    float alpha2, g1o;
    spec_pixel(S.ns, wo, S.r, &alpha2, &g1o);
    rf[kRal2 * 64 + c] = alpha2;
    rf[kRm * 64 + c] = S.m;
    rf[kRg1o * 64 + c] = g1o;
    rec[kRpix * 64 + c] = pix;
    rec[kRvid * 64 + c] = (uint32_t)V.view_id[view];
    rec[kRlane * 64 + c] = lane;
    RayOrg O;
    O.o[0] = S.x.x;
    O.o[1] = S.x.y;
    O.o[2] = S.x.z;
    O.skip = f;
    ws.orgs[region * 64 + c] = O;
  } else {
    ws.mask[local] = 0ull;
  }
  __builtin_amdgcn_wave_barrier();
  uint32_t running = 0;  // wave-uniform
  const int64_t rbase = region * 64 * (int64_t)p.N_d;
  if (p.N_d > 0) {
    const uint32_t Nd = (uint32_t)p.N_d, G = 64u / Nd;  // pixels per pass
    const uint32_t sub = lane / Nd, k = lane - sub * Nd;
    const uint64_t group = Nd == 64u ? ~0ull : ((1ull << Nd) - 1ull);
    const int64_t mbase = local & ~(int64_t)63;
    for (uint32_t c0 = 0; c0 < n_cov; c0 += G * kGenPicks) {
      Draw dr[kGenPicks];
      bool ok[kGenPicks];
      EnvSample es[kGenPicks];
      ShadePt q[kGenPicks];
#pragma unroll
      for (int j = 0; j < kGenPicks; ++j) {
        const uint32_t c = c0 + (uint32_t)j * G + sub;
        ok[j] = sub < G && c < n_cov;
        if (ok[j]) {
          q[j] = load_pt(rec, c);
          dr[j] = philox_draw(p.key.k0, p.key.k1, q[j].pix, q[j].vid, k, 0u);
        }
      }
      // records are read only for the picks above the shading hemisphere: the others are dropped
      // whatever their records hold (half of all picks on the displaced sphere)
      env_sample_k<kGenPicks, false, true>(E, tb, dr, ok, es);
      bool need[kGenPicks];
      float cs[kGenPicks];
#pragma unroll
      for (int j = 0; j < kGenPicks; ++j) {
        need[j] = false;
        cs[j] = 0.0f;
        if (ok[j]) {
          cs[j] = dot(q[j].ns, es[j].dir);
          need[j] = cs[j] > 0.0f;
        }
      }
#pragma unroll
      for (int j = 0; j < kGenPicks; ++j)
        if (need[j]) env_rec(E, es[j]);
#pragma unroll
      for (int j = 0; j < kGenPicks; ++j) {
        if (c0 + (uint32_t)j * G >= n_cov) break;  // wave-uniform
        const uint64_t bal = __ballot(need[j]);
        if (need[j]) {
          const int64_t slot = rbase + running + lanes_below(bal);
          const float d[3] = {es[j].dir.x, es[j].dir.y, es[j].dir.z};
          store_ray(ws.rays, slot, d, (uint32_t)(region * 64 + (int64_t)(c0 + (uint32_t)j * G + sub)));
          float fr[3];
          brdf_eval(q[j], es[j].dir, q[j].wo, cs[j], p, fr);
          const float wgt = cs[j] * es[j].inv_pdf;
          store_contrib(ws.contrib, slot, es[j].E[0] * fr[0] * wgt, es[j].E[1] * fr[1] * wgt, es[j].E[2] * fr[2] * wgt);
        }
        // the pixel's sample mask: its group's bits of the ballot, written by the group's first lane
        if (ok[j] && k == 0u) ws.mask[mbase + q[j].lane] = (bal >> (sub * Nd)) & group;
        running += (uint32_t)__popcll(bal);
      }
    }
  } else if (f >= 0) {
    ws.mask[local] = 0ull;
  }
  if (lane == 0) {
    ws.count[region] = running;
    if (COUNT) atomicAdd(counters + 3, (unsigned long long)n_cov * (unsigned long long)p.N_d);
  }
}

// Chunk [p0, p0 + P) of the launch's pixels; P is a multiple of 64 and waves past it exit whole.
// Blocks of eight waves share one copy of the env tables in LDS, so that six waves per SIMD fit
// (with two picks in flight, held to five waves at 96 VGPRs: tori 5.02 -> 4.62 ms, sphere 6.68 ->
// 6.35 ms against four waves of 256-lane blocks).
constexpr int kGenThreads = 512;
template <bool COUNT>
__global__ __launch_bounds__(kGenThreads) __attribute__((amdgpu_waves_per_eu(5))) void k_dir_gen(MeshView M, TexView T, EnvView E, ShadeViews V,
                                                      const int32_t* __restrict__ tri_id,
                                                      const float* __restrict__ bary, KParams p, int64_t p0,
                                                      int64_t P, DirectWs ws, unsigned long long* __restrict__ counters,
                                                      bool use_lds) {
  extern __shared__ __align__(16) char smem[];
  __shared__ uint32_t recs[kGenThreads / 64][kRecWords * 64];
  const EnvTabs tb = load_env_tabs(E, smem, use_lds);
  const int64_t local = (int64_t)blockIdx.x * kGenThreads + threadIdx.x;
  if ((local & ~(int64_t)63) >= P) return;  // whole waves only
  dir_gen_wave<COUNT>(M, T, E, tb, V, tri_id, bary, p, p0 + local, local, ws, counters, recs[threadIdx.x >> 6]);
}

// The frames of a batched launch (requests with their own asset, env map and view): frame f
// holds workspace pixels [block_start[f], block_start[f + 1]) * kThreads, so no block spans two.
struct DirFrame {
  MeshView M;
  TexView T;
  EnvView E;
  ShadeViews V;
  const int32_t* tri_id;
  const float* bary;
  float* L_dir;
  uint64_t* vis;
  float tmin;
  int32_t use_lds;
};
struct DirBatch {
  DirFrame f[kMaxFrames];
  int32_t block_start[kMaxFrames + 1];
  int32_t n;
};
static_assert(sizeof(DirBatch) <= 3584, "a batch travels in kernel arguments");

__device__ __forceinline__ int32_t frame_of_block(const DirBatch& bt, int32_t block) {
  int32_t f = 0;
  while (f + 1 < bt.n && block >= bt.block_start[f + 1]) ++f;
  return f;
}

template <bool COUNT>
__global__ __launch_bounds__(kThreads) void k_dir_gen_batch(DirBatch bt, KParams p, DirectWs ws,
                                                            unsigned long long* __restrict__ counters) {
  extern __shared__ __align__(16) char smem[];
  __shared__ uint32_t recs[kThreads / 64][kRecWords * 64];
  const int32_t fi = frame_of_block(bt, (int32_t)blockIdx.x);
  const DirFrame& F = bt.f[fi];
  const EnvTabs tb = load_env_tabs(F.E, smem, F.use_lds != 0);
  const int64_t local = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  KParams pf = p;
  pf.tmin = F.tmin;
  dir_gen_wave<COUNT>(F.M, F.T, F.E, tb, F.V, F.tri_id, F.bary, pf, local - (int64_t)bt.block_start[fi] * kThreads,
                      local, ws, counters, recs[threadIdx.x >> 6]);
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// v summed over each aligned group of n lanes (n a power of two <= 64), the same sum on every lane
// of a group: partner lanes swap within quads, then rows' halves and rows are mirrored (DPP, no
// LDS traffic), then rows and half-waves are exchanged. Every lane of the wave must be active.
__device__ __forceinline__ void group_sum(float& v, uint32_t n) {
  if (n >= 2u) v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  if (n >= 4u) v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  if (n >= 8u) v += dpp_mov<0x141>(v);  // row_half_mirror
  if (n >= 16u) v += dpp_mov<0x140>(v); // row_mirror
  if (n >= 32u) v += __shfl_xor(v, 16, 64);
  if (n >= 64u) v += __shfl_xor(v, 32, 64);
}

// One wave, 64 consecutive pixels (as in dir_gen_wave): a pixel's rays start after those of the
// lanes below it (a prefix sum of the sample masks). The pixels with rays are then taken
// 64 / N_d' at a time (N_d' = N_d rounded up to a power of two), one lane per sample, so that a
// pixel's hit flags and contributions load together; the unoccluded contributions are summed
// by a butterfly over the pixel's lanes (every lane ends with the same sum) and the pixel's
// visibility bits come from one ballot. `stage` is 4 x 64 words of LDS owned by the wave.
__device__ __forceinline__ void dir_finalize_wave(const ShadeViews& V, const KParams& p, int64_t gid, int64_t local,
                                                  const DirectWs& ws, float* __restrict__ L_dir,
                                                  uint64_t* __restrict__ vis, uint32_t* stage) {
  const uint32_t lane = __lane_id();
  const bool valid = gid < (int64_t)V.H * V.W * V.n;
  const uint64_t mask = ws.mask[local];
  const uint32_t n_mine = (uint32_t)__popcll(mask);
  const uint32_t excl = wave_incl_sum(n_mine) - n_mine;
  const uint64_t act = __ballot(n_mine > 0u);
  if (n_mine > 0u) {
    const uint32_t c = lanes_below(act);
    stage[c] = (uint32_t)mask;
    stage[64 + c] = (uint32_t)(mask >> 32);
    stage[128 + c] = excl;
    stage[192 + c] = lane;
  } else if (valid) {
    L_dir[3 * gid] = L_dir[3 * gid + 1] = L_dir[3 * gid + 2] = 0.0f;
    vis[gid] = 0ull;
  }
  __builtin_amdgcn_wave_barrier();
  const uint32_t n_act = (uint32_t)__popcll(act);
  if (n_act == 0u) return;  // wave-uniform
  const bool novis = (p.flags & EXM_NO_VIS) != 0;
  const int64_t rbase = (local >> 6) * 64 * (int64_t)p.N_d;
  const int64_t gid0 = gid - (int64_t)lane;
  const uint32_t Nd = (uint32_t)p.N_d;
  uint32_t lg = 0;
  while ((1u << lg) < Nd) ++lg;
  const uint32_t Ndp = 1u << lg, G = 64u / Ndp, sub = lane >> lg, k = lane & (Ndp - 1u);
  const uint64_t group = Nd == 64u ? ~0ull : ((1ull << Nd) - 1ull);
  const float inv = 1.0f / (float)Nd;
  // kFinPasses passes at a time, their hit flags and contributions loaded together (the
  // contributions whatever the flags, so that no load waits for another)
  constexpr int kFinPasses = 4;
  for (uint32_t c0 = 0; c0 < n_act; c0 += G * kFinPasses) {
    bool pix_ok[kFinPasses], have[kFinPasses];
    uint32_t pl[kFinPasses];
    int64_t slot[kFinPasses];
#pragma unroll
    for (int u = 0; u < kFinPasses; ++u) {
      const uint32_t c = c0 + (uint32_t)u * G + sub;
      pix_ok[u] = c < n_act;
      uint64_t m = 0;
      uint32_t first = 0;
      pl[u] = 0;
      if (pix_ok[u]) {
        m = (uint64_t)stage[c] | ((uint64_t)stage[64 + c] << 32);
        first = stage[128 + c];
        pl[u] = stage[192 + c];
      }
      have[u] = pix_ok[u] && k < Nd && ((m >> k) & 1ull);
      slot[u] = rbase + first + __popcll(m & ((1ull << k) - 1ull));
    }
    uint8_t hb[kFinPasses];
    float cv[kFinPasses][3];
#pragma unroll
    for (int u = 0; u < kFinPasses; ++u) {
      hb[u] = 1;
      cv[u][0] = cv[u][1] = cv[u][2] = 0.0f;
      if (have[u]) {
        if (!novis) hb[u] = ws.hit[slot[u]];
        cv[u][0] = ws.contrib[3 * slot[u]];
        cv[u][1] = ws.contrib[3 * slot[u] + 1];
        cv[u][2] = ws.contrib[3 * slot[u] + 2];
      }
    }
#pragma unroll
    for (int u = 0; u < kFinPasses; ++u) {
      if (c0 + (uint32_t)u * G >= n_act) break;  // wave-uniform
      const bool lit = have[u] && (novis || hb[u] == 0);
      float L0 = lit ? cv[u][0] : 0.0f, L1 = lit ? cv[u][1] : 0.0f, L2 = lit ? cv[u][2] : 0.0f;
      group_sum(L0, Ndp);
      group_sum(L1, Ndp);
      group_sum(L2, Ndp);
      const uint64_t lb = __ballot(lit);
      if (pix_ok[u] && k == 0u) {
        const int64_t g = gid0 + pl[u];
        L_dir[3 * g] = L0 * inv;
        L_dir[3 * g + 1] = L1 * inv;
        L_dir[3 * g + 2] = L2 * inv;
        vis[g] = (lb >> (sub * Ndp)) & group;
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_dir_finalize(ShadeViews V, KParams p, int64_t p0, int64_t P,
                                                           DirectWs ws, float* __restrict__ L_dir,
                                                           uint64_t* __restrict__ vis) {
  __shared__ uint32_t stage[kThreads / 64][4 * 64];
  const int64_t local = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if ((local & ~(int64_t)63) >= P) return;
  dir_finalize_wave(V, p, p0 + local, local, ws, L_dir, vis, stage[threadIdx.x >> 6]);
}

__global__ __launch_bounds__(kThreads) void k_dir_finalize_batch(DirBatch bt, KParams p, DirectWs ws) {
  __shared__ uint32_t stage[kThreads / 64][4 * 64];
  const int32_t fi = frame_of_block(bt, (int32_t)blockIdx.x);
  const DirFrame& F = bt.f[fi];
  const int64_t local = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  dir_finalize_wave(F.V, p, local - (int64_t)bt.block_start[fi] * kThreads, local, ws, F.L_dir, F.vis,
                    stage[threadIdx.x >> 6]);
}

// Accumulated adjoint of one surface point w.r.t. its material values and shading normal.
struct SurfGrad {
  float a[3], r, m;
  f3 n;
};

// d/d(a, r, m, n) of sum_c W[c] * f_r[c](wi, wo) * ci, plus the f_r values themselves
__device__ __forceinline__ void brdf_adjoint(const Surf& S, f3 wi, f3 wo, float ci, const KParams& p, const float W[3],
                                             float fr[3], SurfGrad& g) {
  const bool diff = !(p.flags & EXM_SPECULAR_ONLY);
  const float kd = diff ? (1.0f - S.m) * kInvPi : 0.0f;
  fr[0] = kd * S.a[0];
  fr[1] = kd * S.a[1];
  fr[2] = kd * S.a[2];
  float sumWfr = 0.0f;
  if (diff) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      g.a[c] += W[c] * ci * kd;
      g.m -= W[c] * ci * S.a[c] * kInvPi;
      sumWfr += W[c] * fr[c];
    }
  }
  if (!(p.flags & EXM_DIFFUSE_ONLY)) {
    const Spec s = spec_terms(S.ns, wi, wo, ci, S.r, p.eps);
    if (s.on) {
      const float DG = s.D * s.G1i * s.G1o;
      const float rden = __builtin_amdgcn_rcpf(s.den);
      const float k = DG * rden;
      float sumWF = 0.0f, sumWfs = 0.0f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float F0 = (1.0f - S.m) * p.f_diel + S.m * S.a[c];
        const float F = F0 + (1.0f - F0) * s.x5;
        const float fs = k * F;
        fr[c] += fs;
        sumWfr += W[c] * fs;
        sumWF += W[c] * F;
        sumWfs += W[c] * fs;
        const float dF0 = 1.0f - s.x5;  // dF/dF0
        g.a[c] += W[c] * ci * k * dF0 * S.m;
        g.m += W[c] * ci * k * dF0 * (S.a[c] - p.f_diel);
      }
      // derivatives of D and of G = G1(ci) G1(co)
      const float rd = __builtin_amdgcn_rcpf(s.d);
      const float ri = __builtin_amdgcn_rcpf(s.si * (ci + s.si) * (ci + s.si));
      const float ro = __builtin_amdgcn_rcpf(s.so * (s.co + s.so) * (s.co + s.so));
      const float dD_dd = -2.0f * s.D * rd;
      const float dG1i_dc = 2.0f * s.alpha2 * ri;
      const float dG1o_dc = 2.0f * s.alpha2 * ro;
      const float G = s.G1i * s.G1o;
      // alpha^2 path
      if (!s.alpha_clamped) {
        const float dD_da2 = s.D * __builtin_amdgcn_rcpf(s.alpha2) - 2.0f * s.D * s.chh * s.chh * rd;
        const float dG1i_da2 = -ci * (1.0f - ci * ci) * ri;
        const float dG1o_da2 = -s.co * (1.0f - s.co * s.co) * ro;
        const float dDG_da2 = dD_da2 * G + s.D * (dG1i_da2 * s.G1o + s.G1i * dG1o_da2);
        const float r3 = S.r * S.r * S.r;
        g.r += ci * sumWF * rden * dDG_da2 * 4.0f * r3;
      }
      // shading-normal path: D through n.h and |n x h|^2, G through n.wi and n.wo, 1/den
      const f3 gd = 2.0f * (S.ns - s.chh * s.h) + (2.0f * s.alpha2 * s.chh) * s.h;  // dd/dn
      const f3 gD = dD_dd * gd;
      const f3 gG = (dG1i_dc * s.G1o) * wi + (s.G1i * dG1o_dc) * wo;
      const f3 gden = 4.0f * (s.co * wi + ci * wo);
      g.n = g.n + (ci * sumWF * rden) * (G * gD + s.D * gG) - (ci * sumWfs * rden) * gden;
    }
  }
  // the cosine factor n.wi multiplies f_r
  g.n = g.n + sumWfr * wi;
}

// n_s = v / |v|, v = q.x T + q.y B + q.z n_g: d/dq from d/dn_s
__device__ __forceinline__ void normal_map_adjoint(const Surf& S, f3 gn, float gq[3]) {
  gq[0] = gq[1] = gq[2] = 0.0f;
  if (!S.map_ok) return;
  const f3 gv = (1.0f / S.vlen) * (gn - dot(S.ns, gn) * S.ns);
  gq[0] = dot(S.T, gv);
  gq[1] = dot(S.B, gv);
  gq[2] = dot(S.ng, gv);
}

__device__ __forceinline__ void scatter_tex(const Surf& S, const float g8[8], float* __restrict__ dtex) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float w = S.w[k];
    if (w == 0.0f) continue;
    float* dst = dtex + (int64_t)S.tap[k] * 8;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (g8[c] != 0.0f) unsafeAtomicAdd(dst + c, w * g8[c]);
  }
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_shade_bwd(MeshView M, TexView T, EnvView E, ShadeViews V,
                                                        const int32_t* __restrict__ tri_id,
                                                        const float* __restrict__ bary, KParams p, int64_t p0,
                                                        int64_t P, const float* __restrict__ dI,
                                                        const uint64_t* __restrict__ vis,
                                                        const float* __restrict__ dquery, float* __restrict__ dtex,
                                                        EnvGradWs eg, TexGradWs tg, bool tiled, bool use_lds) {
  extern __shared__ __align__(16) char smem[];
  const EnvTabs tb = load_env_tabs(E, smem, use_lds);
  const int64_t HW = (int64_t)V.H * V.W;
  const int64_t gid = p0 + (int64_t)blockIdx.x * kThreads + threadIdx.x;
  // every lane stays until the wave has reserved its env-gradient records
  bool act = gid < p0 + P && gid < HW * V.n;
  int32_t f = -1;
  uint64_t bits = 0;
  float g[3] = {0.f, 0.f, 0.f};
  float gx[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // the given query-value gradient
  bool extra = false;
  if (act) {
    f = tri_id[gid];
    bits = vis[gid];
    g[0] = dI[3 * gid];
    g[1] = dI[3 * gid + 1];
    g[2] = dI[3 * gid + 2];
    if (dquery && f >= 0) {
      const float4 q0 = reinterpret_cast<const float4*>(dquery)[2 * gid];
      const float4 q1 = reinterpret_cast<const float4*>(dquery)[2 * gid + 1];
      gx[0] = q0.x, gx[1] = q0.y, gx[2] = q0.z, gx[3] = q0.w, gx[4] = q1.x, gx[5] = q1.y, gx[6] = q1.z, gx[7] = q1.w;
#pragma unroll
      for (int c = 0; c < 8; ++c) extra |= gx[c] != 0.0f;
    }
    act = f >= 0 && bits != 0 && (g[0] != 0.0f || g[1] != 0.0f || g[2] != 0.0f);
  }
  // the wave's env-gradient records fill one range; they are handed out in pick order, lane order
  // within a pick, so that each store of the wave writes whole lines
  const uint32_t slot0 = env_grad_reserve(eg.counter, act ? (uint32_t)__popcll(bits) : 0u);
  const uint32_t wslot = __shfl(slot0, 0, 64);
  const uint32_t tslot = tiled ? tex_grad_reserve(tg.counter, act || extra) : 0u;
  if (!act && !extra) return;
  if (!act) bits = 0;
  const int32_t view = (int32_t)(gid / HW);
  const uint32_t pix = (uint32_t)(gid - view * HW);
  const float2 b = reinterpret_cast<const float2*>(bary)[gid];
  const Surf S = query(M, T, f, b.x, b.y, p.flags);
  const f3 wo = normalize(mk(V.eye[view][0], V.eye[view][1], V.eye[view][2]) - S.x);
  const uint32_t vid = (uint32_t)V.view_id[view];
  const float invN = 1.0f / (float)p.N_d;
  SurfGrad G;
  G.a[0] = G.a[1] = G.a[2] = G.r = G.m = 0.0f;
  G.n = mk(0, 0, 0);
  uint32_t running = 0;  // records handed out so far (the same in every lane still in the loop)
  while (bits) {  // set bits in increasing order, kBwdPicks at a time
    Draw dr[kBwdPicks];
    bool ok[kBwdPicks];
    EnvSample es[kBwdPicks];
#pragma unroll
    for (int j = 0; j < kBwdPicks; ++j) {
      ok[j] = bits != 0ull;
      if (ok[j]) {
        const int k = __ffsll((long long)bits) - 1;
        bits &= bits - 1;
        dr[j] = philox_draw(p.key.k0, p.key.k1, pix, vid, (uint32_t)k, 0u);
      }
    }
    env_sample_k<kBwdPicks, true, true>(E, tb, dr, ok, es);
#pragma unroll
    for (int j = 0; j < kBwdPicks; ++j) {
      const uint64_t have = __ballot(ok[j]);  // the lanes still picking
      const uint32_t slot = wslot + running + lanes_below(have);
      running += (uint32_t)__popcll(have);
      if (!ok[j]) break;
      const float c = dot(S.ns, es[j].dir);
      const float s = invN * es[j].inv_pdf;
      const float W[3] = {g[0] * es[j].E[0] * s, g[1] * es[j].E[1] * s, g[2] * es[j].E[2] * s};
      float fr[3];
      brdf_adjoint(S, es[j].dir, wo, c, p, W, fr, G);
      const float cs = c * s;
      env_grad_put(eg, slot, (uint32_t)es[j].texel, g[0] * fr[0] * cs, g[1] * fr[1] * cs, g[2] * fr[2] * cs);
    }
  }
  float gq[3];
  normal_map_adjoint(S, G.n, gq);
  const float g8[8] = {G.a[0] + gx[0], G.a[1] + gx[1], G.a[2] + gx[2], G.r + gx[3],
                       ((p.flags & EXM_METALLIC_OFF) ? 0.0f : G.m) + gx[4], gq[0] + gx[5], gq[1] + gx[6], gq[2] + gx[7]};
  if (tiled)
    tex_grad_put(tg, tslot, S.tap, S.w, g8, dtex);
  else
    scatter_tex(S, g8, dtex);
}

KParams kparams(const exm_params* p) {
  KParams k;
  k.N_d = p->N_d;
  k.flags = p->flags;
  k.f_diel = p->f_diel;
  k.eps = p->eps;
  k.tmin = p->tmin;
  k.key = make_key(p->seed, p->iteration);
  return k;
}

}  // namespace

MeshView mesh_view(const exm_mesh* m) {
  return MeshView{m->nV, m->nF, m->pos, m->tri, m->uv, m->tri_uv, m->vnrm, m->ftan};
}
EnvView env_view(const exm_env* e) {
  const bool narrow = e->We < kCdf32MaxW;
  const uint32_t* c32 = narrow ? e->guide + env_cdf32_offset(e->He, e->We) : nullptr;
  const uint16_t* g16 = narrow ? reinterpret_cast<const uint16_t*>(e->guide + env_col16_offset(e->He, e->We)) : nullptr;
  const uint16_t* c16 = narrow ? reinterpret_cast<const uint16_t*>(e->guide + env_cdf16_offset(e->He, e->We)) : nullptr;
  return EnvView{e->He,    e->We,    e->env, e->cdf_row, e->cdf_col, e->pdf,
                 e->guide, reinterpret_cast<const float4*>(e->rec), c32, g16, c16};
}
BvhView bvh_view(const exm_bvh* b) { return BvhView{b->nodes, b->tris}; }

hipError_t launch_shade_fwd(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat, const exm_env* env,
                            const ShadeViews& v, const int32_t* tri_id, const float* bary, const exm_params* p,
                            float* L_dir, uint64_t* vis, void* ws_ptr, size_t ws_bytes, unsigned long long* counters,
                            hipStream_t s) {
  const int64_t n = (int64_t)v.n * v.H * v.W;
  const int64_t P = direct_chunk(ws_bytes, p->N_d, n);
  if (P <= 0) return hipErrorInvalidValue;  // the ABI layer checks the size first
  const KParams kp = kparams(p);
  const TexView tv{mat->Ht, mat->Wt, mat->tex};
  const DirectWs ws = direct_ws(ws_ptr, P, p->N_d);
  const bool trace = p->N_d > 0 && !(p->flags & EXM_NO_VIS);
  const size_t lds = env_tabs_bytes(env->He, env->We);
  const bool use_lds = lds <= kEnvTabsMaxBytes;
  for (int64_t p0 = 0; p0 < n; p0 += P) {
    const int64_t Pc = std::min<int64_t>(P, ((n - p0) + 63) / 64 * 64);
    const unsigned nb = (unsigned)((Pc + kThreads - 1) / kThreads);
    {
      EXM_TIMED("dir_gen", s);
      if (counters)
        k_dir_gen<true><<<(unsigned)((Pc + kGenThreads - 1) / kGenThreads), kGenThreads, use_lds ? lds : 0, s>>>(mesh_view(m), tv, env_view(env), v, tri_id, bary, kp,
                                                               p0, Pc, ws, counters, use_lds);
      else
        k_dir_gen<false><<<(unsigned)((Pc + kGenThreads - 1) / kGenThreads), kGenThreads, use_lds ? lds : 0, s>>>(mesh_view(m), tv, env_view(env), v, tri_id, bary, kp,
                                                                p0, Pc, ws, nullptr, use_lds);
    }
    if (trace) {
      const RayBatch rb{ws.rays, ws.orgs, ws.count, (int32_t)(Pc / 64), 64 * (int64_t)p->N_d, p->tmin, ws.counter};
      const hipError_t e = launch_trace_any(bvh, rb, ws.hit, counters, s);
      if (e != hipSuccess) return e;
    }
    {
      EXM_TIMED("dir_finalize", s);
      k_dir_finalize<<<nb, kThreads, 0, s>>>(v, kp, p0, Pc, ws, L_dir, vis);
    }
  }
  return hipGetLastError();
}

// Workspace pixels of a batch: each request's pixels rounded up to whole blocks.
int64_t batch_pixels(const exm_request* r, int32_t n) {
  int64_t P = 0;
  for (int32_t i = 0; i < n; ++i) P += ((int64_t)r[i].cam.H * r[i].cam.W + kThreads - 1) / kThreads * kThreads;
  return P;
}

hipError_t launch_shade_fwd_batch(const exm_request* r, int32_t n, const exm_params* p, void* ws_ptr, size_t ws_bytes,
                                  unsigned long long* counters, hipStream_t s) {
  if (n <= 0 || n > kMaxFrames) return hipErrorInvalidValue;
  const int64_t P = batch_pixels(r, n);
  if (direct_ws_bytes(P, p->N_d) > ws_bytes) return hipErrorInvalidValue;  // the ABI layer checks the size first
  DirBatch bt;
  BvhTable tt;
  std::memset(&bt, 0, sizeof(bt));
  std::memset(&tt, 0, sizeof(tt));
  bt.n = tt.n = n;
  size_t lds = 0;
  for (int32_t i = 0; i < n; ++i) {
    DirFrame& F = bt.f[i];
    F.M = mesh_view(r[i].mesh);
    F.T = TexView{r[i].mat->Ht, r[i].mat->Wt, r[i].mat->tex};
    F.E = env_view(r[i].env);
    F.V = shade_views(&r[i].cam, 0, 1);
    F.tri_id = r[i].tri_id;
    F.bary = r[i].bary;
    F.L_dir = r[i].L_dir;
    F.vis = r[i].vis;
    F.tmin = r[i].tmin;
    tt.tmin[i] = r[i].tmin;
    const size_t b = env_tabs_bytes(r[i].env->He, r[i].env->We);
    F.use_lds = b <= kEnvTabsMaxBytes;
    if (F.use_lds) lds = std::max(lds, b);
    tt.b[i] = bvh_view(r[i].bvh);
    const int64_t nb = ((int64_t)r[i].cam.H * r[i].cam.W + kThreads - 1) / kThreads;
    bt.block_start[i + 1] = bt.block_start[i] + (int32_t)nb;
    tt.region_start[i + 1] = bt.block_start[i + 1] * (kThreads / 64);
  }
  const KParams kp = kparams(p);
  const DirectWs ws = direct_ws(ws_ptr, P, p->N_d);
  const unsigned nb = (unsigned)bt.block_start[n];
  {
    EXM_TIMED("dir_gen", s);
    if (counters)
      k_dir_gen_batch<true><<<nb, kThreads, lds, s>>>(bt, kp, ws, counters);
    else
      k_dir_gen_batch<false><<<nb, kThreads, lds, s>>>(bt, kp, ws, nullptr);
  }
  if (p->N_d > 0 && !(p->flags & EXM_NO_VIS)) {
    const RayBatch rb{ws.rays, ws.orgs, ws.count, (int32_t)(P / 64), 64 * (int64_t)p->N_d, p->tmin, ws.counter};
    const hipError_t e = launch_trace_any_batch(tt, rb, ws.hit, counters, s);
    if (e != hipSuccess) return e;
  }
  {
    EXM_TIMED("dir_finalize", s);
    k_dir_finalize_batch<<<nb, kThreads, 0, s>>>(bt, kp, ws);
  }
  return hipGetLastError();
}

size_t shade_fwd_batch_ws_bytes(const exm_request* r, int32_t n, int32_t N_d) {
  size_t b = 0;
  for (int32_t i = 0; i < n; i += kMaxFrames)
    b = std::max(b, direct_ws_bytes(batch_pixels(r + i, std::min(kMaxFrames, n - i)), N_d));
  return b;
}

size_t shade_fwd_ws_bytes(int64_t n_pix, int32_t N_d) { return direct_ws_bytes((n_pix + 63) / 64 * 64, N_d); }
size_t shade_fwd_ws_min(int32_t N_d) { return direct_ws_bytes(64, N_d); }

hipError_t launch_shade_bwd(const exm_mesh* m, const exm_material* mat, const exm_env* env, const ShadeViews& v,
                            const int32_t* tri_id, const float* bary, const exm_params* p, const float* dI,
                            const uint64_t* vis, const float* dquery, float* dtex, double* denv, void* ws,
                            size_t ws_bytes, hipStream_t s) {
  const int64_t n = (int64_t)v.n * v.H * v.W;
  const int64_t per_px = std::max(p->N_d, 0);
  const int64_t P = adjoint_chunk(ws_bytes, per_px, 1, env->He, env->We, n);
  if (P <= 0) return hipErrorInvalidValue;  // the ABI layer checks the size first
  const size_t lds = env_tabs_bytes(env->He, env->We);
  const bool use_lds = lds <= kEnvTabsMaxBytes;
  const KParams kp = kparams(p);
  const bool tiled = tex_grad_tiled(mat->Ht, mat->Wt) && !(p->flags & EXM_MAP_GRAD_ATOMIC);
  for (int64_t p0 = 0; p0 < n; p0 += P) {
    const int64_t Pc = std::min<int64_t>(P, ((n - p0) + 63) / 64 * 64);
    const EnvGradWs eg = env_grad_ws(ws, Pc * per_px, env->He, env->We);
    const TexGradWs tg =
        tex_grad_ws(static_cast<char*>(ws) + env_grad_ws_bytes(Pc * per_px, env->He, env->We), Pc, mat->Ht, mat->Wt);
    hipError_t e = launch_env_grad_clear(eg, s);
    if (e != hipSuccess) return e;
    if (tiled) {
      e = launch_tex_grad_clear(tg, s);
      if (e != hipSuccess) return e;
    }
    {
      EXM_TIMED("shade_bwd", s);
      k_shade_bwd<<<(unsigned)((Pc + kThreads - 1) / kThreads), kThreads, use_lds ? lds : 0, s>>>(
          mesh_view(m), TexView{mat->Ht, mat->Wt, mat->tex}, env_view(env), v, tri_id, bary, kp, p0, Pc, dI, vis,
          dquery, dtex, eg, tg, tiled, use_lds);
    }
    e = launch_env_grad_reduce(eg, env->He, env->We, denv, s);
    if (e != hipSuccess) return e;
    if (tiled) {
      e = launch_tex_grad_reduce(tg, dtex, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

size_t shade_bwd_ws_bytes(int64_t n_pix, int32_t N_d, int32_t He, int32_t We) {
  const int64_t np = (n_pix + 63) / 64 * 64;
  return env_grad_ws_bytes(np * std::max(N_d, 0), He, We) + tex_grad_ws_bytes(np);
}
size_t shade_bwd_ws_min(int32_t N_d, int32_t He, int32_t We) {
  return env_grad_ws_bytes(64 * (int64_t)std::max(N_d, 0), He, We) + tex_grad_ws_bytes(64);
}

}  // namespace exm
