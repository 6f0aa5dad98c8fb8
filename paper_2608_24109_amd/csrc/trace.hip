// One-bounce diffuse indirect illumination (One-Bounce Indirect Illumination, Eq. 18-19)
// and its adjoint.
//
// Forward, per covered pixel x: N_b directions w_j cosine-weighted about n_g(x) (Malley's
// method in the Duff et al. orthonormal basis; p_b = max(n_g . w, 0) / pi); closest hit from
// x (t >= t_min, the origin triangle skipped); the hit counts only if it is front facing.
// At a valid hit y: the same attribute query as for primary points, then N_s env samples with
// shadow rays give the diffuse radiance L_sec(y) (Eq. 18, no specular term). Eq. 19 sums
// 1_hit f_d(x) L_sec(y_j) max(n_s(x) . w_j, 0) / p_b over j and divides by N_b.
// It runs per chunk of pixels as gen1 (secondary rays) -> closest-hit trace -> gen2 (hit
// validity, FP64 refinement, query at y, light samples with their shadow rays and their whole
// contribution f_d(x) f_d(y) E c / pdf * (n_s(x).w / p_b) / (N_b N_s)) -> any-hit trace ->
// finalize (sum of the unoccluded contributions in (j, s) order). A covered pixel's N_b secondary
// rays sit together (the covered pixels of a wave ranked by a ballot), so a traversal wave takes
// rays of few origins at a time; gen2 runs one lane per (pixel, secondary ray) pair and then one
// per valid pair, and keeps each light sample's shadow-ray slot (from wave ballots) for finalize.
// The hit records and the light-sample visibility bits are stored for the adjoint.
//
// Adjoint, for upstream G = lambda_ind dLoss/dI: gradients to a, m, n_s at x (through f_d(x)
// and the cosine) and at each y_j (through f_d(y) and n_s(y)), and to E at the light samples.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "env_grad.h"
#include "tex_grad.h"
#include "exm_device.h"
#include "exm_rays.h"

namespace exm {

MeshView mesh_view(const exm_mesh* m);
EnvView env_view(const exm_env* e);
BvhView bvh_view(const exm_bvh* b);

namespace {

constexpr int kThreads = 256;

struct KParams {
  int32_t N_b, N_s;
  uint32_t flags;
  float tmin;
  RngKey key;
};

// Secondary ray in FP64: origin x from the G-buffer barycentrics, n_g from the vertex normals,
// w cosine-weighted about n_g (Malley's method in the Duff et al. 2017 basis), p_b = n_g.w/pi.
// The hit point's barycentrics are refined in FP64 on the triangle the FP32 traversal found:
// with i.i.d. texels a float hit point (error ~1e-7 of the scene size) would already move the
// secondary material by 1e-4 on 1M-triangle meshes with 2048^2 maps.
struct SecRay {
  double o[3], d[3];
  f3 of, df;
  float pb;
};

__device__ __forceinline__ SecRay secondary_ray(const MeshView& M, int32_t f, float b1, float b2, float u2, float u3) {
  SecRay r;
  const double d1 = b1, d2 = b2, d0 = 1.0 - d1 - d2;
  const int32_t v[3] = {M.tri[3 * f], M.tri[3 * f + 1], M.tri[3 * f + 2]};
  const double w[3] = {d0, d1, d2};
  double n[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a) r.o[a] = 0.0;
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < 3; ++a) {
      r.o[a] += w[k] * (double)M.pos[3 * v[k] + a];
      n[a] += w[k] * (double)M.vnrm[3 * v[k] + a];
    }
  const double nl = 1.0 / sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  n[0] *= nl;
  n[1] *= nl;
  n[2] *= nl;
  const double sign = copysign(1.0, n[2]);
  const double a = -1.0 / (sign + n[2]);
  const double bb = n[0] * n[1] * a;
  const double e1[3] = {1.0 + sign * n[0] * n[0] * a, sign * bb, -sign * n[0]};
  const double e2[3] = {bb, sign + n[1] * n[1] * a, -n[1]};
  const double rr = sqrt((double)u2);
  double sp, cp;
  sincospi(2.0 * (double)u3, &sp, &cp);
  const double lz = sqrt(fmax(0.0, 1.0 - (double)u2));
  for (int k = 0; k < 3; ++k) r.d[k] = (rr * cp) * e1[k] + (rr * sp) * e2[k] + lz * n[k];
  const double cg = n[0] * r.d[0] + n[1] * r.d[1] + n[2] * r.d[2];
  r.pb = (float)(fmax(cg, 0.0) / 3.14159265358979323846);
  r.of = mk((float)r.o[0], (float)r.o[1], (float)r.o[2]);
  r.df = mk((float)r.d[0], (float)r.d[1], (float)r.d[2]);
  return r;
}

// FP64 Moller-Trumbore on triangle f for the FP64 ray; keeps (b1, b2) if the ray is parallel
__device__ __forceinline__ void refine_hit(const MeshView& M, int32_t f, const SecRay& r, float* b1, float* b2) {
  const int32_t v0 = M.tri[3 * f], v1 = M.tri[3 * f + 1], v2 = M.tri[3 * f + 2];
  double p0[3], e1[3], e2[3];
  for (int a = 0; a < 3; ++a) {
    p0[a] = M.pos[3 * v0 + a];
    e1[a] = (double)M.pos[3 * v1 + a] - p0[a];
    e2[a] = (double)M.pos[3 * v2 + a] - p0[a];
  }
  const double pv[3] = {r.d[1] * e2[2] - r.d[2] * e2[1], r.d[2] * e2[0] - r.d[0] * e2[2],
                        r.d[0] * e2[1] - r.d[1] * e2[0]};
  const double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
  if (det == 0.0) return;
  const double inv = 1.0 / det;
  const double tv[3] = {r.o[0] - p0[0], r.o[1] - p0[1], r.o[2] - p0[2]};
  const double u = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
  const double qv[3] = {tv[1] * e1[2] - tv[2] * e1[1], tv[2] * e1[0] - tv[0] * e1[2], tv[0] * e1[1] - tv[1] * e1[0]};
  const double w = (r.d[0] * qv[0] + r.d[1] * qv[1] + r.d[2] * qv[2]) * inv;
  // the FP32 traversal decided the hit; keep the refined point on the triangle
  const double uc = fmin(1.0, fmax(0.0, u)), wc = fmin(1.0 - uc, fmax(0.0, w));
  *b1 = (float)uc;
  *b2 = (float)wc;
}

__device__ __forceinline__ bool front_facing(const MeshView& M, int32_t f, f3 w) {
  const int32_t v0 = M.tri[3 * f], v1 = M.tri[3 * f + 1], v2 = M.tri[3 * f + 2];
  const f3 P0 = ld3(M.pos, v0), P1 = ld3(M.pos, v1), P2 = ld3(M.pos, v2);
  return dot(w, cross(P1 - P0, P2 - P0)) < 0.0f;
}

// index of the n-th set bit (from 0) of m, which has more than n set bits
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t m, uint32_t n) {
  uint32_t pos = 0, cnt = 0;
#pragma unroll
  for (uint32_t step = 32; step > 0; step >>= 1) {
    const uint32_t c = (uint32_t)__popcll((m >> pos) & ((1ull << step) - 1ull));
    if (cnt + c <= n) {
      cnt += c;
      pos += step;
    }
  }
  return pos;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return (uint32_t)__popcll(mask & ((1ull << __lane_id()) - 1ull));
}

// One wave per 64 consecutive pixels, one lane per (covered pixel, secondary ray) pair: pair q is
// ray q % N_b of the wave's (q / N_b)-th covered pixel, and its ray goes to slot q of the region,
// so a pixel's rays lie together.
__global__ __launch_bounds__(kThreads) void k_ind_gen1(MeshView M, ShadeViews V, const int32_t* __restrict__ tri_id,
                                                       const float* __restrict__ bary, KParams p, int64_t p0,
                                                       int64_t P, IndirectWs ws) {
  const int64_t local = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if ((local & ~(int64_t)63) >= P) return;  // whole waves only
  const int64_t HW = (int64_t)V.H * V.W;
  const int64_t gid = p0 + local;
  const int64_t gid0 = gid - (int64_t)__lane_id();
  const int32_t f = gid < HW * V.n ? tri_id[gid] : -1;
  const int64_t region = local >> 6;
  const int64_t rbase = region * 64 * (int64_t)p.N_b;
  const uint64_t bal = __ballot(f >= 0);
  const uint32_t n_cov = (uint32_t)__popcll(bal);
  const uint32_t total = n_cov * (uint32_t)max(p.N_b, 0);
  for (uint32_t q = __lane_id(); q < total; q += 64) {
    const uint32_t below = q / (uint32_t)p.N_b, j = q - below * (uint32_t)p.N_b;
    const int64_t pg = gid0 + (int64_t)nth_set_bit(bal, below);
    const int32_t pf = tri_id[pg];
    const int32_t view = (int32_t)(pg / HW);
    const uint32_t pix = (uint32_t)(pg - view * HW), vid = (uint32_t)V.view_id[view];
    const float2 b = reinterpret_cast<const float2*>(bary)[pg];
    const Draw d = philox_draw(p.key.k0, p.key.k1, pix, vid, j, 1u);
    const SecRay sr = secondary_ray(M, pf, b.x, b.y, d.u2, d.u3);
    const int64_t org = region * 64 + (int64_t)below;
    if (j == 0) {  // the origin does not depend on the ray: written by the pixel's first pair
      RayOrg O;
      O.o[0] = sr.of.x;
      O.o[1] = sr.of.y;
      O.o[2] = sr.of.z;
      O.skip = pf;
      ws.sec_orgs[org] = O;
    }
    const float d3[3] = {sr.df.x, sr.df.y, sr.df.z};
    store_ray(ws.sec_rays, rbase + q, d3, (uint32_t)org);
  }
  if (__lane_id() == 0) ws.sec_count[region] = total;
}

// Per-wave staging of the light-sample stage: the covered pixels' values that their secondary
// points need (indexed by the pixel's rank among the wave's covered pixels), a queue of the valid
// (pixel, j) pairs in pair order, and each covered pixel's light-sample mask.
constexpr int kIndPixWords = 12;
enum IndPixField { kIf = 0, kIb1, kIb2, kIpix, kIvid, kIlane, kIfa, kIns = kIfa + 3 };
static_assert(kIns + 3 == kIndPixWords, "staged words");
constexpr int kIndQ = 128;  // queue capacity: fewer than 64 waiting pairs plus one chunk of 64
constexpr int kIndQWords = 5;
enum IndQField { kQq = 0, kQhit, kQb1, kQb2, kQw };
struct IndStage {
  uint32_t px[kIndPixWords * 64];
  uint32_t qe[kIndQWords * kIndQ];
  uint64_t mask[64];
};

// The queued valid pairs [0, n) of a wave (n <= 64), one lane each: the query at y and the N_s
// light samples. A sample whose shadow ray is needed gets the region's next slot (in order of
// sample index, then queue position); the slot is kept per (pixel, sample) for the finalize
// kernel and the sample's bit is set in the pixel's mask.
__device__ __forceinline__ void ind_light_samples(const MeshView& M, const TexView& T, const EnvView& E,
                                                  const EnvTabs& tb, const KParams& p, IndStage& st, uint32_t n,
                                                  int64_t wave_local0, int64_t rbase1, int64_t rbase2, uint32_t& running,
                                                  const IndirectWs& ws) {
  const uint32_t lane = __lane_id();
  const bool act = lane < n;
  const bool diff = !(p.flags & EXM_SPECULAR_ONLY);
  const int n_slots = p.N_b * p.N_s;
  uint32_t below = 0, j = 0, pix = 0, vid = 0, plane = 0, org = 0;
  int32_t hid = -1;
  float fac[3] = {0.f, 0.f, 0.f};
  Surf Y;
  uint64_t bits = 0;
  if (act) {
    const float* qf = reinterpret_cast<const float*>(st.qe);
    const uint32_t q = st.qe[kQq * kIndQ + lane];
    org = (uint32_t)(rbase1 + (int64_t)q);  // the pair's secondary-ray slot
    hid = (int32_t)st.qe[kQhit * kIndQ + lane];
    const float b1 = qf[kQb1 * kIndQ + lane], b2 = qf[kQb2 * kIndQ + lane], w = qf[kQw * kIndQ + lane];
    below = q / (uint32_t)p.N_b;
    j = q - below * (uint32_t)p.N_b;
    pix = st.px[kIpix * 64 + below];
    vid = st.px[kIvid * 64 + below];
    plane = st.px[kIlane * 64 + below];
    const float* pf = reinterpret_cast<const float*>(st.px);
    Y = query(M, T, hid, b1, b2, p.flags, !(p.flags & EXM_NO_SECONDARY_MATERIAL));
    const float kdy = diff ? (1.0f - Y.m) * kInvPi : 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) fac[c] = pf[(kIfa + c) * 64 + below] * (kdy * Y.a[c]) * w;
    RayOrg O;
    O.o[0] = Y.x.x;
    O.o[1] = Y.x.y;
    O.o[2] = Y.x.z;
    O.skip = hid;
    ws.sh_orgs[org] = O;
  }
  for (int s2 = 0; s2 < p.N_s; ++s2) {
    bool need = false;
    EnvSample es;
    float c = 0.0f;
    if (act) {
      es = env_sample(E, tb, philox_draw(p.key.k0, p.key.k1, pix, vid, (uint32_t)s2, 2u + j));
      c = dot(Y.ns, es.dir);
      need = c > 0.0f;
    }
    const uint64_t bal = __ballot(need);
    if (need) {
      const uint32_t rel = running + lanes_below(bal);
      const int64_t slot = rbase2 + rel;
      const float d3[3] = {es.dir.x, es.dir.y, es.dir.z};
      store_ray(ws.sh_rays, slot, d3, org);
      const float* e = es.E;
      const float wgt = c * es.inv_pdf;
      store_contrib(ws.sh_contrib, slot, fac[0] * e[0] * wgt, fac[1] * e[1] * wgt, fac[2] * e[2] * wgt);
      const uint32_t t = j * (uint32_t)p.N_s + (uint32_t)s2;
      ws.sh_slot[(wave_local0 + plane) * n_slots + t] = rel;
      bits |= 1ull << t;
    }
    running += (uint32_t)__popcll(bal);
  }
  if (bits) atomicOr(&st.mask[below], bits);
}

// One wave per 64 consecutive pixels. The covered pixels' secondary rays lie together in pixel
// order (k_ind_gen1), so pair q of the wave is ray q % N_b of its (q / N_b)-th covered pixel. One
// lane per pair tests the hit (validity, FP64 refinement, the record for the adjoint), 64 pairs at a
// time; the valid pairs wait in LDS and their light samples run 64 pairs at a time as well, so
// lanes are idle neither for uncovered pixels nor for missed or back-facing secondary rays. Blocks
// of eight waves share one copy of the env tables in LDS, so that four waves per SIMD fit beside the
// per-wave staging (held to 128 VGPRs: tori 1.43 -> 1.15 ms against three waves of 256-lane blocks).
constexpr int kIg2Threads = 512;
__global__ __launch_bounds__(kIg2Threads) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_ind_gen2(MeshView M, TexView T, EnvView E, ShadeViews V,
                                                       const int32_t* __restrict__ tri_id,
                                                       const float* __restrict__ bary, KParams p, int64_t p0,
                                                       int64_t P, IndirectWs ws, exm_sec_rec* __restrict__ rec,
                                                       bool use_lds) {
  extern __shared__ __align__(16) char smem[];
  __shared__ IndStage stage_all[kIg2Threads / 64];
  IndStage& st = stage_all[threadIdx.x >> 6];
  const EnvTabs tb = load_env_tabs(E, smem, use_lds);
  const int64_t local = (int64_t)blockIdx.x * kIg2Threads + threadIdx.x;
  if ((local & ~(int64_t)63) >= P) return;
  const uint32_t lane = __lane_id();
  const int64_t HW = (int64_t)V.H * V.W;
  const int64_t gid = p0 + local;
  const int64_t gid0 = gid - (int64_t)lane, wave_local0 = local - (int64_t)lane;
  const bool in_range = gid < HW * V.n;
  const int32_t f = in_range ? tri_id[gid] : -1;
  const int64_t region = local >> 6;
  const int64_t rbase1 = region * 64 * (int64_t)p.N_b;
  const int64_t rbase2 = rbase1 * (int64_t)p.N_s;
  const uint64_t bal1 = __ballot(f >= 0);
  const uint32_t below1 = lanes_below(bal1), n_cov = (uint32_t)__popcll(bal1);
  const bool diff = !(p.flags & EXM_SPECULAR_ONLY);
  const float invNbNs = (p.N_b > 0 && p.N_s > 0) ? 1.0f / ((float)p.N_b * (float)p.N_s) : 0.0f;
  st.mask[lane] = 0ull;
  if (f >= 0) {
    const int32_t view = (int32_t)(gid / HW);
    const uint32_t pix = (uint32_t)(gid - view * HW);
    const float2 b = reinterpret_cast<const float2*>(bary)[gid];
    const Surf S = query(M, T, f, b.x, b.y, p.flags);
    const float kdx = diff ? (1.0f - S.m) * kInvPi : 0.0f;
    float* pf = reinterpret_cast<float*>(st.px);
    st.px[kIf * 64 + below1] = (uint32_t)f;
    pf[kIb1 * 64 + below1] = b.x;
    pf[kIb2 * 64 + below1] = b.y;
    st.px[kIpix * 64 + below1] = pix;
    st.px[kIvid * 64 + below1] = (uint32_t)V.view_id[view];
    st.px[kIlane * 64 + below1] = lane;
#pragma unroll
    for (int c = 0; c < 3; ++c) pf[(kIfa + c) * 64 + below1] = kdx * S.a[c];
    pf[kIns * 64 + below1] = S.ns.x;
    pf[(kIns + 1) * 64 + below1] = S.ns.y;
    pf[(kIns + 2) * 64 + below1] = S.ns.z;
  } else if (in_range) {
    for (int j = 0; j < p.N_b; ++j) rec[gid * p.N_b + j] = exm_sec_rec{-1, 0.f, 0.f};
  }
  __builtin_amdgcn_wave_barrier();
  const uint32_t total = n_cov * (uint32_t)max(p.N_b, 0);  // wave-uniform
  uint32_t qn = 0, running = 0;                             // wave-uniform
  for (uint32_t c0 = 0; c0 < total; c0 += 64) {
    const uint32_t q = c0 + lane;
    bool valid = false;
    int32_t hid = -1;
    float hb1 = 0.0f, hb2 = 0.0f, w = 0.0f;
    if (q < total) {
      const uint32_t below = q / (uint32_t)p.N_b, j = q - below * (uint32_t)p.N_b;
      const float* pf = reinterpret_cast<const float*>(st.px);
      const int32_t pf_tri = (int32_t)st.px[kIf * 64 + below];
      const float b1 = pf[kIb1 * 64 + below], b2 = pf[kIb2 * 64 + below];
      const uint32_t pix = st.px[kIpix * 64 + below], vid = st.px[kIvid * 64 + below];
      const uint32_t plane = st.px[kIlane * 64 + below];
      const f3 ns = mk(pf[kIns * 64 + below], pf[(kIns + 1) * 64 + below], pf[(kIns + 2) * 64 + below]);
      HitRec h = ws.sec_hits[rbase1 + q];
      const Draw d = philox_draw(p.key.k0, p.key.k1, pix, vid, j, 1u);
      const SecRay sr = secondary_ray(M, pf_tri, b1, b2, d.u2, d.u3);
      exm_sec_rec r{-1, 0.f, 0.f};
      if (h.id >= 0 && front_facing(M, h.id, sr.df)) {
        refine_hit(M, h.id, sr, &h.b1, &h.b2);
        r = exm_sec_rec{h.id, h.b1, h.b2};
        const float cx = fmaxf(dot(ns, sr.df), 0.0f);
        w = cx / sr.pb * invNbNs;
        hid = h.id;
        hb1 = h.b1;
        hb2 = h.b2;
        valid = true;
      }
      rec[(gid0 + (int64_t)plane) * p.N_b + j] = r;
    }
    const uint64_t vb = __ballot(valid);
    if (valid) {
      const uint32_t at = qn + lanes_below(vb);
      float* qf = reinterpret_cast<float*>(st.qe);
      st.qe[kQq * kIndQ + at] = q;
      st.qe[kQhit * kIndQ + at] = (uint32_t)hid;
      qf[kQb1 * kIndQ + at] = hb1;
      qf[kQb2 * kIndQ + at] = hb2;
      qf[kQw * kIndQ + at] = w;
    }
    qn += (uint32_t)__popcll(vb);
    __builtin_amdgcn_wave_barrier();
    if (qn >= 64) {
      ind_light_samples(M, T, E, tb, p, st, 64u, wave_local0, rbase1, rbase2, running, ws);
      // the waiting pairs (fewer than 64) move to the front of the queue
      const bool mv = lane + 64u < qn;
      uint32_t e[kIndQWords];
#pragma unroll
      for (int k = 0; k < kIndQWords; ++k) e[k] = mv ? st.qe[k * kIndQ + 64 + lane] : 0u;
      __builtin_amdgcn_wave_barrier();
      if (mv) {
#pragma unroll
        for (int k = 0; k < kIndQWords; ++k) st.qe[k * kIndQ + lane] = e[k];
      }
      qn -= 64u;
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (qn > 0) ind_light_samples(M, T, E, tb, p, st, qn, wave_local0, rbase1, rbase2, running, ws);
  __builtin_amdgcn_wave_barrier();
  ws.sh_mask[local] = f >= 0 ? st.mask[below1] : 0ull;
  if (lane == 0) ws.sh_count[region] = running;
}

// Per pixel: the unoccluded light samples' contributions summed in (j, s) order, their bits kept
// for the adjoint.
__global__ __launch_bounds__(kThreads) void k_ind_finalize(ShadeViews V, KParams p, int64_t p0, int64_t P,
                                                           IndirectWs ws, float* __restrict__ L_ind,
                                                           uint64_t* __restrict__ sec_vis) {
  const int64_t local = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (local >= P) return;
  const int64_t gid = p0 + local;
  if (gid >= (int64_t)V.H * V.W * V.n) return;
  const uint64_t mask = ws.sh_mask[local];
  const bool novis = (p.flags & EXM_NO_VIS) != 0;
  const int64_t rbase = (local >> 6) * 64 * (int64_t)p.N_b * p.N_s;
  const int64_t n_slots = (int64_t)p.N_b * p.N_s;
  float L[3] = {0.f, 0.f, 0.f};
  uint64_t bits = 0;
  for (uint64_t m = mask; m != 0ull; m &= m - 1ull) {
    const int t = __ffsll((long long)m) - 1;
    const int64_t slot = rbase + ws.sh_slot[local * n_slots + t];
    if (novis || ws.sh_hit[slot] == 0) {
      bits |= 1ull << t;
      L[0] += ws.sh_contrib[3 * slot];
      L[1] += ws.sh_contrib[3 * slot + 1];
      L[2] += ws.sh_contrib[3 * slot + 2];
    }
  }
  L_ind[3 * gid] = L[0];
  L_ind[3 * gid + 1] = L[1];
  L_ind[3 * gid + 2] = L[2];
  sec_vis[gid] = bits;
}

// the map adjoint of one surface point (roughness has none here: f_d does not depend on it), as a
// record of the tiled reduction in `slot`, or with one atomic per tap and channel
__device__ __forceinline__ void scatter7(const Surf& S, const float ga[3], float gm, const float gq[3],
                                         float* __restrict__ dtex, const TexGradWs& tg, bool tiled, uint32_t slot) {
  const float g8[8] = {ga[0], ga[1], ga[2], 0.0f, gm, gq[0], gq[1], gq[2]};
  if (tiled) {
    tex_grad_put(tg, slot, S.tap, S.w, g8, dtex);
    return;
  }
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

__device__ __forceinline__ void nmap_adjoint(const Surf& S, f3 gn, float gq[3]) {
  gq[0] = gq[1] = gq[2] = 0.0f;
  if (!S.map_ok) return;
  const f3 gv = (1.0f / S.vlen) * (gn - dot(S.ns, gn) * S.ns);
  gq[0] = dot(S.T, gv);
  gq[1] = dot(S.B, gv);
  gq[2] = dot(S.ng, gv);
}

// secondary light samples per secondary point kept between the adjoint's two passes (the others are
// drawn again in the second pass): one frees the registers of three (tori 1.49 -> 1.44 ms; two: 1.50)
constexpr int kCacheS = 1;


// Per-wave staging of the indirect adjoint: the pixels' values the secondary points need, the
// (pixel, secondary ray) pairs of each ray index j (a ballot mask and the index of its first pair),
// and each pair's contribution to its pixel's x-side gradient (d/d f_d(x), d/d n_s(x)).
constexpr int kBwdPixWords = 20;
enum BwdPixField {
  kBf = 0, kBb1, kBb2, kBpix, kBvid, kBfdx, kBns = kBfdx + 3, kBG = kBns + 3, kBslot = kBG + 3, kBtslot, kBbits,
  kBvm = kBbits + 2
};
static_assert(kBvm + 2 == kBwdPixWords, "staged words");
struct BwdStage {
  uint32_t px[kBwdPixWords * 64];
  float pair[6 * 64];
  uint64_t bal[64];
  uint32_t base[65];
};

// One wave per 64 consecutive pixels. The work of a valid secondary hit (its secondary ray, the
// query at y, the light samples, the env-map records and the map record of y) runs one lane per
// (pixel, j) pair, the wave's pairs taken 64 at a time, so that lanes are not left idle by pixels
// with fewer valid hits; each chunk's contributions to the x side are added by the pixel's lane in
// order of j, and x's map record is written last. Records go to fixed places in the pixel's
// reserved ranges (those of a pair whose gradient vanishes are marked unused). Blocks of eight
// waves share one copy of the env tables in LDS; held to four waves per SIMD (128 VGPRs with some
// spilled: 1.57 -> 1.49 ms on the tori against three waves of 256-lane blocks at 168 VGPRs).
constexpr int kTbThreads = 512;
__global__ __launch_bounds__(kTbThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_trace_bwd(MeshView M, TexView T, EnvView E, ShadeViews V,
                                                        const int32_t* __restrict__ tri_id,
                                                        const float* __restrict__ bary, KParams p, float lambda_ind,
                                                        const float* __restrict__ dI,
                                                        const exm_sec_rec* __restrict__ rec,
                                                        const uint64_t* __restrict__ sec_vis, int64_t p0, int64_t P,
                                                        float* __restrict__ dtex, EnvGradWs eg, TexGradWs tg,
                                                        bool tiled, bool use_lds) {
  extern __shared__ __align__(16) char smem[];
  __shared__ BwdStage stage_all[kTbThreads / 64];
  BwdStage& st = stage_all[threadIdx.x >> 6];
  const EnvTabs tb = load_env_tabs(E, smem, use_lds);
  const int64_t HW = (int64_t)V.H * V.W;
  const int64_t gid = p0 + (int64_t)blockIdx.x * kTbThreads + threadIdx.x;
  const uint32_t lane = __lane_id();
  // every lane stays to the end (the wave shares its pairs); f_d = 0 at every point under
  // EXM_SPECULAR_ONLY (no indirect light)
  bool act = gid < p0 + P && gid < HW * V.n && p.N_b > 0 && !(p.flags & EXM_SPECULAR_ONLY);
  int32_t f = -1;
  uint64_t bits = 0, vm = 0;
  float G[3] = {0.f, 0.f, 0.f};
  if (act) {
    f = tri_id[gid];
    bits = sec_vis[gid];
    G[0] = lambda_ind * dI[3 * gid];
    G[1] = lambda_ind * dI[3 * gid + 1];
    G[2] = lambda_ind * dI[3 * gid + 2];
    act = f >= 0 && (G[0] != 0.0f || G[1] != 0.0f || G[2] != 0.0f);
  }
  const bool y_mat = !(p.flags & EXM_NO_SECONDARY_MATERIAL);
  if (act)
    for (int j = 0; j < p.N_b; ++j)
      if (rec[gid * p.N_b + j].tri >= 0) vm |= 1ull << j;
  // map-gradient records: one for each secondary hit whose maps are queried, then one for x
  const uint32_t n_tex = (act && tiled) ? 1u + (y_mat ? (uint32_t)__popcll(vm) : 0u) : 0u;
  const uint32_t n_rec = act ? (uint32_t)__popcll(bits) : 0u;
  const uint32_t slot = env_grad_reserve(eg.counter, n_rec);
  const uint32_t tslot = tiled ? tex_grad_reserve_n(tg.counter, n_tex) : 0u;
  if (__ballot(act) == 0ull) return;  // the whole wave
  const float invNb = 1.0f / (float)p.N_b;
  const float invNs = p.N_s > 0 ? 1.0f / (float)p.N_s : 0.0f;
  {
    float fdx[3] = {0.f, 0.f, 0.f};
    f3 ns = mk(0, 0, 0);
    float2 b = make_float2(0.f, 0.f);
    uint32_t pix = 0, vid = 0;
    if (act) {
      const int32_t view = (int32_t)(gid / HW);
      pix = (uint32_t)(gid - view * HW);
      vid = (uint32_t)V.view_id[view];
      b = reinterpret_cast<const float2*>(bary)[gid];
      const Surf S = query(M, T, f, b.x, b.y, p.flags);
      const float kdx = (1.0f - S.m) * kInvPi;
      fdx[0] = kdx * S.a[0];
      fdx[1] = kdx * S.a[1];
      fdx[2] = kdx * S.a[2];
      ns = S.ns;
    }
    float* fp = reinterpret_cast<float*>(st.px);
    st.px[kBf * 64 + lane] = (uint32_t)f;
    fp[kBb1 * 64 + lane] = b.x;
    fp[kBb2 * 64 + lane] = b.y;
    st.px[kBpix * 64 + lane] = pix;
    st.px[kBvid * 64 + lane] = vid;
    fp[kBfdx * 64 + lane] = fdx[0];
    fp[(kBfdx + 1) * 64 + lane] = fdx[1];
    fp[(kBfdx + 2) * 64 + lane] = fdx[2];
    fp[kBns * 64 + lane] = ns.x;
    fp[(kBns + 1) * 64 + lane] = ns.y;
    fp[(kBns + 2) * 64 + lane] = ns.z;
    fp[kBG * 64 + lane] = G[0];
    fp[(kBG + 1) * 64 + lane] = G[1];
    fp[(kBG + 2) * 64 + lane] = G[2];
    st.px[kBslot * 64 + lane] = slot;
    st.px[kBtslot * 64 + lane] = tslot;
    st.px[kBbits * 64 + lane] = (uint32_t)bits;
    st.px[(kBbits + 1) * 64 + lane] = (uint32_t)(bits >> 32);
    st.px[kBvm * 64 + lane] = (uint32_t)vm;
    st.px[(kBvm + 1) * 64 + lane] = (uint32_t)(vm >> 32);
  }
  uint32_t total = 0;  // wave-uniform
  for (int j = 0; j < p.N_b; ++j) {
    const uint64_t bj = __ballot((vm >> j) & 1ull);
    if (lane == 0) {
      st.bal[j] = bj;
      st.base[j] = total;
    }
    total += (uint32_t)__popcll(bj);
  }
  __builtin_amdgcn_wave_barrier();
  float gfx[3] = {0.f, 0.f, 0.f};  // d/d f_d(x) of the lane's pixel
  f3 gnx = mk(0, 0, 0);             // d/d n_s(x)
  for (uint32_t c0 = 0; c0 < total; c0 += 64) {
    const uint32_t q = c0 + lane;
    float pg[3] = {0.f, 0.f, 0.f}, pn[3] = {0.f, 0.f, 0.f};
    if (q < total) {
      int j = 0;
      for (int jj = 1; jj < p.N_b; ++jj)
        if (st.base[jj] <= q) j = jj;
      const uint32_t pl = nth_set_bit(st.bal[j], q - st.base[j]);
      const float* fp = reinterpret_cast<const float*>(st.px);
      const int32_t pf = (int32_t)st.px[kBf * 64 + pl];
      const float b1 = fp[kBb1 * 64 + pl], b2 = fp[kBb2 * 64 + pl];
      const uint32_t ppix = st.px[kBpix * 64 + pl], pvid = st.px[kBvid * 64 + pl];
      const float fdx[3] = {fp[kBfdx * 64 + pl], fp[(kBfdx + 1) * 64 + pl], fp[(kBfdx + 2) * 64 + pl]};
      const f3 xns = mk(fp[kBns * 64 + pl], fp[(kBns + 1) * 64 + pl], fp[(kBns + 2) * 64 + pl]);
      const float Gp[3] = {fp[kBG * 64 + pl], fp[(kBG + 1) * 64 + pl], fp[(kBG + 2) * 64 + pl]};
      const uint64_t pbits = (uint64_t)st.px[kBbits * 64 + pl] | ((uint64_t)st.px[(kBbits + 1) * 64 + pl] << 32);
      const uint64_t pvm = (uint64_t)st.px[kBvm * 64 + pl] | ((uint64_t)st.px[(kBvm + 1) * 64 + pl] << 32);
      // this pair's records: its light samples' env records and (with maps at y) y's map record
      uint32_t eslot = st.px[kBslot * 64 + pl] + (uint32_t)__popcll(pbits & ((1ull << (j * p.N_s)) - 1ull));
      const uint32_t yslot = st.px[kBtslot * 64 + pl] + (uint32_t)__popcll(pvm & ((1ull << j) - 1ull));
      const int64_t pgid = gid - (int64_t)lane + (int64_t)pl;
      const exm_sec_rec r = rec[pgid * p.N_b + j];
      const Draw d = philox_draw(p.key.k0, p.key.k1, ppix, pvid, (uint32_t)j, 1u);
      const SecRay sr = secondary_ray(M, pf, b1, b2, d.u2, d.u3);
      const f3 w = sr.df;
      const float pb = sr.pb;
      const float cxr = dot(xns, w);
      const float cx = fmaxf(cxr, 0.0f);
      const Surf Y = query(M, T, r.tri, r.b1, r.b2, p.flags, y_mat);
      const float kdy = (1.0f - Y.m) * kInvPi;
      const float fdy[3] = {kdy * Y.a[0], kdy * Y.a[1], kdy * Y.a[2]};
      // L_sec(y) without the f_d(y) factor, per channel: (1/N_s) sum E c / pdf. The first kCacheS
      // samples are kept for the second pass below, which would otherwise draw them again.
      float Es[3] = {0.f, 0.f, 0.f};
      EnvSample cache[kCacheS];
#pragma unroll
      for (int s2 = 0; s2 < kCacheS; ++s2) {
        if (s2 >= p.N_s || !((pbits >> (j * p.N_s + s2)) & 1ull)) continue;
        const Draw ds = philox_draw(p.key.k0, p.key.k1, ppix, pvid, (uint32_t)s2, 2u + (uint32_t)j);
        cache[s2] = env_sample(E, tb, ds);
        const float c = dot(Y.ns, cache[s2].dir);
        const float* e = cache[s2].E;
        const float wgt = c * cache[s2].inv_pdf * invNs;
        Es[0] += e[0] * wgt;
        Es[1] += e[1] * wgt;
        Es[2] += e[2] * wgt;
      }
      for (int s2 = kCacheS; s2 < p.N_s; ++s2) {
        if (!((pbits >> (j * p.N_s + s2)) & 1ull)) continue;
        const Draw ds = philox_draw(p.key.k0, p.key.k1, ppix, pvid, (uint32_t)s2, 2u + (uint32_t)j);
        const EnvSample es = env_sample(E, tb, ds);
        const float c = dot(Y.ns, es.dir);
        const float* e = es.E;
        const float wgt = c * es.inv_pdf * invNs;
        Es[0] += e[0] * wgt;
        Es[1] += e[1] * wgt;
        Es[2] += e[2] * wgt;
      }
      const float fac = invNb * cx / pb;  // weight of f_d(x) L_sec(y) in L_ind
      float H[3];                          // dLoss/dL_sec(y)
      for (int c = 0; c < 3; ++c) {
        const float Lsec = fdy[c] * Es[c];
        pg[c] = Gp[c] * Lsec * fac;
        H[c] = Gp[c] * fdx[c] * fac;
      }
      if (cxr > 0.0f) {
        const float sc = invNb / pb * (Gp[0] * fdx[0] * fdy[0] * Es[0] + Gp[1] * fdx[1] * fdy[1] * Es[1] +
                                       Gp[2] * fdx[2] * fdy[2] * Es[2]);
        pn[0] = sc * w.x;
        pn[1] = sc * w.y;
        pn[2] = sc * w.z;
      }
      if (H[0] == 0.0f && H[1] == 0.0f && H[2] == 0.0f) {  // nothing reaches y: its records stay unused
        for (int s2 = 0; s2 < p.N_s; ++s2)
          if ((pbits >> (j * p.N_s + s2)) & 1ull) env_grad_put(eg, eslot++, kNoTexel, 0.f, 0.f, 0.f);
        if (tiled && y_mat) tex_grad_skip(tg, yslot);
      } else {
        // secondary point: env texels, f_d(y) and n_s(y)
        float gfy[3] = {H[0] * Es[0], H[1] * Es[1], H[2] * Es[2]};
        f3 gny = mk(0, 0, 0);
        for (int s2 = 0; s2 < p.N_s; ++s2) {
          if (!((pbits >> (j * p.N_s + s2)) & 1ull)) continue;
          EnvSample es;
          if (s2 < kCacheS) {
#pragma unroll
            for (int qq = 0; qq < kCacheS; ++qq)
              if (qq == s2) es = cache[qq];
          } else {
            const Draw ds = philox_draw(p.key.k0, p.key.k1, ppix, pvid, (uint32_t)s2, 2u + (uint32_t)j);
            es = env_sample(E, tb, ds);
          }
          const float c = dot(Y.ns, es.dir);
          const float* e = es.E;
          const float ip = es.inv_pdf * invNs;
          env_grad_put(eg, eslot++, (uint32_t)es.texel, H[0] * fdy[0] * c * ip, H[1] * fdy[1] * c * ip,
                       H[2] * fdy[2] * c * ip);
          const float sn = (H[0] * fdy[0] * e[0] + H[1] * fdy[1] * e[1] + H[2] * fdy[2] * e[2]) * ip;
          gny = gny + sn * es.dir;
        }
        if (y_mat) {  // nothing at y depends on the maps otherwise
          float gay[3], gmy = 0.0f, gqy[3];
          for (int c = 0; c < 3; ++c) {
            gay[c] = gfy[c] * kdy;
            gmy -= gfy[c] * Y.a[c] * kInvPi;
          }
          if (p.flags & EXM_METALLIC_OFF) gmy = 0.0f;
          nmap_adjoint(Y, gny, gqy);
          scatter7(Y, gay, gmy, gqy, dtex, tg, tiled, yslot);
        }
      }
    }
    st.pair[0 * 64 + lane] = pg[0];
    st.pair[1 * 64 + lane] = pg[1];
    st.pair[2 * 64 + lane] = pg[2];
    st.pair[3 * 64 + lane] = pn[0];
    st.pair[4 * 64 + lane] = pn[1];
    st.pair[5 * 64 + lane] = pn[2];
    __builtin_amdgcn_wave_barrier();
    // the pixel's pairs in this chunk, in order of j
    if (act) {
      for (int j = 0; j < p.N_b; ++j) {
        if (!((vm >> j) & 1ull)) continue;
        const uint32_t qj = st.base[j] + (uint32_t)__popcll(st.bal[j] & ((1ull << lane) - 1ull));
        if (qj < c0 || qj >= c0 + 64u) continue;
        const uint32_t i = qj - c0;
        for (int c = 0; c < 3; ++c) gfx[c] += st.pair[c * 64 + i];
        gnx = gnx + mk(st.pair[3 * 64 + i], st.pair[4 * 64 + i], st.pair[5 * 64 + i]);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (!act) return;
  // x: queried again (cheaper than keeping its surface live through the pairs)
  const float2 b = reinterpret_cast<const float2*>(bary)[gid];
  const Surf S = query(M, T, f, b.x, b.y, p.flags);
  const float kdx = (1.0f - S.m) * kInvPi;
  float gax[3], gmx = 0.0f, gqx[3];
  for (int c = 0; c < 3; ++c) {
    gax[c] = gfx[c] * kdx;
    gmx -= gfx[c] * S.a[c] * kInvPi;
  }
  if (p.flags & EXM_METALLIC_OFF) gmx = 0.0f;
  nmap_adjoint(S, gnx, gqx);
  scatter7(S, gax, gmx, gqx, dtex, tg, tiled, tslot + n_tex - 1u);
}

KParams kparams(const exm_params* p) {
  KParams k;
  k.N_b = p->N_b;
  k.N_s = p->N_s;
  k.flags = p->flags;
  k.tmin = p->tmin;
  k.key = make_key(p->seed, p->iteration);
  return k;
}

}  // namespace

hipError_t launch_trace_indirect(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat, const exm_env* env,
                                 const ShadeViews& v, const int32_t* tri_id, const float* bary, const exm_params* p,
                                 float* L_ind, exm_sec_rec* sec_rec, uint64_t* sec_vis, void* ws_ptr, size_t ws_bytes,
                                 unsigned long long* counters, hipStream_t s) {
  const int64_t n = (int64_t)v.n * v.H * v.W;
  const int64_t P = indirect_chunk(ws_bytes, p->N_b, p->N_s, n);
  if (P <= 0) return hipErrorInvalidValue;  // the ABI layer checks the size first
  const KParams kp = kparams(p);
  const TexView tv{mat->Ht, mat->Wt, mat->tex};
  const IndirectWs ws = indirect_ws(ws_ptr, P, p->N_b, p->N_s);
  const bool vis_rays = !(p->flags & EXM_NO_VIS) && p->N_s > 0;
  const size_t lds = env_tabs_bytes(env->He, env->We);
  const bool use_lds = lds <= kEnvTabsMaxBytes;
  for (int64_t p0 = 0; p0 < n; p0 += P) {
    const int64_t Pc = std::min<int64_t>(P, ((n - p0) + 63) / 64 * 64);
    const unsigned nb = (unsigned)((Pc + kThreads - 1) / kThreads);
    if (p->N_b > 0) {
      {
        EXM_TIMED("ind_gen1", s);
        k_ind_gen1<<<nb, kThreads, 0, s>>>(mesh_view(m), v, tri_id, bary, kp, p0, Pc, ws);
      }
      const RayBatch rb1{ws.sec_rays, ws.sec_orgs, ws.sec_count, (int32_t)(Pc / 64), 64 * (int64_t)p->N_b, p->tmin,
                         ws.counter};
      hipError_t e = launch_trace_closest(bvh, rb1, ws.sec_hits, counters, s);
      if (e != hipSuccess) return e;
    }
    {
      EXM_TIMED("ind_gen2", s);
      k_ind_gen2<<<(unsigned)((Pc + kIg2Threads - 1) / kIg2Threads), kIg2Threads, use_lds ? lds : 0, s>>>(mesh_view(m), tv, env_view(env), v, tri_id, bary, kp, p0,
                                                         Pc, ws, sec_rec, use_lds);
    }
    if (vis_rays && p->N_b > 0) {
      const RayBatch rb2{ws.sh_rays,  ws.sh_orgs, ws.sh_count, (int32_t)(Pc / 64), 64 * (int64_t)p->N_b * p->N_s,
                         p->tmin, ws.counter};
      hipError_t e = launch_trace_any(bvh, rb2, ws.sh_hit, counters ? counters + 3 : nullptr, s);
      if (e != hipSuccess) return e;
    }
    {
      EXM_TIMED("ind_finalize", s);
      k_ind_finalize<<<nb, kThreads, 0, s>>>(v, kp, p0, Pc, ws, L_ind, sec_vis);
    }
  }
  return hipGetLastError();
}

size_t trace_indirect_ws_bytes(int64_t n_pix, int32_t N_b, int32_t N_s) {
  return indirect_ws_bytes((n_pix + 63) / 64 * 64, N_b, N_s);
}
size_t trace_indirect_ws_min(int32_t N_b, int32_t N_s) { return indirect_ws_bytes(64, N_b, N_s); }

hipError_t launch_trace_bwd(const exm_mesh* m, const exm_material* mat, const exm_env* env, const ShadeViews& v,
                            const int32_t* tri_id, const float* bary, const exm_params* p, float lambda_ind,
                            const float* dI, const exm_sec_rec* sec_rec, const uint64_t* sec_vis, float* dtex,
                            double* denv, void* ws, size_t ws_bytes, hipStream_t s) {
  const int64_t n = (int64_t)v.n * v.H * v.W;
  const int64_t per_px = (int64_t)std::max(p->N_b, 0) * std::max(p->N_s, 0);
  const int64_t tex_px = 1 + (int64_t)std::max(p->N_b, 0);
  const int64_t P = adjoint_chunk(ws_bytes, per_px, tex_px, env->He, env->We, n);
  if (P <= 0) return hipErrorInvalidValue;  // the ABI layer checks the size first
  const size_t lds = env_tabs_bytes(env->He, env->We);
  const bool use_lds = lds <= kEnvTabsMaxBytes;
  const KParams kp = kparams(p);
  const bool tiled = tex_grad_tiled(mat->Ht, mat->Wt) && !(p->flags & EXM_MAP_GRAD_ATOMIC);
  for (int64_t p0 = 0; p0 < n; p0 += P) {
    const int64_t Pc = std::min<int64_t>(P, ((n - p0) + 63) / 64 * 64);
    const EnvGradWs eg = env_grad_ws(ws, Pc * per_px, env->He, env->We);
    const TexGradWs tg = tex_grad_ws(static_cast<char*>(ws) + env_grad_ws_bytes(Pc * per_px, env->He, env->We),
                                     Pc * tex_px, mat->Ht, mat->Wt);
    hipError_t e = launch_env_grad_clear(eg, s);
    if (e != hipSuccess) return e;
    if (tiled) {
      e = launch_tex_grad_clear(tg, s);
      if (e != hipSuccess) return e;
    }
    {
      EXM_TIMED("trace_bwd", s);
      k_trace_bwd<<<(unsigned)((Pc + kTbThreads - 1) / kTbThreads), kTbThreads, use_lds ? lds : 0, s>>>(
          mesh_view(m), TexView{mat->Ht, mat->Wt, mat->tex}, env_view(env), v, tri_id, bary, kp, lambda_ind, dI,
          sec_rec, sec_vis, p0, Pc, dtex, eg, tg, tiled, use_lds);
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

size_t trace_bwd_ws_bytes(int64_t n_pix, int32_t N_b, int32_t N_s, int32_t He, int32_t We) {
  const int64_t np = (n_pix + 63) / 64 * 64;
  return env_grad_ws_bytes(np * std::max(N_b, 0) * std::max(N_s, 0), He, We) +
         tex_grad_ws_bytes(np * (1 + (int64_t)std::max(N_b, 0)));
}
size_t trace_bwd_ws_min(int32_t N_b, int32_t N_s, int32_t He, int32_t We) {
  return env_grad_ws_bytes(64 * (int64_t)std::max(N_b, 0) * std::max(N_s, 0), He, We) +
         tex_grad_ws_bytes(64 * (1 + (int64_t)std::max(N_b, 0)));
}

}  // namespace exm
