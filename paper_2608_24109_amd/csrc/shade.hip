// Direct illumination (Direct Illumination, Eq. 12-17) and its adjoint.
//
// Forward, per covered pixel: attribute query at the visible point (Eq. 10-11), then N_d
// env samples drawn from the importance-sampling tables; a sample with n_s . w > 0 traces an
// any-hit shadow ray and, if unoccluded, adds E f_r (n_s . w) / pdf (Eq. 13-16 for f_r).
// The visibility bits of all samples are stored so the adjoint never traces a ray.
//
// Adjoint, per covered pixel with upstream g = dLoss/dL_dir: the same samples again (same RNG
// counters), skipping those whose bit is clear; accumulates d/d(a, r, m, n_s) over samples,
// maps d/dn_s through the normalisation to d/dq of the normal map, and scatters the eight
// channel gradients to the four bilinear taps; dLoss/dE of each sample goes to its env texel.
// The pdf and every discrete choice are held fixed.
#include <hip/hip_runtime.h>

#include "exm_device.h"

namespace exm {
namespace {

constexpr int kThreads = 256;

struct KParams {
  int32_t N_d;
  uint32_t flags;
  float f_diel, eps, tmin;
  RngKey key;
};

__device__ __forceinline__ void brdf_eval(const Surf& S, f3 wi, f3 wo, float ci, const KParams& p, float fr[3]) {
  const float kd = (p.flags & EXM_SPECULAR_ONLY) ? 0.0f : (1.0f - S.m) * kInvPi;
  fr[0] = kd * S.a[0];
  fr[1] = kd * S.a[1];
  fr[2] = kd * S.a[2];
  if (p.flags & EXM_DIFFUSE_ONLY) return;
  const Spec s = spec_terms(S.ns, wi, wo, ci, S.r, p.eps);
  if (!s.on) return;
  const float k = s.D * s.G1i * s.G1o / s.den;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float F0 = (1.0f - S.m) * p.f_diel + S.m * S.a[c];
    fr[c] += k * (F0 + (1.0f - F0) * s.x5);
  }
}

// COUNT: measurement variant that also accumulates [shadow rays, node visits, triangle tests,
// samples drawn] into counters
template <bool COUNT>
__global__ __launch_bounds__(kThreads) void k_shade_fwd(MeshView M, TexView T, EnvView E, BvhView B, ShadeViews V,
                                                        const int32_t* __restrict__ tri_id,
                                                        const float* __restrict__ bary, KParams p,
                                                        float* __restrict__ L_dir, uint64_t* __restrict__ vis,
                                                        unsigned long long* __restrict__ counters) {
  __shared__ int32_t stack[kStack * kThreads];
  const int64_t HW = (int64_t)V.H * V.W;
  const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (gid >= HW * V.n) return;
  const int32_t view = (int32_t)(gid / HW);
  const uint32_t pix = (uint32_t)(gid - view * HW);
  const int32_t f = tri_id[gid];
  float L[3] = {0.f, 0.f, 0.f};
  uint64_t bits = 0;
  TraceCount tc;
  uint32_t n_rays = 0;
  if (f >= 0) {
    const float2 b = reinterpret_cast<const float2*>(bary)[gid];
    const Surf S = query(M, T, f, b.x, b.y, p.flags);
    const f3 wo = normalize(mk(V.eye[view][0], V.eye[view][1], V.eye[view][2]) - S.x);
    const uint32_t vid = (uint32_t)V.view_id[view];
    for (int k = 0; k < p.N_d; ++k) {
      const Draw d = philox_draw(p.key.k0, p.key.k1, pix, vid, (uint32_t)k, 0u);
      const EnvSample es = env_sample(E, d);
      const float c = dot(S.ns, es.dir);
      if (!(c > 0.0f)) continue;
      if (!(p.flags & EXM_NO_VIS)) {
        const Ray r = make_ray(S.x, es.dir);
        if (COUNT) ++n_rays;
        const HitRec h = trace<true, COUNT>(B, r, p.tmin, f, stack + threadIdx.x, kThreads, &tc);
        if (h.id >= 0) continue;
      }
      bits |= 1ull << k;
      float fr[3];
      brdf_eval(S, es.dir, wo, c, p, fr);
      const float* e = E.env + 3 * (int64_t)es.texel;
      const float wgt = c * es.inv_pdf;
      L[0] += e[0] * fr[0] * wgt;
      L[1] += e[1] * fr[1] * wgt;
      L[2] += e[2] * fr[2] * wgt;
    }
    const float inv = p.N_d > 0 ? 1.0f / (float)p.N_d : 0.0f;
    L[0] *= inv;
    L[1] *= inv;
    L[2] *= inv;
  }
  L_dir[3 * gid] = L[0];
  L_dir[3 * gid + 1] = L[1];
  L_dir[3 * gid + 2] = L[2];
  vis[gid] = bits;
  if (COUNT && f >= 0) {
    atomicAdd(counters + 0, (unsigned long long)n_rays);
    atomicAdd(counters + 1, (unsigned long long)tc.nodes);
    atomicAdd(counters + 2, (unsigned long long)tc.tris);
    atomicAdd(counters + 3, (unsigned long long)p.N_d);
  }
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
      const float k = DG / s.den;
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
      const float dD_dd = -2.0f * s.D / s.d;
      const float dG1i_dc = 2.0f * s.alpha2 / (s.si * (ci + s.si) * (ci + s.si));
      const float dG1o_dc = 2.0f * s.alpha2 / (s.so * (s.co + s.so) * (s.co + s.so));
      const float G = s.G1i * s.G1o;
      // alpha^2 path
      if (!s.alpha_clamped) {
        const float dD_da2 = s.D / s.alpha2 - 2.0f * s.D * s.chh * s.chh / s.d;
        const float dG1i_da2 = -ci * (1.0f - ci * ci) / (s.si * (ci + s.si) * (ci + s.si));
        const float dG1o_da2 = -s.co * (1.0f - s.co * s.co) / (s.so * (s.co + s.so) * (s.co + s.so));
        const float dDG_da2 = dD_da2 * G + s.D * (dG1i_da2 * s.G1o + s.G1i * dG1o_da2);
        const float r3 = S.r * S.r * S.r;
        g.r += ci * sumWF / s.den * dDG_da2 * 4.0f * r3;
      }
      // shading-normal path: D through n.h and |n x h|^2, G through n.wi and n.wo, 1/den
      const f3 gd = 2.0f * (S.ns - s.chh * s.h) + (2.0f * s.alpha2 * s.chh) * s.h;  // dd/dn
      const f3 gD = dD_dd * gd;
      const f3 gG = (dG1i_dc * s.G1o) * wi + (s.G1i * dG1o_dc) * wo;
      const f3 gden = 4.0f * (s.co * wi + ci * wo);
      g.n = g.n + (ci * sumWF / s.den) * (G * gD + s.D * gG) - (ci * sumWfs / s.den) * gden;
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

__global__ __launch_bounds__(kThreads) void k_shade_bwd(MeshView M, TexView T, EnvView E, ShadeViews V,
                                                        const int32_t* __restrict__ tri_id,
                                                        const float* __restrict__ bary, KParams p,
                                                        const float* __restrict__ dI, const uint64_t* __restrict__ vis,
                                                        float* __restrict__ dtex, double* __restrict__ denv) {
  const int64_t HW = (int64_t)V.H * V.W;
  const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (gid >= HW * V.n) return;
  const int32_t f = tri_id[gid];
  uint64_t bits = vis[gid];
  if (f < 0 || bits == 0) return;
  const float g[3] = {dI[3 * gid], dI[3 * gid + 1], dI[3 * gid + 2]};
  if (g[0] == 0.0f && g[1] == 0.0f && g[2] == 0.0f) return;
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
  while (bits) {
    const int k = __ffsll((long long)bits) - 1;
    bits &= bits - 1;
    const Draw d = philox_draw(p.key.k0, p.key.k1, pix, vid, (uint32_t)k, 0u);
    const EnvSample es = env_sample(E, d);
    const float c = dot(S.ns, es.dir);
    const float* e = E.env + 3 * (int64_t)es.texel;
    const float s = invN * es.inv_pdf;
    const float W[3] = {g[0] * e[0] * s, g[1] * e[1] * s, g[2] * e[2] * s};
    float fr[3];
    brdf_adjoint(S, es.dir, wo, c, p, W, fr, G);
    double* de = denv + 3 * (int64_t)es.texel;
    const float cs = c * s;
    unsafeAtomicAdd(de, (double)(g[0] * fr[0] * cs));
    unsafeAtomicAdd(de + 1, (double)(g[1] * fr[1] * cs));
    unsafeAtomicAdd(de + 2, (double)(g[2] * fr[2] * cs));
  }
  float gq[3];
  normal_map_adjoint(S, G.n, gq);
  const float g8[8] = {G.a[0], G.a[1], G.a[2], G.r, (p.flags & EXM_METALLIC_OFF) ? 0.0f : G.m, gq[0], gq[1], gq[2]};
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
EnvView env_view(const exm_env* e) { return EnvView{e->He, e->We, e->env, e->cdf_row, e->cdf_col, e->pdf}; }
BvhView bvh_view(const exm_bvh* b) { return BvhView{b->nodes, b->tris, b->root_is_leaf}; }

hipError_t launch_shade_fwd(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat, const exm_env* env,
                            const ShadeViews& v, const int32_t* tri_id, const float* bary, const exm_params* p,
                            float* L_dir, uint64_t* vis, unsigned long long* counters, hipStream_t s) {
  const int64_t n = (int64_t)v.n * v.H * v.W;
  const unsigned nb = (unsigned)((n + kThreads - 1) / kThreads);
  const TexView tv{mat->Ht, mat->Wt, mat->tex};
  if (counters)
    k_shade_fwd<true><<<nb, kThreads, 0, s>>>(mesh_view(m), tv, env_view(env), bvh_view(bvh), v, tri_id, bary,
                                              kparams(p), L_dir, vis, counters);
  else
    k_shade_fwd<false><<<nb, kThreads, 0, s>>>(mesh_view(m), tv, env_view(env), bvh_view(bvh), v, tri_id, bary,
                                               kparams(p), L_dir, vis, nullptr);
  return hipGetLastError();
}

hipError_t launch_shade_bwd(const exm_mesh* m, const exm_material* mat, const exm_env* env, const ShadeViews& v,
                            const int32_t* tri_id, const float* bary, const exm_params* p, const float* dI,
                            const uint64_t* vis, float* dtex, double* denv, hipStream_t s) {
  const int64_t n = (int64_t)v.n * v.H * v.W;
  k_shade_bwd<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(
      mesh_view(m), TexView{mat->Ht, mat->Wt, mat->tex}, env_view(env), v, tri_id, bary, kparams(p), dI, vis, dtex,
      denv);
  return hipGetLastError();
}

}  // namespace exm
