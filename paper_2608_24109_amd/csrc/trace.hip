// One-bounce diffuse indirect illumination (One-Bounce Indirect Illumination, Eq. 18-19)
// and its adjoint.
//
// Forward, per covered pixel x: N_b directions w_j cosine-weighted about n_g(x) (Malley's
// method in the Duff et al. orthonormal basis; p_b = max(n_g . w, 0) / pi); closest hit from
// x (t >= t_min, the origin triangle skipped); the hit counts only if it is front facing.
// At a valid hit y: the same attribute query as for primary points, then N_s env samples with
// shadow rays give the diffuse radiance L_sec(y) (Eq. 18, no specular term). Eq. 19 sums
// 1_hit f_d(x) L_sec(y_j) max(n_s(x) . w_j, 0) / p_b over j and divides by N_b.
// The hit records and the light-sample visibility bits are stored for the adjoint.
//
// Adjoint, for upstream G = lambda_ind dLoss/dI: gradients to a, m, n_s at x (through f_d(x)
// and the cosine) and at each y_j (through f_d(y) and n_s(y)), and to E at the light samples.
#include <hip/hip_runtime.h>

#include "exm_device.h"

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

// COUNT: measurement variant that also accumulates [secondary rays, their node visits, their
// triangle tests, light shadow rays, their node visits, their triangle tests] into counters
template <bool COUNT>
__global__ __launch_bounds__(kThreads) void k_trace_indirect(MeshView M, TexView T, EnvView E, BvhView B,
                                                             ShadeViews V, const int32_t* __restrict__ tri_id,
                                                             const float* __restrict__ bary, KParams p,
                                                             float* __restrict__ L_ind, exm_sec_rec* __restrict__ rec,
                                                             uint64_t* __restrict__ sec_vis,
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
  exm_sec_rec* myrec = rec + gid * p.N_b;
  TraceCount tc_sec, tc_sh;
  uint32_t n_sh = 0;
  if (f >= 0) {
    const float2 b = reinterpret_cast<const float2*>(bary)[gid];
    const Surf S = query(M, T, f, b.x, b.y, p.flags);
    const uint32_t vid = (uint32_t)V.view_id[view];
    const bool diff = !(p.flags & EXM_SPECULAR_ONLY);
    const float kdx = diff ? (1.0f - S.m) * kInvPi : 0.0f;
    const float invNs = p.N_s > 0 ? 1.0f / (float)p.N_s : 0.0f;
    for (int j = 0; j < p.N_b; ++j) {
      exm_sec_rec r{-1, 0.f, 0.f};
      const Draw d = philox_draw(p.key.k0, p.key.k1, pix, vid, (uint32_t)j, 1u);
      const SecRay sr = secondary_ray(M, f, b.x, b.y, d.u2, d.u3);
      const f3 w = sr.df;
      const float pb = sr.pb;
      HitRec h = trace<false, COUNT>(B, make_ray(sr.of, w), p.tmin, f, stack + threadIdx.x, kThreads, &tc_sec);
      if (h.id >= 0 && front_facing(M, h.id, w)) {
        refine_hit(M, h.id, sr, &h.b1, &h.b2);
        r = exm_sec_rec{h.id, h.b1, h.b2};
        const Surf Y = query(M, T, h.id, h.b1, h.b2, p.flags);
        const float kdy = diff ? (1.0f - Y.m) * kInvPi : 0.0f;
        float Ls[3] = {0.f, 0.f, 0.f};
        for (int s = 0; s < p.N_s; ++s) {
          const Draw ds = philox_draw(p.key.k0, p.key.k1, pix, vid, (uint32_t)s, 2u + (uint32_t)j);
          const EnvSample es = env_sample(E, ds);
          const float c = dot(Y.ns, es.dir);
          if (!(c > 0.0f)) continue;
          if (!(p.flags & EXM_NO_VIS)) {
            if (COUNT) ++n_sh;
            const HitRec hs =
                trace<true, COUNT>(B, make_ray(Y.x, es.dir), p.tmin, h.id, stack + threadIdx.x, kThreads, &tc_sh);
            if (hs.id >= 0) continue;
          }
          bits |= 1ull << (j * p.N_s + s);
          const float* e = E.env + 3 * (int64_t)es.texel;
          const float wgt = c * es.inv_pdf;
          Ls[0] += e[0] * wgt;
          Ls[1] += e[1] * wgt;
          Ls[2] += e[2] * wgt;
        }
        const float cx = fmaxf(dot(S.ns, w), 0.0f);
        const float fac = cx / pb * invNs;
        L[0] += kdx * S.a[0] * (kdy * Y.a[0] * Ls[0]) * fac;
        L[1] += kdx * S.a[1] * (kdy * Y.a[1] * Ls[1]) * fac;
        L[2] += kdx * S.a[2] * (kdy * Y.a[2] * Ls[2]) * fac;
      }
      myrec[j] = r;
    }
    const float inv = p.N_b > 0 ? 1.0f / (float)p.N_b : 0.0f;
    L[0] *= inv;
    L[1] *= inv;
    L[2] *= inv;
  } else {
    for (int j = 0; j < p.N_b; ++j) myrec[j] = exm_sec_rec{-1, 0.f, 0.f};
  }
  L_ind[3 * gid] = L[0];
  L_ind[3 * gid + 1] = L[1];
  L_ind[3 * gid + 2] = L[2];
  sec_vis[gid] = bits;
  if (COUNT && f >= 0) {
    atomicAdd(counters + 0, (unsigned long long)p.N_b);
    atomicAdd(counters + 1, (unsigned long long)tc_sec.nodes);
    atomicAdd(counters + 2, (unsigned long long)tc_sec.tris);
    atomicAdd(counters + 3, (unsigned long long)n_sh);
    atomicAdd(counters + 4, (unsigned long long)tc_sh.nodes);
    atomicAdd(counters + 5, (unsigned long long)tc_sh.tris);
  }
}

__device__ __forceinline__ void scatter7(const Surf& S, const float ga[3], float gm, const float gq[3],
                                         float* __restrict__ dtex) {
  const float g8[8] = {ga[0], ga[1], ga[2], 0.0f, gm, gq[0], gq[1], gq[2]};
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

__global__ __launch_bounds__(kThreads) void k_trace_bwd(MeshView M, TexView T, EnvView E, ShadeViews V,
                                                        const int32_t* __restrict__ tri_id,
                                                        const float* __restrict__ bary, KParams p, float lambda_ind,
                                                        const float* __restrict__ dI,
                                                        const exm_sec_rec* __restrict__ rec,
                                                        const uint64_t* __restrict__ sec_vis,
                                                        float* __restrict__ dtex, double* __restrict__ denv) {
  const int64_t HW = (int64_t)V.H * V.W;
  const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (gid >= HW * V.n) return;
  const int32_t f = tri_id[gid];
  if (f < 0 || p.N_b == 0) return;
  if (p.flags & EXM_SPECULAR_ONLY) return;  // f_d = 0 at every point: no indirect light
  const float G[3] = {lambda_ind * dI[3 * gid], lambda_ind * dI[3 * gid + 1], lambda_ind * dI[3 * gid + 2]};
  if (G[0] == 0.0f && G[1] == 0.0f && G[2] == 0.0f) return;
  const int32_t view = (int32_t)(gid / HW);
  const uint32_t pix = (uint32_t)(gid - view * HW);
  const float2 b = reinterpret_cast<const float2*>(bary)[gid];
  const Surf S = query(M, T, f, b.x, b.y, p.flags);
  const uint32_t vid = (uint32_t)V.view_id[view];
  const uint64_t bits = sec_vis[gid];
  const float invNb = 1.0f / (float)p.N_b;
  const float invNs = p.N_s > 0 ? 1.0f / (float)p.N_s : 0.0f;
  const float kdx = (1.0f - S.m) * kInvPi;
  float gfx[3] = {0.f, 0.f, 0.f};  // d/d f_d(x)
  f3 gnx = mk(0, 0, 0);             // d/d n_s(x)
  for (int j = 0; j < p.N_b; ++j) {
    const exm_sec_rec r = rec[gid * p.N_b + j];
    if (r.tri < 0) continue;
    const Draw d = philox_draw(p.key.k0, p.key.k1, pix, vid, (uint32_t)j, 1u);
    const SecRay sr = secondary_ray(M, f, b.x, b.y, d.u2, d.u3);
    const f3 w = sr.df;
    const float pb = sr.pb;
    const float cxr = dot(S.ns, w);
    const float cx = fmaxf(cxr, 0.0f);
    const Surf Y = query(M, T, r.tri, r.b1, r.b2, p.flags);
    const float kdy = (1.0f - Y.m) * kInvPi;
    const float fdy[3] = {kdy * Y.a[0], kdy * Y.a[1], kdy * Y.a[2]};
    const float fdx[3] = {kdx * S.a[0], kdx * S.a[1], kdx * S.a[2]};
    // L_sec(y) without the f_d(y) factor, per channel: (1/N_s) sum E c / pdf
    float Es[3] = {0.f, 0.f, 0.f};
    for (int s = 0; s < p.N_s; ++s) {
      if (!((bits >> (j * p.N_s + s)) & 1ull)) continue;
      const Draw ds = philox_draw(p.key.k0, p.key.k1, pix, vid, (uint32_t)s, 2u + (uint32_t)j);
      const EnvSample es = env_sample(E, ds);
      const float c = dot(Y.ns, es.dir);
      const float* e = E.env + 3 * (int64_t)es.texel;
      const float wgt = c * es.inv_pdf * invNs;
      Es[0] += e[0] * wgt;
      Es[1] += e[1] * wgt;
      Es[2] += e[2] * wgt;
    }
    const float fac = invNb * cx / pb;  // weight of f_d(x) L_sec(y) in L_ind
    float H[3];                          // dLoss/dL_sec(y)
    for (int c = 0; c < 3; ++c) {
      const float Lsec = fdy[c] * Es[c];
      gfx[c] += G[c] * Lsec * fac;
      H[c] = G[c] * fdx[c] * fac;
    }
    if (cxr > 0.0f) {
      const float sc = invNb / pb * (G[0] * fdx[0] * fdy[0] * Es[0] + G[1] * fdx[1] * fdy[1] * Es[1] +
                                     G[2] * fdx[2] * fdy[2] * Es[2]);
      gnx = gnx + sc * w;
    }
    if (H[0] == 0.0f && H[1] == 0.0f && H[2] == 0.0f) continue;
    // secondary point: env texels, f_d(y) and n_s(y)
    float gfy[3] = {H[0] * Es[0], H[1] * Es[1], H[2] * Es[2]};
    f3 gny = mk(0, 0, 0);
    for (int s = 0; s < p.N_s; ++s) {
      if (!((bits >> (j * p.N_s + s)) & 1ull)) continue;
      const Draw ds = philox_draw(p.key.k0, p.key.k1, pix, vid, (uint32_t)s, 2u + (uint32_t)j);
      const EnvSample es = env_sample(E, ds);
      const float c = dot(Y.ns, es.dir);
      const float* e = E.env + 3 * (int64_t)es.texel;
      const float ip = es.inv_pdf * invNs;
      double* de = denv + 3 * (int64_t)es.texel;
      unsafeAtomicAdd(de, (double)(H[0] * fdy[0] * c * ip));
      unsafeAtomicAdd(de + 1, (double)(H[1] * fdy[1] * c * ip));
      unsafeAtomicAdd(de + 2, (double)(H[2] * fdy[2] * c * ip));
      const float sn = (H[0] * fdy[0] * e[0] + H[1] * fdy[1] * e[1] + H[2] * fdy[2] * e[2]) * ip;
      gny = gny + sn * es.dir;
    }
    float gay[3], gmy = 0.0f, gqy[3];
    for (int c = 0; c < 3; ++c) {
      gay[c] = gfy[c] * kdy;
      gmy -= gfy[c] * Y.a[c] * kInvPi;
    }
    if (p.flags & EXM_METALLIC_OFF) gmy = 0.0f;
    nmap_adjoint(Y, gny, gqy);
    scatter7(Y, gay, gmy, gqy, dtex);
  }
  float gax[3], gmx = 0.0f, gqx[3];
  for (int c = 0; c < 3; ++c) {
    gax[c] = gfx[c] * kdx;
    gmx -= gfx[c] * S.a[c] * kInvPi;
  }
  if (p.flags & EXM_METALLIC_OFF) gmx = 0.0f;
  nmap_adjoint(S, gnx, gqx);
  scatter7(S, gax, gmx, gqx, dtex);
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
                                 float* L_ind, exm_sec_rec* sec_rec, uint64_t* sec_vis, unsigned long long* counters,
                                 hipStream_t s) {
  const int64_t n = (int64_t)v.n * v.H * v.W;
  const unsigned nb = (unsigned)((n + kThreads - 1) / kThreads);
  const TexView tv{mat->Ht, mat->Wt, mat->tex};
  if (counters)
    k_trace_indirect<true><<<nb, kThreads, 0, s>>>(mesh_view(m), tv, env_view(env), bvh_view(bvh), v, tri_id, bary,
                                                   kparams(p), L_ind, sec_rec, sec_vis, counters);
  else
    k_trace_indirect<false><<<nb, kThreads, 0, s>>>(mesh_view(m), tv, env_view(env), bvh_view(bvh), v, tri_id, bary,
                                                    kparams(p), L_ind, sec_rec, sec_vis, nullptr);
  return hipGetLastError();
}

hipError_t launch_trace_bwd(const exm_mesh* m, const exm_material* mat, const exm_env* env, const ShadeViews& v,
                            const int32_t* tri_id, const float* bary, const exm_params* p, float lambda_ind,
                            const float* dI, const exm_sec_rec* sec_rec, const uint64_t* sec_vis, float* dtex,
                            double* denv, hipStream_t s) {
  const int64_t n = (int64_t)v.n * v.H * v.W;
  k_trace_bwd<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(
      mesh_view(m), TexView{mat->Ht, mat->Wt, mat->tex}, env_view(env), v, tri_id, bary, kparams(p), lambda_ind, dI,
      sec_rec, sec_vis, dtex, denv);
  return hipGetLastError();
}

}  // namespace exm
