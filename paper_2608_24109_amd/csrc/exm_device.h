// Device-side building blocks of the render pass (gfx950, wave64).
//
// Shared by the forward and adjoint kernels so that both take every discrete decision
// (texel picks, ray directions, bilinear taps) from the same arithmetic.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "exm_internal.h"

namespace exm {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kInvPi = 0.318309886183790671538f;

// ------------------------------------------------------------------------------------------
// small vector helpers
// ------------------------------------------------------------------------------------------
struct f3 {
  float x, y, z;
};
__device__ __forceinline__ f3 mk(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator*(float s, f3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float len(f3 a) { return sqrtf(dot(a, a)); }
__device__ __forceinline__ f3 normalize(f3 a) { return (1.0f / len(a)) * a; }
__device__ __forceinline__ f3 ld3(const float* p, int64_t i) { return {p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }
__device__ __forceinline__ f3 ld3d(const double* p, int64_t i) {
  return {(float)p[3 * i], (float)p[3 * i + 1], (float)p[3 * i + 2]};
}

// ------------------------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon et al., SC'11)
// ------------------------------------------------------------------------------------------
struct Draw {
  uint64_t x;  // 64-bit word for the integer CDF target
  float u2, u3;
};

__device__ __forceinline__ Draw philox_draw(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                                            uint32_t c2, uint32_t c3) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Draw d;
  d.x = ((uint64_t)c0 << 32) | c1;
  d.u2 = (float)(c2 >> 8) * (1.0f / 16777216.0f);
  d.u3 = (float)(c3 >> 8) * (1.0f / 16777216.0f);
  return d;
}

struct RngKey {
  uint32_t k0, k1;
};
__host__ __device__ inline RngKey make_key(uint64_t seed, uint64_t iteration) {
  return {(uint32_t)seed ^ (uint32_t)(seed >> 32), (uint32_t)iteration};
}

// ------------------------------------------------------------------------------------------
// env importance sampling: integer CDF inversion, then uniform in solid angle in the texel
// ------------------------------------------------------------------------------------------
struct EnvView {
  int32_t He, We;
  const float* env;
  const uint64_t* cdf_row;
  const uint64_t* cdf_col;
  const float* pdf;
  const uint32_t* guide;  // cutpoint tables over cdf_row and each row of cdf_col (layout below)
  const float4* rec;      // per texel (E.r, E.g, E.b, 1/pdf)
  const uint32_t* cdf32;  // 32-bit copy of cdf_col inside guide, or null for maps too wide for it
  const uint16_t* col16;  // 16-bit copy of the column entries inside guide (null when cdf32 is)
  const uint16_t* cdf16;  // (cdf_col - 1) mod 2^16 inside guide (null when cdf32 is)
};

struct EnvSample {
  int32_t texel;
  f3 dir;
  float inv_pdf;
  float E[3];
};

// first index in [0, n) with a[i] > t (a is non-decreasing, a[n-1] > t)
__device__ __forceinline__ int32_t upper_bound_u64(const uint64_t* a, int32_t n, uint64_t t) {
  int32_t lo = 0, cnt = n;
  while (cnt > 0) {
    int32_t step = cnt >> 1;
    if (a[lo + step] <= t) {
      lo += step + 1;
      cnt -= step + 1;
    } else {
      cnt = step;
    }
  }
  return lo;
}

// first index in [lo, hi] with a[i] > t, given that one exists there (hi if none before it)
__device__ __forceinline__ int32_t upper_bound_range(const uint64_t* a, int32_t lo, int32_t hi, uint64_t t) {
  int32_t cnt = max(hi - lo, 0);
  while (cnt > 0) {
    const int32_t step = cnt >> 1;
    if (a[lo + step] <= t) {
      lo += step + 1;
      cnt -= step + 1;
    } else {
      cnt = step;
    }
  }
  return lo;
}

// Per-row constants of the within-texel theta sampling: (1 - cos(theta_i) for rows of the upper
// half or 1 + cos(theta_{i+1}) for the lower half, cos(theta_i) - cos(theta_{i+1})), from
// half-angle sines so that sin(theta) keeps full precision at both poles.
__device__ __forceinline__ float2 env_row_consts(int32_t row, int32_t He) {
  const float inv2He = 0.5f / (float)He;
  const float dlt = 2.0f * sinpif((float)(2 * row + 1) * inv2He) * sinpif(inv2He);
  float base;
  if (2 * row < He) {
    const float sa = sinpif((float)row * inv2He);
    base = 2.0f * sa * sa;
  } else {
    const float sb = sinpif((float)(He - row - 1) * inv2He);
    base = 2.0f * sb * sb;
  }
  return make_float2(base, dlt);
}

// (sin, cos) of phi_j = 2 pi j / We
__device__ __forceinline__ float2 env_col_consts(int32_t col, int32_t We) {
  float sj, cj;
  sincospif(2.0f * (float)col / (float)We, &sj, &cj);
  return make_float2(sj, cj);
}

// Block-shared copies of the row CDF, the row/column constants and the row cutpoints (LDS), or
// global pointers when the map is too large for them; either way env_sample computes
// bit-identical results.
struct EnvTabs {
  const uint64_t* cdf_row;
  const float2* rowc;
  const float2* colc;
  const uint32_t* rguide;  // row shift + row entries (He + 2)
  const uint32_t* cshift;  // column shift of each row (He)
};

__host__ __device__ inline size_t env_tabs_bytes(int32_t He, int32_t We) {
  return (size_t)He * 8 + (size_t)He * 8 + (size_t)We * 8 + (size_t)(2 * He + 2) * 4;
}
constexpr size_t kEnvTabsMaxBytes = 48 * 1024;

// Every thread of the block must call this (it synchronises the block).
__device__ __forceinline__ EnvTabs load_env_tabs(const EnvView& e, void* lds, bool use) {
  EnvTabs t{e.cdf_row, nullptr, nullptr, e.guide, e.guide + e.He + 2};
  if (!use) return t;
  uint64_t* cr = static_cast<uint64_t*>(lds);
  float2* rc = reinterpret_cast<float2*>(cr + e.He);
  float2* cc = rc + e.He;
  uint32_t* gd = reinterpret_cast<uint32_t*>(cc + e.We);
  for (int32_t i = threadIdx.x; i < e.He; i += blockDim.x) {
    cr[i] = e.cdf_row[i];
    rc[i] = env_row_consts(i, e.He);
  }
  for (int32_t j = threadIdx.x; j < e.We; j += blockDim.x) cc[j] = env_col_consts(j, e.We);
  for (int32_t k = threadIdx.x; k < 2 * e.He + 2; k += blockDim.x) gd[k] = e.guide[k];
  __syncthreads();
  t.cdf_row = cr;
  t.rowc = rc;
  t.colc = cc;
  t.rguide = gd;
  t.cshift = gd + e.He + 2;
  return t;
}

// sin(pi x) and cos(pi x) for |x| <= 1/32 by their Taylor series (terms to t^5 and t^6, t = pi x;
// the first omitted terms, t^7/5040 and t^8/40320, stay below 2e-11 and 3e-13: far under a float's
// rounding), in place of the general range-reduced evaluation
__device__ __forceinline__ void sincospi_small(float x, float* s, float* c) {
  const float t = x * kPi;
  const float t2 = t * t;
  *s = t * fmaf(t2, fmaf(t2, 1.0f / 120.0f, -1.0f / 6.0f), 1.0f);
  *c = fmaf(t2, fmaf(t2, fmaf(t2, -1.0f / 720.0f, 1.0f / 24.0f), -0.5f), 1.0f);
}

// K independent picks advanced stage by stage (rows in LDS, then the K cutpoint pairs, a
// lockstep column search, the K records), so that each thread has K loads in flight at every
// stage; every pick is the one a lone search returns. Picks with valid[j] false read nothing
// and leave out[j] untouched. REC false skips the record loads: out[j].E and out[j].inv_pdf are
// then left unset, for the caller to fetch with env_rec only for the picks it keeps.
// SMALL_PHI: the in-texel azimuth of maps at least 64 texels wide through sincospi_small (the
// direct pass, forward and adjoint; in the indirect kernels the second code path cost spills).
// A forward pass and its adjoint take the same path, so they draw identical directions.
template <int K, bool REC = true, bool SMALL_PHI = false>
__device__ __forceinline__ void env_sample_k(const EnvView& e, const EnvTabs& tb, const Draw (&d)[K],
                                             const bool (&valid)[K], EnvSample (&out)[K]) {
  const uint64_t Q = tb.cdf_row[e.He - 1];
  int32_t row[K], lo[K], cnt[K];
  uint64_t rem[K];
  int64_t cbase[K];  // offset of the picked row in cdf_col (or its 32-bit copy)
#pragma unroll
  for (int j = 0; j < K; ++j) {
    // target < Q whenever the tables are well formed; the clamps only keep a malformed table
    // (e.g. built from a NaN map) inside the arrays
    const uint64_t target = __umul64hi(d[j].x, Q);
    const uint32_t gr = (uint32_t)min(target >> tb.rguide[0], (uint64_t)(e.He - 1));
    const int32_t r = min(upper_bound_range(tb.cdf_row, (int32_t)tb.rguide[1 + gr], (int32_t)tb.rguide[2 + gr], target),
                          e.He - 1);
    row[j] = r;
    rem[j] = target - (r > 0 ? tb.cdf_row[r - 1] : 0ull);
    cbase[j] = (int64_t)r * e.We;
  }
  const bool narrow = e.cdf32 != nullptr;  // uniform; the compact copies hold the same values
  uint32_t g0[K], g1[K], mask16[K];  // mask16: 2^s - 1 for a row whose shift s is at most 16, else 0
#pragma unroll
  for (int j = 0; j < K; ++j) {
    g0[j] = g1[j] = 0u;
    mask16[j] = 0u;
    if (valid[j]) {
      const uint32_t cs = tb.cshift[row[j]];
      if (narrow && cs <= 16u) mask16[j] = (1u << cs) - 1u;
      const uint32_t gc = (uint32_t)min(rem[j] >> cs, (uint64_t)(e.We - 1));
      const int64_t at = (int64_t)row[j] * (e.We + 1) + gc;
      if (narrow) {
        g0[j] = e.col16[at];
        g1[j] = e.col16[at + 1];
      } else {
        const uint32_t* cg = e.guide + 2 * (int64_t)e.He + 2 + at;
        g0[j] = cg[0];
        g1[j] = cg[1];
      }
    }
  }
  bool more = false;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    lo[j] = (int32_t)g0[j];
    cnt[j] = valid[j] ? max((int32_t)g1[j] - (int32_t)g0[j], 0) : 0;
    more |= cnt[j] > 0;
  }
  while (more) {  // binary search over [lo, lo + cnt], one probe of every pick per round
    bool le[K];  // cdf_col[probe] <= rem
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (cnt[j] > 0) {
        const int64_t at = cbase[j] + lo[j] + (cnt[j] >> 1);
        // a row with shift 0 (mask16 0, every probe above rem) takes the 32-bit path
        if (mask16[j] != 0u)
          le[j] = ((uint32_t)e.cdf16[at] & mask16[j]) < ((uint32_t)rem[j] & mask16[j]);
        else
          le[j] = (narrow ? (uint64_t)e.cdf32[at] : e.cdf_col[at]) <= rem[j];
      }
    more = false;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (cnt[j] > 0) {
        const int32_t step = cnt[j] >> 1;
        if (le[j]) {
          lo[j] += step + 1;
          cnt[j] -= step + 1;
        } else {
          cnt[j] = step;
        }
      }
      more |= cnt[j] > 0;
    }
  }
  float4 rec[K];
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (REC && valid[j]) rec[j] = e.rec[row[j] * e.We + min(lo[j], e.We - 1)];
  const float two_over_We = 2.0f / (float)e.We;  // one division per call instead of one per pick
  const bool small_phi = SMALL_PHI && e.We >= 64;  // the in-texel angle is then at most pi/32
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (!valid[j]) continue;
    const int32_t r = row[j], col = min(lo[j], e.We - 1);
    EnvSample s;
    s.texel = r * e.We + col;
    // theta in [row, row+1] * pi/He with cos(theta) uniform
    const float2 rc = tb.rowc ? tb.rowc[r] : env_row_consts(r, e.He);
    float ct, st2;
    if (2 * r < e.He) {
      const float omc = rc.x + d[j].u3 * rc.y;  // 1 - cos(theta)
      ct = 1.0f - omc;
      st2 = omc * (2.0f - omc);
    } else {
      const float opc = rc.x + (1.0f - d[j].u3) * rc.y;  // 1 + cos(theta)
      ct = opc - 1.0f;
      st2 = opc * (2.0f - opc);
    }
    const float st = sqrtf(fmaxf(st2, 0.0f));
    // phi = 2 pi (col + u2) / We by angle addition (keeps u2's resolution at large col)
    const float2 cj = tb.colc ? tb.colc[col] : env_col_consts(col, e.We);
    float sd, cd;
    if (small_phi)
      sincospi_small(d[j].u2 * two_over_We, &sd, &cd);
    else
      sincospif(d[j].u2 * two_over_We, &sd, &cd);
    const float cphi = cj.y * cd - cj.x * sd, sphi = cj.x * cd + cj.y * sd;
    s.dir = mk(st * cphi, ct, st * sphi);
    if (REC) {
      s.inv_pdf = rec[j].w;
      s.E[0] = rec[j].x;
      s.E[1] = rec[j].y;
      s.E[2] = rec[j].z;
    }
    out[j] = s;
  }
}

// the record (E, 1/pdf) of a pick taken with REC false
__device__ __forceinline__ void env_rec(const EnvView& e, EnvSample& s) {
  const float4 r = e.rec[s.texel];
  s.inv_pdf = r.w;
  s.E[0] = r.x;
  s.E[1] = r.y;
  s.E[2] = r.z;
}

__device__ __forceinline__ EnvSample env_sample(const EnvView& e, const EnvTabs& tb, const Draw& d) {
  const Draw dd[1] = {d};
  const bool ok[1] = {true};
  EnvSample s[1];
  env_sample_k<1>(e, tb, dd, ok, s);
  return s[0];
}

// ------------------------------------------------------------------------------------------
// attribute query at a surface point (Attribute Query, Eq. 10-11)
// ------------------------------------------------------------------------------------------
struct MeshView {
  int32_t nV, nF;
  const float* pos;
  const int32_t* tri;
  const float* uv;
  const int32_t* tri_uv;
  const double* vnrm;
  const float* ftan;
};

struct TexView {
  int32_t Ht, Wt;
  const float* tex;
};

struct Surf {
  f3 x, ng;
  f3 T, B;       // Gram-Schmidt tangent frame (valid if map_ok)
  f3 ns;         // shading normal
  float vlen;    // |q.x T + q.y B + q.z n_g| (map_ok only)
  bool map_ok;   // normal map applied (otherwise n_s = n_g)
  int32_t tap[4];
  float w[4];
  float a[3], r, m, q[3];
};

// Texel-space position in FP64: with i.i.d. texel values the material is sensitive to the
// sample position at the scale of one texel, and a float u (ulp 6e-8) would already move it by
// 1e-4 texel on a 2048^2 map.
__device__ __forceinline__ void bilinear_taps(const TexView& t, double u, double v, int32_t tap[4], float w[4]) {
  u = fmin(1.0, fmax(0.0, u));
  v = fmin(1.0, fmax(0.0, v));
  const double s = u * (double)t.Wt - 0.5, tt = v * (double)t.Ht - 0.5;
  const double s0 = floor(s), t0 = floor(tt);
  const float fs = (float)(s - s0), ft = (float)(tt - t0);
  const int32_t i0 = (int32_t)s0, j0 = (int32_t)t0;
  const int32_t ia = min(t.Wt - 1, max(0, i0)), ib = min(t.Wt - 1, max(0, i0 + 1));
  const int32_t ja = min(t.Ht - 1, max(0, j0)), jb = min(t.Ht - 1, max(0, j0 + 1));
  tap[0] = ja * t.Wt + ia;
  tap[1] = ja * t.Wt + ib;
  tap[2] = jb * t.Wt + ia;
  tap[3] = jb * t.Wt + ib;
  w[0] = (1.0f - fs) * (1.0f - ft);
  w[1] = fs * (1.0f - ft);
  w[2] = (1.0f - fs) * ft;
  w[3] = fs * ft;
}

// bilinear taps of the maps at the point (b1, b2) of face f (UVs interpolated in FP64)
__device__ __forceinline__ void surface_taps(const MeshView& M, const TexView& T, int32_t f, float b1, float b2,
                                             int32_t tap[4], float w[4]) {
  const int32_t t0 = M.tri_uv[3 * f], t1 = M.tri_uv[3 * f + 1], t2 = M.tri_uv[3 * f + 2];
  const double d1 = b1, d2 = b2, d0 = 1.0 - d1 - d2;
  const double u = (d0 * M.uv[2 * t0] + d1 * M.uv[2 * t1]) + d2 * M.uv[2 * t2];
  const double v = (d0 * M.uv[2 * t0 + 1] + d1 * M.uv[2 * t1 + 1]) + d2 * M.uv[2 * t2 + 1];
  bilinear_taps(T, u, v, tap, w);
}

// Albedo of secondary hits under EXM_NO_SECONDARY_MATERIAL (a grey Lambertian, metallic 0,
// shading normal = n_g; the "No Secondary Material" ablation of the Ablation Study).
constexpr float kSecondaryAlbedo = 0.5f;

// with_material = false: the maps are not read (the no-secondary-material reading above).
__device__ __forceinline__ Surf query(const MeshView& M, const TexView& T, int32_t f, float b1, float b2,
                                      uint32_t flags, bool with_material = true) {
  Surf S;
  const float b0 = 1.0f - b1 - b2;
  const int32_t v0 = M.tri[3 * f], v1 = M.tri[3 * f + 1], v2 = M.tri[3 * f + 2];
  const f3 P0 = ld3(M.pos, v0), P1 = ld3(M.pos, v1), P2 = ld3(M.pos, v2);
  S.x = (b0 * P0 + b1 * P1) + b2 * P2;
  const f3 N0 = ld3d(M.vnrm, v0), N1 = ld3d(M.vnrm, v1), N2 = ld3d(M.vnrm, v2);
  S.ng = normalize((b0 * N0 + b1 * N1) + b2 * N2);
  if (!with_material) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      S.tap[k] = 0;
      S.w[k] = 0.0f;
    }
    S.a[0] = S.a[1] = S.a[2] = kSecondaryAlbedo;
    S.r = 1.0f;
    S.m = 0.0f;
    S.q[0] = S.q[1] = 0.0f;
    S.q[2] = 1.0f;
    S.map_ok = false;
    S.ns = S.ng;
    S.vlen = 1.0f;
    S.T = S.B = mk(0, 0, 0);
    return S;
  }
  surface_taps(M, T, f, b1, b2, S.tap, S.w);
  float ch[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) ch[c] = 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float4* tp = reinterpret_cast<const float4*>(T.tex + (int64_t)S.tap[k] * 8);
    const float4 lo = tp[0], hi = tp[1];
    ch[0] += S.w[k] * lo.x;
    ch[1] += S.w[k] * lo.y;
    ch[2] += S.w[k] * lo.z;
    ch[3] += S.w[k] * lo.w;
    ch[4] += S.w[k] * hi.x;
    ch[5] += S.w[k] * hi.y;
    ch[6] += S.w[k] * hi.z;
    ch[7] += S.w[k] * hi.w;
  }
  S.a[0] = ch[0];
  S.a[1] = ch[1];
  S.a[2] = ch[2];
  S.r = ch[3];
  S.m = (flags & EXM_METALLIC_OFF) ? 0.0f : ch[4];
  S.q[0] = ch[5];
  S.q[1] = ch[6];
  S.q[2] = ch[7];
  const float4 ft = reinterpret_cast<const float4*>(M.ftan)[f];
  const f3 Tf = mk(ft.x, ft.y, ft.z);
  f3 Tp = Tf - dot(S.ng, Tf) * S.ng;
  const float lt = len(Tp);
  S.map_ok = false;
  S.ns = S.ng;
  S.vlen = 1.0f;
  S.T = S.B = mk(0, 0, 0);
  if (lt >= 1e-12f) {
    Tp = (1.0f / lt) * Tp;
    const f3 Bp = ft.w * cross(S.ng, Tp);
    const f3 vv = (S.q[0] * Tp + S.q[1] * Bp) + S.q[2] * S.ng;
    const float lv = len(vv);
    if (lv >= 1e-12f) {
      S.map_ok = true;
      S.T = Tp;
      S.B = Bp;
      S.vlen = lv;
      S.ns = (1.0f / lv) * vv;
    }
  }
  return S;
}

// ------------------------------------------------------------------------------------------
// metallic-roughness BRDF (Eq. 13-16): GGX D with sin^2 = |n x h|^2, separable Smith-GGX G,
// Schlick F, alpha = r^2
// ------------------------------------------------------------------------------------------
struct Spec {
  bool on;               // f_s evaluated (n.wi > 0, n.wo > 0, |wi + wo| > 0)
  f3 h;
  float ci, co, alpha2;  // n.wi, n.wo, alpha^2
  float chh, d;          // n.h, sin^2 + alpha^2 cos^2
  float D, G1i, G1o, si, so;  // D, G1(wi), G1(wo), sqrt terms of G1
  float den, x5;          // 4 ci co + eps, (1 - wi.h)^5
  bool alpha_clamped;
};

__device__ __forceinline__ Spec spec_terms(f3 n, f3 wi, f3 wo, float ci, float r, float eps) {
  Spec s;
  s.on = false;
  const f3 hs = wi + wo;
  const float hl = len(hs);
  s.co = dot(n, wo);
  s.ci = ci;
  if (!(hl >= 1e-12f) || !(s.co > 0.0f) || !(ci > 0.0f)) return s;
  s.on = true;
  s.h = __builtin_amdgcn_rcpf(hl) * hs;
  const float alpha = r * r;
  s.alpha2 = alpha * alpha;
  s.alpha_clamped = s.alpha2 < 1e-12f;
  if (s.alpha_clamped) s.alpha2 = 1e-12f;
  s.chh = dot(n, s.h);
  const f3 nx = cross(n, s.h);
  s.d = dot(nx, nx) + s.alpha2 * s.chh * s.chh;
  s.D = s.alpha2 * __builtin_amdgcn_rcpf(kPi * s.d * s.d);
  s.si = sqrtf(s.alpha2 + (1.0f - s.alpha2) * ci * ci);
  s.so = sqrtf(s.alpha2 + (1.0f - s.alpha2) * s.co * s.co);
  s.G1i = 2.0f * ci * __builtin_amdgcn_rcpf(ci + s.si);
  s.G1o = 2.0f * s.co * __builtin_amdgcn_rcpf(s.co + s.so);
  const float x = 1.0f - fmaxf(dot(wi, s.h), 0.0f);
  const float x2 = x * x;
  s.x5 = x2 * x2 * x;
  s.den = 4.0f * ci * s.co + eps;
  return s;
}

// ------------------------------------------------------------------------------------------
// BVH (binned SAH, collapsed to 128-byte 4-wide nodes) and ray queries
// ------------------------------------------------------------------------------------------
struct BvhView {
  const BvhNode4* nodes;  // 4-wide nodes, root at 0
  const BvhTri* tris;
};

// ray precomputation for the watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013)
struct Ray {
  f3 o, d, inv;
  f3 off_n, off_f;    // slab offsets of the entry and exit planes: o * inv moved outwards per axis
  int32_t nb_x, nb_y, nb_z;  // byte offsets of the entry planes of an axis in a wide node
  int kx, ky, kz;
  float Sx, Sy, Sz;
};

// Slab offsets for the one-FMA slab distance fma(plane, inv, -off): off approximates o * inv,
// moved by 2^-21 |o * inv| (at least three ulps after rounding) so that the entry distance of
// each axis comes out no larger (the entry plane's offset, oi + e) and the exit distance no
// smaller (the exit plane's, oi - e) than (plane - o) * inv would give: the box test stays
// conservative, and the padding is a few ulps of the coordinates along that axis alone. The entry
// plane of an axis is its lo plane where inv >= 0 and its hi plane otherwise.
__device__ __forceinline__ void slab_offsets(float o, float inv, float* off_n, float* off_f) {
  const float oi = o * inv;
  const float e = fabsf(oi) * 0x1p-21f;
  *off_n = oi + e;
  *off_f = oi - e;
}

__device__ __forceinline__ float comp(f3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

__device__ __forceinline__ Ray make_ray(f3 o, f3 d) {
  Ray r;
  r.o = o;
  r.d = d;
  // hardware reciprocals (1 ulp): the slab test pads its interval by a few ulps, and the shear
  // below only needs to be the same for every triangle a ray meets
  // a zero component gives +-2^64 instead of an infinite reciprocal, so that the slab distances
  // below stay finite (inf - inf would read as NaN and could drop a slab the ray lies in)
  r.inv = mk(copysignf(fminf(fabsf(__builtin_amdgcn_rcpf(d.x)), 0x1p64f), d.x),
             copysignf(fminf(fabsf(__builtin_amdgcn_rcpf(d.y)), 0x1p64f), d.y),
             copysignf(fminf(fabsf(__builtin_amdgcn_rcpf(d.z)), 0x1p64f), d.z));
  slab_offsets(o.x, r.inv.x, &r.off_n.x, &r.off_f.x);
  slab_offsets(o.y, r.inv.y, &r.off_n.y, &r.off_f.y);
  slab_offsets(o.z, r.inv.z, &r.off_n.z, &r.off_f.z);
  // a wide node stores lo x, y, z then hi x, y, z, 16 bytes each (four children)
  r.nb_x = r.inv.x >= 0.0f ? 0 : 48;
  r.nb_y = r.inv.y >= 0.0f ? 16 : 64;
  r.nb_z = r.inv.z >= 0.0f ? 32 : 80;
  const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  r.kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
  r.kx = r.kz == 2 ? 0 : r.kz + 1;
  r.ky = r.kx == 2 ? 0 : r.kx + 1;
  if (comp(d, r.kz) < 0.0f) {
    int t = r.kx;
    r.kx = r.ky;
    r.ky = t;
  }
  const float dz = comp(d, r.kz);
  r.Sz = __builtin_amdgcn_rcpf(dz);
  r.Sx = comp(d, r.kx) * r.Sz;
  r.Sy = comp(d, r.ky) * r.Sz;
  return r;
}

// returns true on hit with t in [tmin, tmax]; writes t and barycentrics (b1, b2)
__device__ __forceinline__ bool tri_hit(const Ray& r, const BvhTri& T, float tmin, float tmax, float* t_out,
                                        float* b1, float* b2) {
  const f3 A = mk(T.v0[0], T.v0[1], T.v0[2]) - r.o;
  const f3 B = mk(T.v1[0], T.v1[1], T.v1[2]) - r.o;
  const f3 C = mk(T.v2[0], T.v2[1], T.v2[2]) - r.o;
  const float Az0 = comp(A, r.kz), Bz0 = comp(B, r.kz), Cz0 = comp(C, r.kz);
  const float Ax = comp(A, r.kx) - r.Sx * Az0, Ay = comp(A, r.ky) - r.Sy * Az0;
  const float Bx = comp(B, r.kx) - r.Sx * Bz0, By = comp(B, r.ky) - r.Sy * Bz0;
  const float Cx = comp(C, r.kx) - r.Sx * Cz0, Cy = comp(C, r.ky) - r.Sy * Cz0;
  float U = Cx * By - Cy * Bx;
  float V = Ax * Cy - Ay * Cx;
  float W = Bx * Ay - By * Ax;
  if (U == 0.0f || V == 0.0f || W == 0.0f) {  // edge case: redo in double for watertightness
    U = (float)((double)Cx * By - (double)Cy * Bx);
    V = (float)((double)Ax * Cy - (double)Ay * Cx);
    W = (float)((double)Bx * Ay - (double)By * Ax);
  }
  if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
  const float det = U + V + W;
  if (det == 0.0f) return false;
  const float Tn = U * (r.Sz * Az0) + V * (r.Sz * Bz0) + W * (r.Sz * Cz0);
  const float inv = __builtin_amdgcn_rcpf(det);
  const float t = Tn * inv;
  if (!(t >= tmin && t <= tmax)) return false;
  *t_out = t;
  *b1 = V * inv;
  *b2 = W * inv;
  return true;
}

// Slab test of one child box given its entry planes (nx, ny, nz) and exit planes (fx, fy, fz) for
// this ray: the entry distance if the ray's interval [0, tmax] meets the box, kSlabMiss otherwise.
// Taking each axis's entry and exit plane by the sign of 1/d gives the same distances as the
// minimum and maximum of its two plane distances would for every valid box, and a box with
// lo = +inf and hi = -inf (an empty slot) always has entry +inf and exit -inf, so it is never
// met. Any-hit queries pass CLAMP = false: their tmax stays +inf for the whole query, and
// min(x, +inf) = x for every x (a NaN operand included, under the IEEE minimum the clamp would
// use), so dropping the clamp gives the same answer.
constexpr float kSlabMiss = __builtin_huge_valf();
template <bool CLAMP>
__device__ __forceinline__ float slab_entry(float nx, float ny, float nz, float fx, float fy, float fz, const Ray& r,
                                            float tmax) {
  const float tnx = fmaf(nx, r.inv.x, -r.off_n.x), tfx = fmaf(fx, r.inv.x, -r.off_f.x);
  const float tny = fmaf(ny, r.inv.y, -r.off_n.y), tfy = fmaf(fy, r.inv.y, -r.off_f.y);
  const float tnz = fmaf(nz, r.inv.z, -r.off_n.z), tfz = fmaf(fz, r.inv.z, -r.off_f.z);
  const float tn = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, 0.0f));
  const float fzc = CLAMP ? fminf(tfz, tmax) : tfz;
  const float tf = fminf(fminf(tfx, tfy), fzc);
  // conservative by a few ulps so rays grazing a box face are not lost
  return tn <= tf * 1.00000024f ? tn : kSlabMiss;
}

struct HitRec {
  int32_t id;  // original triangle id, -1 = miss
  float t, b1, b2;
};

// work counters of the measurement variants (node visits, triangle tests)
struct TraceCount {
  uint32_t nodes = 0, tris = 0;
};

// Resumable traversal state: the node to visit next, one postponed leaf, the depth of the
// lane's stack of deferred node references (LaneStack), and the number of rounds the query has
// taken.
struct TravState {
  int32_t ref;
  int32_t leaf;
  int32_t sp;
  uint32_t rounds;
};

constexpr int32_t kEmptyRef = (int32_t)0x80000000;
// Work caps: node visits of one round (counted per wave: the lanes still in a round's node loop
// have all made the same number of passes) and rounds of one query. The builder bounds the work
// far below both; they only keep a corrupted structure from trapping a wave.
constexpr uint32_t kMaxSteps = 1u << 22;
constexpr uint32_t kMaxRounds = 1u << 22;

__device__ __forceinline__ bool is_leaf(int32_t ref) { return ref < 0 && ref != kEmptyRef; }

// The lane's stack: entries [0, kStackLds) in LDS at stack[i * stride], the rest in its private
// overflow array. The overflow pointer carries the private address space so that the compiler
// keeps its accesses apart from the LDS ones (as two generic pointers, the two loads of a pop merge
// into one generic-address load on every pop).
typedef volatile __attribute__((address_space(5))) int32_t private_i32;  // private (scratch) memory, kept there
struct LaneStack {
  int32_t* lds;
  private_i32* ovf;
  int stride;
};

// The lane's stack starts with kEmptyRef as a sentinel in its bottom slot: popping it ends the
// query, so a pop never needs to test for an empty stack (a query pops nothing after it).
__device__ __forceinline__ void trav_begin(const BvhView& B, TravState& s, HitRec& h, const LaneStack& st) {
  (void)B;
  s.ref = 0;  // the wide root always exists (a mesh in one leaf, or none, hangs from its slots)
  s.leaf = kEmptyRef;
  st.lds[0] = kEmptyRef;
  s.sp = 1;
  s.rounds = 0;
  h.id = -1;
  h.t = __builtin_huge_valf();
  h.b1 = h.b2 = 0.0f;
}

__device__ __forceinline__ int32_t trav_pop(TravState& s, const LaneStack& st) {
  --s.sp;
  if (s.sp < kStackLds) return st.lds[s.sp * st.stride];
  return st.ovf[s.sp - kStackLds];
}

// order in which an any-hit query visits the hit children of a wide node: 0 slot order, 1 nearest
// first, 2 by distance
constexpr int kAnyOrder = 1;

// guarded push: the builder's depth bound keeps the stack within kStack entries
__device__ __forceinline__ void trav_push(TravState& s, const LaneStack& st, int32_t ref) {
  if (s.sp < kStackLds) {
    st.lds[(s.sp++) * st.stride] = ref;
  } else if (s.sp < kStack) {
    st.ovf[s.sp - kStackLds] = ref;
    ++s.sp;
  }
}

// (ka, ra), (kb, rb) in ascending order of k (ties keep their order)
__device__ __forceinline__ void sort2(float& ka, int32_t& ra, float& kb, int32_t& rb) {
  const bool sw = kb < ka;
  const float k = sw ? kb : ka;
  const int32_t r = sw ? rb : ra;
  kb = sw ? ka : kb;
  rb = sw ? ra : rb;
  ka = k;
  ra = r;
}

// inclusive prefix sum of x over the 64 lanes of the wave (every lane must be active)
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if ((int)__lane_id() >= o) x += y;
  }
  return x;
}

// Any-hit test of up to two leaves of one lane by that lane alone (their triangles in order).
template <bool COUNT>
__device__ __forceinline__ bool leaves_any_lane(const BvhView& B, const Ray& r, float tmin, int32_t skip,
                                                int32_t leaf_a, int32_t leaf_b, TraceCount* counts) {
  const int32_t leaves[2] = {leaf_a, leaf_b};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (leaves[k] == kEmptyRef) continue;
    const uint32_t v = ~(uint32_t)leaves[k];
    const uint32_t first = v >> 4, cnt = v & 15u;
    for (uint32_t i = first; i < first + cnt; ++i) {
      const float4* qp = reinterpret_cast<const float4*>(B.tris + i);
      const float4 q0 = qp[0], q1 = qp[1], q2 = qp[2];
      BvhTri T;
      T.v0[0] = q0.x; T.v0[1] = q0.y; T.v0[2] = q0.z;
      T.v1[0] = q0.w; T.v1[1] = q1.x; T.v1[2] = q1.y;
      T.v2[0] = q1.z; T.v2[1] = q1.w; T.v2[2] = q2.x;
      T.id = __float_as_int(q2.y);
      if (COUNT) counts->tris++;
      float t, b1, b2;
      if (tri_hit(r, T, tmin, __builtin_huge_valf(), &t, &b1, &b2) && T.id != skip) return true;
    }
  }
  return false;
}

// Any-hit test of every lane's pending leaves (up to two) against that lane's ray, with the
// (lane, triangle) pairs of the whole wave spread over its 64 lanes: pair q (in lane order) goes
// to lane q mod 64 in pass q / 64, which finds the pair's owner by a 4-ary search over the lanes'
// prefix sums (three rounds of three independent cross-lane reads), takes the owner's ray,
// triangle ranges and skipped triangle by cross-lane reads and runs the watertight test. A lane's
// own pairs are a run of consecutive lanes in each pass, so one ballot tells every owner whether
// any of its tests hit. The cross-lane reads need every lane of the wave to take part: if the
// call is reached with some lanes inactive, each active lane tests its own leaves instead (same
// answers). kEmptyRef stands for no leaf; returns true where the lane's ray hit something
// (t >= tmin, its own triangle skipped).
template <bool COUNT, bool PER_LANE_BVH>
__device__ __forceinline__ bool leaves_any_wave(const BvhView& B, const Ray& r, float tmin, int32_t skip,
                                                int32_t leaf_a, int32_t leaf_b, TraceCount* counts) {
  if (__ballot(1) != ~0ull) return leaves_any_lane<COUNT>(B, r, tmin, skip, leaf_a, leaf_b, counts);
  uint32_t ca = 0, fa = 0, cb = 0, fb = 0;
  if (leaf_a != kEmptyRef) {
    const uint32_t v = ~(uint32_t)leaf_a;
    fa = v >> 4;
    ca = v & 15u;
  }
  if (leaf_b != kEmptyRef) {
    const uint32_t v = ~(uint32_t)leaf_b;
    fb = v >> 4;
    cb = v & 15u;
  }
  const uint32_t cnt = ca + cb;
  const uint32_t incl = wave_incl_sum(cnt);
  const uint32_t excl = incl - cnt;
  // the wave's pair count, in a scalar register (every lane reads the same lane)
  const uint32_t total = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)incl, 63, 64));
  const uint32_t lane = __lane_id();
  const int kpack = r.kx | (r.ky << 2) | (r.kz << 4);
  const uint64_t tris_addr = reinterpret_cast<uint64_t>(B.tris);
  bool hit = false;
  for (uint32_t base = 0; base < total; base += 64) {  // scalar loop
    const uint32_t q = base + lane;
    // owner = the number of lanes whose pairs all come before q (incl[o - 1] <= q < incl[o]),
    // found 16, 4 and 1 lanes at a time
    uint32_t o = 0;
#pragma unroll
    for (uint32_t st = 16; st >= 1; st >>= 2) {
      const uint32_t e1 = (uint32_t)__shfl((int)incl, (int)(o + st - 1), 64);
      const uint32_t e2 = (uint32_t)__shfl((int)incl, (int)(o + 2 * st - 1), 64);
      const uint32_t e3 = (uint32_t)__shfl((int)incl, (int)(o + 3 * st - 1), 64);
      o += st * ((e1 <= q) + (e2 <= q) + (e3 <= q));
    }
    o = min(o, 63u);  // a q past the last pair has no owner; its reads below are unused
    const uint32_t o_fa = (uint32_t)__shfl((int)fa, (int)o, 64);
    const uint32_t o_ca = (uint32_t)__shfl((int)ca, (int)o, 64);
    const uint32_t o_fb = (uint32_t)__shfl((int)fb, (int)o, 64);
    const uint32_t o_excl = (uint32_t)__shfl((int)excl, (int)o, 64);
    Ray ro;
    ro.o = mk(__shfl(r.o.x, (int)o, 64), __shfl(r.o.y, (int)o, 64), __shfl(r.o.z, (int)o, 64));
    ro.Sx = __shfl(r.Sx, (int)o, 64);
    ro.Sy = __shfl(r.Sy, (int)o, 64);
    ro.Sz = __shfl(r.Sz, (int)o, 64);
    const int o_k = __shfl(kpack, (int)o, 64);
    ro.kx = o_k & 3;
    ro.ky = (o_k >> 2) & 3;
    ro.kz = (o_k >> 4) & 3;
    const float o_tmin = __shfl(tmin, (int)o, 64);
    const int32_t o_skip = __shfl(skip, (int)o, 64);
    const BvhTri* tris = B.tris;
    if (PER_LANE_BVH) {
      const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)tris_addr, (int)o, 64);
      const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(tris_addr >> 32), (int)o, 64);
      tris = reinterpret_cast<const BvhTri*>(((uint64_t)hi << 32) | lo);
    }
    bool my = false;
    const uint32_t k = q - o_excl;  // the pair's place among its owner's (first leaf, then second)
    if (q < total && k < 30u) {
      const uint32_t idx = k < o_ca ? o_fa + k : o_fb + (k - o_ca);
      const float4* qp = reinterpret_cast<const float4*>(tris + idx);
      const float4 q0 = qp[0], q1 = qp[1], q2 = qp[2];
      BvhTri T;
      T.v0[0] = q0.x; T.v0[1] = q0.y; T.v0[2] = q0.z;
      T.v1[0] = q0.w; T.v1[1] = q1.x; T.v1[2] = q1.y;
      T.v2[0] = q1.z; T.v2[1] = q1.w; T.v2[2] = q2.x;
      T.id = __float_as_int(q2.y);
      float t, b1, b2;
      my = tri_hit(ro, T, o_tmin, __builtin_huge_valf(), &t, &b1, &b2) && T.id != o_skip;
    }
    const uint64_t hits = __ballot(my);
    // this lane's own pairs occupy lanes [lo, hi) of the pass
    const uint32_t lo = min(max(excl, base), base + 64u) - base, hi = min(max(incl, base), base + 64u) - base;
    const uint32_t n = hi - lo;
    const uint64_t mine = n == 0 ? 0ull : ((n == 64 ? ~0ull : ((1ull << n) - 1ull)) << lo);
    hit = hit || (hits & mine) != 0ull;
    if (COUNT) counts->tris += n;
  }
  return hit;
}

// One round of the speculative while-while traversal (Aila and Laine 2009): internal nodes are
// visited until fewer than leaf_gate lanes of the wave lack a postponed leaf, then the postponed
// leaves are intersected together, so node and leaf work each run with most lanes of the wave
// active. Every lane of the wave calls it (lanes without a query hold s.ref = s.leaf = kEmptyRef):
// any-hit queries test their leaves across the whole wave (leaf_any_wave). Returns true when
// the lane's query is finished: nothing left to visit, or ANY and a hit was found.
template <bool ANY, bool COUNT, bool PER_LANE_BVH = false>
__device__ __forceinline__ bool trav_round(const BvhView& B, const Ray& r, float tmin, int32_t skip,
                                           const LaneStack& st, TravState& s, HitRec& h, TraceCount* counts,
                                           int32_t leaf_gate = 1) {
  bool capped = false;
  if (++s.rounds > kMaxRounds) {  // drop the query (no early return: the leaf phase needs every lane)
    s.ref = s.leaf = kEmptyRef;
    capped = true;
  }
  uint32_t steps = 0;
  while (s.ref >= 0) {
    steps = __builtin_amdgcn_readfirstlane(steps) + 1u;  // wave-uniform: kept in a scalar register
    if (steps > kMaxSteps) {
      s.ref = s.leaf = kEmptyRef;
      capped = true;
      break;
    }
    if (COUNT) counts->nodes++;
    // one 4-wide node: the entry and exit planes of the four children for this ray's direction
    // signs (per-lane byte offsets into the node), then the child references
    // 32-bit byte offsets from the node array (a wide tree of at most 2^25 triangles stays under
    // 2^31 bytes), so that each load is a scalar base plus one vector offset
    const char* nb = reinterpret_cast<const char*>(B.nodes);
    const uint32_t at = (uint32_t)s.ref * (uint32_t)sizeof(BvhNode4);
    const float4 nx = *reinterpret_cast<const float4*>(nb + (at + (uint32_t)r.nb_x));
    const float4 fx = *reinterpret_cast<const float4*>(nb + (at + (uint32_t)(48 - r.nb_x)));
    const float4 ny = *reinterpret_cast<const float4*>(nb + (at + (uint32_t)r.nb_y));
    const float4 fy = *reinterpret_cast<const float4*>(nb + (at + (uint32_t)(80 - r.nb_y)));
    const float4 nz = *reinterpret_cast<const float4*>(nb + (at + (uint32_t)r.nb_z));
    const float4 fz = *reinterpret_cast<const float4*>(nb + (at + (uint32_t)(112 - r.nb_z)));
    const int4 cr = *reinterpret_cast<const int4*>(nb + (at + 96u));
    constexpr float kMiss = kSlabMiss;
    // entry distance of a hit child, kMiss otherwise
    float k0 = slab_entry<!ANY>(nx.x, ny.x, nz.x, fx.x, fy.x, fz.x, r, h.t);
    float k1 = slab_entry<!ANY>(nx.y, ny.y, nz.y, fx.y, fy.y, fz.y, r, h.t);
    float k2 = slab_entry<!ANY>(nx.z, ny.z, nz.z, fx.z, fy.z, fz.z, r, h.t);
    float k3 = slab_entry<!ANY>(nx.w, ny.w, nz.w, fx.w, fy.w, fz.w, r, h.t);
    int32_t r0 = cr.x, r1 = cr.y, r2 = cr.z, r3 = cr.w;
    // the child references are needed only when a child is hit, and the compiler would load them
    // after the test (a second round trip per visit); taking them here keeps the load beside the
    // six plane loads
    asm volatile("" ::"v"(r0), "v"(r1), "v"(r2), "v"(r3));
    if (ANY && kAnyOrder == 0) {  // slot order: descend into the first hit child, defer the others
      int32_t nxt = kEmptyRef;
      if (k3 != kMiss) nxt = r3;
      if (k2 != kMiss) {
        if (nxt != kEmptyRef) trav_push(s, st, nxt);
        nxt = r2;
      }
      if (k1 != kMiss) {
        if (nxt != kEmptyRef) trav_push(s, st, nxt);
        nxt = r1;
      }
      if (k0 != kMiss) {
        if (nxt != kEmptyRef) trav_push(s, st, nxt);
        nxt = r0;
      }
      s.ref = nxt != kEmptyRef ? nxt : trav_pop(s, st);
    } else {
      // nearest first: a four-input sorting network on (distance, reference), misses last; any-hit
      // queries with kAnyOrder 1 only bring the nearest to the front (the first three exchanges)
      sort2(k0, r0, k1, r1);
      sort2(k2, r2, k3, r3);
      sort2(k0, r0, k2, r2);
      if (!(ANY && kAnyOrder == 1)) {
        sort2(k1, r1, k3, r3);
        sort2(k1, r1, k2, r2);
      }
      if (k0 == kMiss) {
        s.ref = trav_pop(s, st);
      } else {  // descend into the nearest, defer the others (farthest first when sorted)
        s.ref = r0;
        const bool c1 = k1 != kMiss, c2 = k2 != kMiss, c3 = k3 != kMiss;
        if (s.sp + 3 <= kStackLds) {
          // room for three in LDS: the deferred ones packed in the order r3, r2, r1 (r1 on top),
          // all three slots written and the depth advanced by their number (what lies above the
          // new top is never read)
          const int32_t e0 = c3 ? r3 : (c2 ? r2 : r1);
          const int32_t e1 = c3 ? (c2 ? r2 : r1) : r1;
          st.lds[s.sp * st.stride] = e0;
          st.lds[(s.sp + 1) * st.stride] = e1;
          st.lds[(s.sp + 2) * st.stride] = r1;
          s.sp += (int32_t)c1 + (int32_t)c2 + (int32_t)c3;
        } else {
          if (c3) trav_push(s, st, r3);
          if (c2) trav_push(s, st, r2);
          if (c1) trav_push(s, st, r1);
        }
      }
    }
    if (is_leaf(s.ref) && s.leaf == kEmptyRef) {  // postpone the leaf, keep descending
      s.leaf = s.ref;
      s.ref = trav_pop(s, st);
    }
    if (__popcll(__ballot(s.leaf == kEmptyRef)) < leaf_gate) break;
  }
  if (s.leaf == kEmptyRef && is_leaf(s.ref)) {  // a round that starts on a leaf (a root leaf, or the
                                                // second of two leaves met in the last round)
    s.leaf = s.ref;
    s.ref = trav_pop(s, st);
  }
  if (ANY) {
    // the postponed leaf and, when the next reference is a leaf as well, that one too, tested
    // across the wave (straight-line code: no lane may leave before the cross-lane reads)
    const bool second = s.leaf != kEmptyRef && is_leaf(s.ref);
    const int32_t leaf_b = second ? s.ref : kEmptyRef;
    if (second) s.ref = trav_pop(s, st);
    const bool hit = leaves_any_wave<COUNT, PER_LANE_BVH>(B, r, tmin, skip, s.leaf, leaf_b, counts);
    s.leaf = kEmptyRef;
    if (hit) h.id = 0;  // any-hit queries report only that something was hit
    return hit || capped || s.ref == kEmptyRef;
  }
  while (s.leaf != kEmptyRef) {
    const uint32_t v = ~(uint32_t)s.leaf;
    const int32_t first = (int32_t)(v >> 4), cnt = (int32_t)(v & 15u);
    for (int32_t i = first; i < first + cnt; ++i) {
      // the whole 48-byte record in three 16-byte loads; the triangle the ray leaves from is
      // tested like the others and its hit ignored, so that no branch on the id has to wait
      // for a load of its own before the vertices are fetched
      const float4* q = reinterpret_cast<const float4*>(B.tris + i);
      const float4 q0 = q[0], q1 = q[1], q2 = q[2];
      BvhTri T;
      T.v0[0] = q0.x; T.v0[1] = q0.y; T.v0[2] = q0.z;
      T.v1[0] = q0.w; T.v1[1] = q1.x; T.v1[2] = q1.y;
      T.v2[0] = q1.z; T.v2[1] = q1.w; T.v2[2] = q2.x;
      T.id = __float_as_int(q2.y);
      if (COUNT) counts->tris++;
      float t, b1, b2;
      if (tri_hit(r, T, tmin, h.t, &t, &b1, &b2) && T.id != skip) {
        if (t < h.t || (t == h.t && T.id < h.id)) {
          h.id = T.id;
          h.t = t;
          h.b1 = b1;
          h.b2 = b2;
        }
      }
    }
    s.leaf = kEmptyRef;
    if (is_leaf(s.ref)) {
      s.leaf = s.ref;
      s.ref = trav_pop(s, st);
    }
  }
  return capped || s.ref == kEmptyRef;
}

}  // namespace exm
