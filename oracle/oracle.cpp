// FP64 CPU oracle of the Stage-II UV-PBR render pass.
//
// TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the CPU-baseline leg
// of the benchmark, never by the product path. It shares no code with the HIP library.
//
// Plain and slow on purpose: one pixel at a time, the steps in the order the paper gives them,
// double precision throughout. The estimator is templated on the scalar type so the same code
// yields values (T = double) and forward-mode derivatives (T = Dual: value + tangent), which
// serve as the reference gradient (a JVP) for the hand-written adjoint of the HIP path.
//
// Readings of points the paper leaves open (all shared with the HIP path by specification only):
//  * Projection/snap: clip = MVP [p,1] in FP64 without FMA; pixel x = ((x/w)+1)/2 W,
//    y = (1-(y/w))/2 H (y down), z01 = ((z/w)+1)/2; rint to 1/256 pixel; a triangle with a
//    vertex at w <= 0, outside a +-2^30 sub-pixel guard band, or non-finite, is dropped.
//  * Coverage: one sample at the pixel centre, integer edge functions, top-left fill rule in
//    y-down space, both windings rasterised, zero-area triangles never cover.
//  * Visibility: minimum of (float bits of the FP64-interpolated z01) << 32 | triangle id.
//  * D = GGX with sin^2 theta_h = |n x h|^2, G = separable Smith-GGX, F = Schlick, alpha = r^2,
//    alpha^2 >= 1e-12, F_dielectric = 0.04, epsilon = 1e-6.
//  * Env sampling: Rec.709 luminance times exact texel solid angle, quantised to integers
//    q = max(1, floor(w / w_max * 2^20)); integer CDF inversion; uniform in solid angle inside
//    the texel; nearest-texel E; pdf = q / (Q Omega).
//  * RNG: Philox4x32-10 keyed by (seed_lo ^ seed_hi, iteration_lo), counter
//    (pixel, view, sample, stream); stream 0 direct, 1 secondary direction, 2+j light samples
//    of secondary ray j.
//  * Secondary rays: cosine-weighted about n_g (Malley's method, Duff et al. basis); a hit is
//    valid iff it is front facing; shadow and secondary rays start at t >= t_min and skip the
//    triangle they leave from.
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------------------------------------
// dual numbers: value + tangent (forward-mode derivative)
// ------------------------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double x) : v(x), d(0) {}
  Dual(double x, double t) : v(x), d(t) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return {s, s > 0 ? a.d / (2 * s) : 0.0};
}
inline double sqrt(double a) { return std::sqrt(a); }
inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }
template <class T> inline T max0(T x) { return val(x) > 0 ? x : T(0.0); }

template <class T> struct V3 {
  T x, y, z;
};
template <class T> inline V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> inline V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T, class S> inline V3<T> mul(S s, V3<T> a) { return {T(s) * a.x, T(s) * a.y, T(s) * a.z}; }
template <class T> inline T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> inline V3<T> cross(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> inline V3<T> lift(V3<double> a) { return {T(a.x), T(a.y), T(a.z)}; }
using D3 = V3<double>;
inline double norm(D3 a) { return std::sqrt(dot(a, a)); }
inline D3 normalize(D3 a) { double n = norm(a); return {a.x / n, a.y / n, a.z / n}; }

inline D3 vtx(const ora_mesh* m, int32_t i) {
  return {(double)m->pos[3 * i], (double)m->pos[3 * i + 1], (double)m->pos[3 * i + 2]};
}

// ------------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64 products
// with xor of the key, the key advanced by the two Weyl constants between rounds.
// ------------------------------------------------------------------------------------------
void philox(const uint32_t in[4], const uint32_t k_in[2], uint32_t out[4]) {
  uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
  uint32_t k0 = k_in[0], k1 = k_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

struct Draw {
  uint64_t x;    // 64-bit selection word
  double u2, u3; // uniforms in [0,1)
};

Draw draw(const ora_params* p, uint32_t pixel, uint32_t view, uint32_t sample, uint32_t stream) {
  uint32_t key[2] = {(uint32_t)p->seed ^ (uint32_t)(p->seed >> 32), (uint32_t)p->iteration};
  uint32_t ctr[4] = {pixel, view, sample, stream};
  uint32_t o[4];
  philox(ctr, key, o);
  Draw d;
  d.x = ((uint64_t)o[0] << 32) | o[1];
  d.u2 = (double)(o[2] >> 8) * (1.0 / 16777216.0);
  d.u3 = (double)(o[3] >> 8) * (1.0 / 16777216.0);
  return d;
}

// ------------------------------------------------------------------------------------------
// projection and coverage
// ------------------------------------------------------------------------------------------
struct Proj {
  bool ok;
  int64_t X[3], Y[3];
  double z01[3], w[3];
};

Proj project(const ora_mesh* m, const ora_camera* c, int32_t f) {
  Proj P;
  P.ok = true;
  const double lim = 1073741824.0;  // 2^30 sub-pixel guard band
  for (int k = 0; k < 3; ++k) {
    D3 p = vtx(m, m->tri[3 * f + k]);
    const double* M = c->mvp;
    double cx = ((M[0] * p.x + M[1] * p.y) + M[2] * p.z) + M[3];
    double cy = ((M[4] * p.x + M[5] * p.y) + M[6] * p.z) + M[7];
    double cz = ((M[8] * p.x + M[9] * p.y) + M[10] * p.z) + M[11];
    double cw = ((M[12] * p.x + M[13] * p.y) + M[14] * p.z) + M[15];
    if (!(cw > 0.0)) { P.ok = false; return P; }
    double xp = (((cx / cw) + 1.0) * 0.5) * (double)c->W;
    double yp = ((1.0 - (cy / cw)) * 0.5) * (double)c->H;
    double zz = ((cz / cw) + 1.0) * 0.5;
    double xs = xp * 256.0, ys = yp * 256.0;
    if (!(std::fabs(xs) <= lim && std::fabs(ys) <= lim) || !std::isfinite(zz)) { P.ok = false; return P; }
    P.X[k] = (int64_t)std::nearbyint(xs);
    P.Y[k] = (int64_t)std::nearbyint(ys);
    P.z01[k] = zz;
    P.w[k] = cw;
  }
  return P;
}

// Edge functions at sample point (Px,Py) in sub-pixel units. Returns false if the sample is
// not covered; otherwise E[k] (original vertex labels) and A2 > 0.
bool cover(const Proj& P, int64_t Px, int64_t Py, int64_t E[3], int64_t* A2out) {
  int64_t A2 = (P.X[1] - P.X[0]) * (P.Y[2] - P.Y[0]) - (P.X[2] - P.X[0]) * (P.Y[1] - P.Y[0]);
  if (A2 == 0) return false;
  int idx[3] = {0, 1, 2};
  if (A2 < 0) { idx[1] = 2; idx[2] = 1; A2 = -A2; }
  for (int s = 0; s < 3; ++s) {
    int ia = idx[(s + 1) % 3], ib = idx[(s + 2) % 3];
    int64_t dx = P.X[ib] - P.X[ia], dy = P.Y[ib] - P.Y[ia];
    int64_t e = dx * (Py - P.Y[ia]) - dy * (Px - P.X[ia]);
    bool in = e > 0 || (e == 0 && (dy < 0 || (dy == 0 && dx > 0)));
    if (!in) return false;
    E[idx[s]] = e;
  }
  *A2out = A2;
  return true;
}

void pixel_range(const Proj& P, int32_t W, int32_t H, int32_t* x0, int32_t* x1, int32_t* y0, int32_t* y1) {
  int64_t xmin = std::min({P.X[0], P.X[1], P.X[2]}), xmax = std::max({P.X[0], P.X[1], P.X[2]});
  int64_t ymin = std::min({P.Y[0], P.Y[1], P.Y[2]}), ymax = std::max({P.Y[0], P.Y[1], P.Y[2]});
  // pixel px has its sample at 256 px + 128
  auto lo = [](int64_t v) { return (int64_t)std::ceil((double)(v - 128) / 256.0); };
  auto hi = [](int64_t v) { return (int64_t)std::floor((double)(v - 128) / 256.0); };
  *x0 = (int32_t)std::max<int64_t>(0, lo(xmin));
  *x1 = (int32_t)std::min<int64_t>(W - 1, hi(xmax));
  *y0 = (int32_t)std::max<int64_t>(0, lo(ymin));
  *y1 = (int32_t)std::min<int64_t>(H - 1, hi(ymax));
}

// ------------------------------------------------------------------------------------------
// BVH: object-median split on the longest centroid axis, leaves of <= 4 triangles
// ------------------------------------------------------------------------------------------
struct Box {
  double lo[3], hi[3];
};
struct BNode {
  Box b;
  int32_t left, right;  // children (internal) or -1
  int32_t first, count; // leaf range in `order`
};

}  // namespace

struct ora_bvh {
  std::vector<BNode> nodes;
  std::vector<int32_t> order;
};

namespace {

Box tri_box(const ora_mesh* m, int32_t f) {
  Box b;
  for (int a = 0; a < 3; ++a) { b.lo[a] = 1e300; b.hi[a] = -1e300; }
  for (int k = 0; k < 3; ++k) {
    D3 p = vtx(m, m->tri[3 * f + k]);
    double c[3] = {p.x, p.y, p.z};
    for (int a = 0; a < 3; ++a) { b.lo[a] = std::min(b.lo[a], c[a]); b.hi[a] = std::max(b.hi[a], c[a]); }
  }
  return b;
}

int32_t build_rec(ora_bvh* B, const ora_mesh* m, const std::vector<D3>& cen, int32_t first, int32_t count) {
  BNode nd;
  for (int a = 0; a < 3; ++a) { nd.b.lo[a] = 1e300; nd.b.hi[a] = -1e300; }
  double clo[3] = {1e300, 1e300, 1e300}, chi[3] = {-1e300, -1e300, -1e300};
  for (int32_t i = first; i < first + count; ++i) {
    Box tb = tri_box(m, B->order[i]);
    D3 c = cen[B->order[i]];
    double cc[3] = {c.x, c.y, c.z};
    for (int a = 0; a < 3; ++a) {
      nd.b.lo[a] = std::min(nd.b.lo[a], tb.lo[a]); nd.b.hi[a] = std::max(nd.b.hi[a], tb.hi[a]);
      clo[a] = std::min(clo[a], cc[a]); chi[a] = std::max(chi[a], cc[a]);
    }
  }
  int32_t id = (int32_t)B->nodes.size();
  nd.left = nd.right = -1; nd.first = first; nd.count = count;
  B->nodes.push_back(nd);
  if (count <= 4) return id;
  int axis = 0;
  for (int a = 1; a < 3; ++a) if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
  int32_t mid = first + count / 2;
  auto key = [&](int32_t f) { D3 c = cen[f]; return axis == 0 ? c.x : axis == 1 ? c.y : c.z; };
  std::nth_element(B->order.begin() + first, B->order.begin() + mid, B->order.begin() + first + count,
                   [&](int32_t a, int32_t b) { double ka = key(a), kb = key(b); return ka < kb || (ka == kb && a < b); });
  int32_t l = build_rec(B, m, cen, first, mid - first);
  int32_t r = build_rec(B, m, cen, mid, first + count - mid);
  B->nodes[id].left = l; B->nodes[id].right = r; B->nodes[id].count = 0;
  return id;
}

// slab test against a box, returns entry t or +inf
double box_hit(const Box& b, D3 o, D3 inv, double tmax) {
  double t0 = 0.0, t1 = tmax;
  double oo[3] = {o.x, o.y, o.z}, iv[3] = {inv.x, inv.y, inv.z};
  for (int a = 0; a < 3; ++a) {
    double ta = (b.lo[a] - oo[a]) * iv[a], tb = (b.hi[a] - oo[a]) * iv[a];
    if (std::isnan(ta) || std::isnan(tb)) { // direction component 0 with origin on a slab face
      if (oo[a] < b.lo[a] || oo[a] > b.hi[a]) return INFINITY;
      continue;
    }
    if (ta > tb) std::swap(ta, tb);
    t0 = std::max(t0, ta); t1 = std::min(t1, tb);
    if (t0 > t1 * (1.0 + 1e-12) + 1e-300) return INFINITY;
  }
  return t0;
}

// Moller-Trumbore in FP64, both windings; returns t (or -1 on miss) and b1, b2
double tri_hit(const ora_mesh* m, int32_t f, D3 o, D3 d, double* b1, double* b2) {
  D3 p0 = vtx(m, m->tri[3 * f]), p1 = vtx(m, m->tri[3 * f + 1]), p2 = vtx(m, m->tri[3 * f + 2]);
  D3 e1 = p1 - p0, e2 = p2 - p0;
  D3 pv = cross(d, e2);
  double det = dot(e1, pv);
  if (det == 0.0) return -1.0;
  double inv = 1.0 / det;
  D3 tv = o - p0;
  double u = dot(tv, pv) * inv;
  if (u < 0.0 || u > 1.0) return -1.0;
  D3 qv = cross(tv, e1);
  double v = dot(d, qv) * inv;
  if (v < 0.0 || u + v > 1.0) return -1.0;
  *b1 = u; *b2 = v;
  return dot(e2, qv) * inv;
}

struct Hit {
  int32_t id;
  double t, b1, b2;
};

Hit closest(const ora_mesh* m, const ora_bvh* B, D3 o, D3 d, double tmin, int32_t skip) {
  Hit h{-1, INFINITY, 0, 0};
  auto test = [&](int32_t f) {
    if (f == skip) return;
    double b1, b2, t = tri_hit(m, f, o, d, &b1, &b2);
    if (t >= tmin && (t < h.t || (t == h.t && f < h.id))) { h = {f, t, b1, b2}; }
  };
  if (!B) {
    for (int32_t f = 0; f < m->nF; ++f) test(f);
    return h;
  }
  D3 inv = {1.0 / d.x, 1.0 / d.y, 1.0 / d.z};
  int32_t stack[128];
  int sp = 0;
  stack[sp++] = 0;
  while (sp) {
    const BNode& n = B->nodes[stack[--sp]];
    if (box_hit(n.b, o, inv, h.t) == INFINITY) continue;
    if (n.left < 0) {
      for (int32_t i = n.first; i < n.first + n.count; ++i) test(B->order[i]);
    } else {
      stack[sp++] = n.left;
      stack[sp++] = n.right;
    }
  }
  return h;
}

bool any_hit(const ora_mesh* m, const ora_bvh* B, D3 o, D3 d, double tmin, int32_t skip) {
  auto test = [&](int32_t f) {
    if (f == skip) return false;
    double b1, b2, t = tri_hit(m, f, o, d, &b1, &b2);
    return t >= tmin;
  };
  if (!B) {
    for (int32_t f = 0; f < m->nF; ++f) if (test(f)) return true;
    return false;
  }
  D3 inv = {1.0 / d.x, 1.0 / d.y, 1.0 / d.z};
  int32_t stack[128];
  int sp = 0;
  stack[sp++] = 0;
  while (sp) {
    const BNode& n = B->nodes[stack[--sp]];
    if (box_hit(n.b, o, inv, INFINITY) == INFINITY) continue;
    if (n.left < 0) {
      for (int32_t i = n.first; i < n.first + n.count; ++i) if (test(B->order[i])) return true;
    } else {
      stack[sp++] = n.left;
      stack[sp++] = n.right;
    }
  }
  return false;
}

// ------------------------------------------------------------------------------------------
// attribute query (Attribute Query, Eq. 10-11)
// ------------------------------------------------------------------------------------------
struct MeshAttr {
  std::vector<double> vnrm;  // [nV,3]
  std::vector<double> ftan;  // [nF,4]
};

void vertex_normals(const ora_mesh* m, double* out) {
  std::fill(out, out + 3 * (size_t)m->nV, 0.0);
  for (int32_t f = 0; f < m->nF; ++f) {
    D3 p0 = vtx(m, m->tri[3 * f]), p1 = vtx(m, m->tri[3 * f + 1]), p2 = vtx(m, m->tri[3 * f + 2]);
    D3 n = cross(p1 - p0, p2 - p0);  // area-weighted face normal
    for (int k = 0; k < 3; ++k) {
      int32_t v = m->tri[3 * f + k];
      out[3 * v] += n.x; out[3 * v + 1] += n.y; out[3 * v + 2] += n.z;
    }
  }
  for (int32_t v = 0; v < m->nV; ++v) {
    D3 n = {out[3 * v], out[3 * v + 1], out[3 * v + 2]};
    double l = norm(n);
    if (l > 0) { out[3 * v] = n.x / l; out[3 * v + 1] = n.y / l; out[3 * v + 2] = n.z / l; }
  }
}

// Per-face tangent from UV derivatives, handedness sign(((e1 x e2) x T) . B), 0 -> +1.
// A face with |det| < 1e-20 gets T = 0 (the shading normal then falls back to n_g).
void face_tangents(const ora_mesh* m, double* out) {
  for (int32_t f = 0; f < m->nF; ++f) {
    D3 p0 = vtx(m, m->tri[3 * f]), p1 = vtx(m, m->tri[3 * f + 1]), p2 = vtx(m, m->tri[3 * f + 2]);
    const float* u0 = m->uv + 2 * m->tri_uv[3 * f];
    const float* u1 = m->uv + 2 * m->tri_uv[3 * f + 1];
    const float* u2 = m->uv + 2 * m->tri_uv[3 * f + 2];
    D3 e1 = p1 - p0, e2 = p2 - p0;
    double d1x = (double)u1[0] - u0[0], d1y = (double)u1[1] - u0[1];
    double d2x = (double)u2[0] - u0[0], d2y = (double)u2[1] - u0[1];
    double det = d1x * d2y - d2x * d1y;
    double* o = out + 4 * (size_t)f;
    if (std::fabs(det) < 1e-20) { o[0] = o[1] = o[2] = 0; o[3] = 1; continue; }
    D3 T = mul(1.0 / det, mul(d2y, e1) - mul(d1y, e2));
    D3 Bv = mul(1.0 / det, mul(d1x, e2) - mul(d2x, e1));
    double s = dot(cross(cross(e1, e2), T), Bv);
    o[0] = T.x; o[1] = T.y; o[2] = T.z; o[3] = s < 0 ? -1.0 : 1.0;
  }
}

struct Scene {
  const ora_mesh* m;
  const ora_bvh* bvh;
  const ora_params_theta* th;
  const ora_tables* tab;
  const ora_params* p;
  MeshAttr attr;
};

// bilinear tap indices/weights: s = u Wt - 0.5, t = v Ht - 0.5, clamp-to-edge taps
struct Taps {
  int64_t idx[4];
  double w[4];
};
Taps bilinear_taps(int32_t Ht, int32_t Wt, double u, double v) {
  u = std::min(1.0, std::max(0.0, u));
  v = std::min(1.0, std::max(0.0, v));
  double s = u * Wt - 0.5, t = v * Ht - 0.5;
  double fs0 = std::floor(s), ft0 = std::floor(t);
  double fs = s - fs0, ft = t - ft0;
  int64_t i0 = (int64_t)fs0, j0 = (int64_t)ft0;
  Taps T;
  int k = 0;
  for (int dj = 0; dj < 2; ++dj)
    for (int di = 0; di < 2; ++di) {
      int64_t i = std::min<int64_t>(Wt - 1, std::max<int64_t>(0, i0 + di));
      int64_t j = std::min<int64_t>(Ht - 1, std::max<int64_t>(0, j0 + dj));
      T.idx[k] = j * Wt + i;
      T.w[k] = (di ? fs : 1.0 - fs) * (dj ? ft : 1.0 - ft);
      ++k;
    }
  return T;
}

template <class T> T tex_chan(const ora_params_theta* th, int64_t texel, int c) {
  size_t i = (size_t)texel * 8 + c;
  return T(th->tex[i], th->tex_dot ? th->tex_dot[i] : 0.0);
}
template <> double tex_chan<double>(const ora_params_theta* th, int64_t texel, int c) {
  return th->tex[(size_t)texel * 8 + c];
}
template <class T> T env_chan(const ora_params_theta* th, int64_t texel, int c) {
  size_t i = (size_t)texel * 3 + c;
  return T(th->env[i], th->env_dot ? th->env_dot[i] : 0.0);
}
template <> double env_chan<double>(const ora_params_theta* th, int64_t texel, int c) {
  return th->env[(size_t)texel * 3 + c];
}

template <class T> struct Attr {
  D3 x, ng;
  V3<T> ns;
  T a[3], r, m;
};

// surface point of face f at barycentrics b: position, n_g, uv, bilinear material, n_s
template <class T> Attr<T> query(const Scene& S, int32_t f, const double b[3]) {
  const ora_mesh* m = S.m;
  Attr<T> A;
  D3 P[3], N[3];
  double u = 0, v = 0;
  for (int k = 0; k < 3; ++k) {
    int32_t vi = m->tri[3 * f + k];
    P[k] = vtx(m, vi);
    N[k] = {S.attr.vnrm[3 * vi], S.attr.vnrm[3 * vi + 1], S.attr.vnrm[3 * vi + 2]};
  }
  A.x = (mul(b[0], P[0]) + mul(b[1], P[1])) + mul(b[2], P[2]);
  A.ng = normalize((mul(b[0], N[0]) + mul(b[1], N[1])) + mul(b[2], N[2]));
  for (int k = 0; k < 3; ++k) {
    const float* uvk = m->uv + 2 * m->tri_uv[3 * f + k];
    u += b[k] * (double)uvk[0];
    v += b[k] * (double)uvk[1];
  }
  const ora_params_theta* th = S.th;
  Taps tp = bilinear_taps(th->Ht, th->Wt, u, v);
  T ch[8];
  for (int c = 0; c < 8; ++c) {
    ch[c] = T(0.0);
    for (int k = 0; k < 4; ++k) ch[c] = ch[c] + T(tp.w[k]) * tex_chan<T>(th, tp.idx[k], c);
  }
  A.a[0] = ch[0]; A.a[1] = ch[1]; A.a[2] = ch[2];
  A.r = ch[3];
  A.m = (S.p->flags & ORA_METALLIC_OFF) ? T(0.0) : ch[4];
  // tangent frame of the face, Gram-Schmidt against n_g
  const double* ft = &S.attr.ftan[4 * (size_t)f];
  D3 Tf = {ft[0], ft[1], ft[2]};
  D3 Tp = Tf - mul(dot(A.ng, Tf), A.ng);
  double lt = norm(Tp);
  if (!(lt >= 1e-12)) { A.ns = lift<T>(A.ng); return A; }
  Tp = mul(1.0 / lt, Tp);
  D3 Bp = mul(ft[3], cross(A.ng, Tp));
  V3<T> vv = (mul(ch[5], lift<T>(Tp)) + mul(ch[6], lift<T>(Bp))) + mul(ch[7], lift<T>(A.ng));
  T ln = sqrt(dot(vv, vv));
  if (!(val(ln) >= 1e-12)) { A.ns = lift<T>(A.ng); return A; }
  A.ns = {vv.x / ln, vv.y / ln, vv.z / ln};
  return A;
}

// ------------------------------------------------------------------------------------------
// BRDF (Eq. 13-16)
// ------------------------------------------------------------------------------------------
template <class T> T ggx_D(T alpha2, T ch, T sh2) {
  T d = sh2 + alpha2 * ch * ch;
  return alpha2 / (T(kPi) * d * d);
}
template <class T> T smith_G1(T alpha2, T c) {
  return T(2.0) * c / (c + sqrt(alpha2 + (T(1.0) - alpha2) * c * c));
}

// f_r for one (wi, wo); writes 3 channels
template <class T>
void brdf(const T a[3], T r, T m, V3<T> n, D3 wi, D3 wo, double f_diel, double eps, uint32_t flags, T out[3]) {
  T fd[3], fs[3];
  for (int c = 0; c < 3; ++c) { fd[c] = (T(1.0) - m) * a[c] / T(kPi); fs[c] = T(0.0); }
  D3 hs = wi + wo;
  double hl = norm(hs);
  T ci = max0(dot(n, lift<T>(wi)));
  T co = max0(dot(n, lift<T>(wo)));
  if (hl >= 1e-12 && val(co) > 0 && val(ci) > 0) {
    D3 h = mul(1.0 / hl, hs);
    T alpha = r * r;
    T alpha2 = alpha * alpha;
    if (val(alpha2) < 1e-12) alpha2 = T(1e-12);
    V3<T> hT = lift<T>(h);
    T chh = dot(n, hT);
    V3<T> nx = cross(n, hT);
    T sh2 = dot(nx, nx);
    T D = ggx_D(alpha2, chh, sh2);
    T G = smith_G1(alpha2, ci) * smith_G1(alpha2, co);
    double x = 1.0 - std::max(dot(wi, h), 0.0);
    double x5 = x * x * x * x * x;
    T den = T(4.0) * ci * co + T(eps);
    for (int c = 0; c < 3; ++c) {
      T F0 = (T(1.0) - m) * T(f_diel) + m * a[c];
      T F = F0 + (T(1.0) - F0) * T(x5);
      fs[c] = D * G * F / den;
    }
  }
  for (int c = 0; c < 3; ++c) {
    T d = (flags & ORA_SPECULAR_ONLY) ? T(0.0) : fd[c];
    T s = (flags & ORA_DIFFUSE_ONLY) ? T(0.0) : fs[c];
    out[c] = d + s;
  }
}

// ------------------------------------------------------------------------------------------
// env importance sampling (Direct Illumination)
// ------------------------------------------------------------------------------------------
struct EnvSample {
  int64_t texel;
  D3 dir;
  double pdf;
};

EnvSample env_sample(const ora_tables* t, uint64_t x, double u2, double u3) {
  unsigned __int128 prod = (unsigned __int128)x * t->Q;
  uint64_t target = (uint64_t)(prod >> 64);
  const uint64_t* cr = t->cdf_row;
  int32_t row = (int32_t)(std::upper_bound(cr, cr + t->He, target) - cr);
  uint64_t rem = target - (row > 0 ? cr[row - 1] : 0);
  const uint64_t* cc = t->cdf_col + (size_t)row * t->We;
  int32_t col = (int32_t)(std::upper_bound(cc, cc + t->We, rem) - cc);
  double ci = std::cos(row * kPi / t->He), ci1 = std::cos((row + 1) * kPi / t->He);
  double phi = 2.0 * kPi * (col + u2) / t->We;
  double ct = ci - u3 * (ci - ci1);
  double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
  EnvSample s;
  s.texel = (int64_t)row * t->We + col;
  s.dir = {st * std::cos(phi), ct, st * std::sin(phi)};
  double omega = 2.0 * kPi / t->We * (ci - ci1);
  s.pdf = (double)t->q[s.texel] / ((double)t->Q * omega);
  return s;
}

// Duff et al. 2017 orthonormal basis around unit n
void onb(D3 n, D3* b1, D3* b2) {
  double sign = std::copysign(1.0, n.z);
  double a = -1.0 / (sign + n.z);
  double b = n.x * n.y * a;
  *b1 = {1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x};
  *b2 = {b, sign + n.y * n.y * a, -n.y};
}

// ------------------------------------------------------------------------------------------
// per-pixel estimator (Eq. 17 direct, Eq. 18-19 indirect)
// ------------------------------------------------------------------------------------------
template <class T>
void shade_pixel(const Scene& S, const ora_camera* cam, uint32_t pixel, int32_t f, const double b[3],
                 T Ldir[3], T Lind[3], uint64_t* vis, int32_t* sec_tri, double* sec_bary,
                 uint64_t* sec_vis, int32_t* n_shadow) {
  const ora_params* p = S.p;
  const ora_params_theta* th = S.th;
  Attr<T> A = query<T>(S, f, b);
  D3 wo = normalize(D3{cam->eye[0], cam->eye[1], cam->eye[2]} - A.x);
  for (int c = 0; c < 3; ++c) { Ldir[c] = T(0.0); Lind[c] = T(0.0); }
  *vis = 0;
  *n_shadow = 0;
  uint32_t view = (uint32_t)cam->view_id;
  // direct: N_d env samples
  for (int k = 0; k < p->N_d; ++k) {
    Draw dr = draw(p, pixel, view, (uint32_t)k, 0u);
    EnvSample es = env_sample(S.tab, dr.x, dr.u2, dr.u3);
    T c = dot(A.ns, lift<T>(es.dir));
    if (!(val(c) > 0)) continue;
    bool V = true;
    if (!(p->flags & ORA_NO_VIS)) {
      ++*n_shadow;
      V = !any_hit(S.m, S.bvh, A.x, es.dir, p->tmin, f);
    }
    if (!V) continue;
    *vis |= (uint64_t)1 << k;
    T fr[3];
    brdf<T>(A.a, A.r, A.m, A.ns, es.dir, wo, p->f_diel, p->eps, p->flags, fr);
    for (int ch = 0; ch < 3; ++ch)
      Ldir[ch] = Ldir[ch] + env_chan<T>(th, es.texel, ch) * fr[ch] * c / T(es.pdf);
  }
  if (p->N_d > 0)
    for (int ch = 0; ch < 3; ++ch) Ldir[ch] = Ldir[ch] / T((double)p->N_d);
  // indirect: N_b cosine-weighted secondary rays about n_g, N_s light samples per valid hit
  *sec_vis = 0;
  if (p->N_b <= 0) return;
  T fdx[3];
  for (int ch = 0; ch < 3; ++ch)
    fdx[ch] = (p->flags & ORA_SPECULAR_ONLY) ? T(0.0) : (T(1.0) - A.m) * A.a[ch] / T(kPi);
  D3 b1, b2;
  onb(A.ng, &b1, &b2);
  for (int j = 0; j < p->N_b; ++j) {
    sec_tri[j] = -1;
    sec_bary[2 * j] = sec_bary[2 * j + 1] = 0.0;
    Draw dr = draw(p, pixel, view, (uint32_t)j, 1u);
    double rr = std::sqrt(dr.u2), phi = 2.0 * kPi * dr.u3;
    double lz = std::sqrt(std::max(0.0, 1.0 - dr.u2));
    D3 w = (mul(rr * std::cos(phi), b1) + mul(rr * std::sin(phi), b2)) + mul(lz, A.ng);
    double pb = std::max(dot(A.ng, w), 0.0) / kPi;
    Hit h = closest(S.m, S.bvh, A.x, w, p->tmin, f);
    if (h.id < 0) continue;
    D3 q0 = vtx(S.m, S.m->tri[3 * h.id]), q1 = vtx(S.m, S.m->tri[3 * h.id + 1]), q2 = vtx(S.m, S.m->tri[3 * h.id + 2]);
    if (!(dot(w, cross(q1 - q0, q2 - q0)) < 0.0)) continue;  // back face: invalid
    sec_tri[j] = h.id;
    sec_bary[2 * j] = h.b1;
    sec_bary[2 * j + 1] = h.b2;
    double by[3] = {1.0 - h.b1 - h.b2, h.b1, h.b2};
    Attr<T> Y = query<T>(S, h.id, by);
    if (p->flags & ORA_NO_SECONDARY_MATERIAL) {  // the material at y is not queried
      for (int ch = 0; ch < 3; ++ch) Y.a[ch] = T(ORA_SECONDARY_ALBEDO);
      Y.m = T(0.0);
      Y.ns = lift<T>(Y.ng);
    }
    T fdy[3];
    for (int ch = 0; ch < 3; ++ch)
      fdy[ch] = (p->flags & ORA_SPECULAR_ONLY) ? T(0.0) : (T(1.0) - Y.m) * Y.a[ch] / T(kPi);
    T Lsec[3] = {T(0.0), T(0.0), T(0.0)};
    for (int s = 0; s < p->N_s; ++s) {
      Draw ds = draw(p, pixel, view, (uint32_t)s, (uint32_t)(2 + j));
      EnvSample es = env_sample(S.tab, ds.x, ds.u2, ds.u3);
      T c = dot(Y.ns, lift<T>(es.dir));
      if (!(val(c) > 0)) continue;
      bool V = true;
      if (!(p->flags & ORA_NO_VIS)) V = !any_hit(S.m, S.bvh, Y.x, es.dir, p->tmin, h.id);
      if (!V) continue;
      *sec_vis |= (uint64_t)1 << (j * p->N_s + s);
      for (int ch = 0; ch < 3; ++ch)
        Lsec[ch] = Lsec[ch] + env_chan<T>(th, es.texel, ch) * fdy[ch] * c / T(es.pdf);
    }
    T cx = max0(dot(A.ns, lift<T>(w)));
    for (int ch = 0; ch < 3; ++ch) {
      // Eq. 18's average over the N_s light samples; with none (N_s = 0) the empty estimator is zero,
      // as Eq. 17's is above for N_d = 0
      T ls = p->N_s > 0 ? Lsec[ch] / T((double)p->N_s) : T(0.0);
      Lind[ch] = Lind[ch] + fdx[ch] * ls * cx / T(pb);
    }
  }
  for (int ch = 0; ch < 3; ++ch) Lind[ch] = Lind[ch] / T((double)p->N_b);
}

}  // namespace

// ==========================================================================================
// C API
// ==========================================================================================
extern "C" {

void ora_vertex_normals(const ora_mesh* m, double* vnrm) { vertex_normals(m, vnrm); }
void ora_face_tangents(const ora_mesh* m, double* ftan) { face_tangents(m, ftan); }

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) { philox(ctr, key, out); }

void ora_raster(const ora_mesh* m, const ora_camera* cam, int32_t* tri_id, double* bary) {
  const int32_t H = cam->H, W = cam->W;
  std::vector<uint64_t> key((size_t)H * W, ~(uint64_t)0);
  for (int32_t f = 0; f < m->nF; ++f) {
    Proj P = project(m, cam, f);
    if (!P.ok) continue;
    int32_t x0, x1, y0, y1;
    pixel_range(P, W, H, &x0, &x1, &y0, &y1);
    for (int32_t py = y0; py <= y1; ++py)
      for (int32_t px = x0; px <= x1; ++px) {
        int64_t E[3], A2;
        if (!cover(P, 256 * (int64_t)px + 128, 256 * (int64_t)py + 128, E, &A2)) continue;
        double z = (((double)E[0] * P.z01[0] + (double)E[1] * P.z01[1]) + (double)E[2] * P.z01[2]) / (double)A2;
        if (!(z >= 0.0 && z <= 1.0)) continue;
        float zf = (float)z;
        if (zf == 0.0f) zf = 0.0f;
        uint32_t zb;
        std::memcpy(&zb, &zf, 4);
        uint64_t k = ((uint64_t)zb << 32) | (uint32_t)f;
        uint64_t& slot = key[(size_t)py * W + px];
        if (k < slot) slot = k;
      }
  }
  for (size_t i = 0; i < (size_t)H * W; ++i) {
    int32_t f = key[i] == ~(uint64_t)0 ? -1 : (int32_t)(uint32_t)key[i];
    tri_id[i] = f;
    bary[3 * i] = bary[3 * i + 1] = bary[3 * i + 2] = 0.0;
    if (f < 0) continue;
    Proj P = project(m, cam, f);
    int64_t px = (int64_t)(i % W), py = (int64_t)(i / W);
    int64_t E[3], A2;
    cover(P, 256 * px + 128, 256 * py + 128, E, &A2);
    double q[3], s = 0;
    for (int k = 0; k < 3; ++k) { q[k] = (double)E[k] / P.w[k]; s += q[k]; }
    for (int k = 0; k < 3; ++k) bary[3 * i + k] = q[k] / s;
  }
}

void ora_coverage_count(const ora_mesh* m, const ora_camera* cam, int32_t* count) {
  const int32_t H = cam->H, W = cam->W;
  std::fill(count, count + (size_t)H * W, 0);
  for (int32_t f = 0; f < m->nF; ++f) {
    Proj P = project(m, cam, f);
    if (!P.ok) continue;
    int32_t x0, x1, y0, y1;
    pixel_range(P, W, H, &x0, &x1, &y0, &y1);
    for (int32_t py = y0; py <= y1; ++py)
      for (int32_t px = x0; px <= x1; ++px) {
        int64_t E[3], A2;
        if (cover(P, 256 * (int64_t)px + 128, 256 * (int64_t)py + 128, E, &A2)) count[(size_t)py * W + px]++;
      }
  }
}

void ora_env_tables(int32_t He, int32_t We, const float* env, uint64_t* q, uint64_t* cdf_row,
                    uint64_t* cdf_col, double* pdf, uint64_t* Qout, double* wout) {
  std::vector<double> w((size_t)He * We);
  double wmax = 0.0;
  for (int32_t i = 0; i < He; ++i) {
    double omega = 2.0 * kPi / We * (std::cos(i * kPi / He) - std::cos((i + 1) * kPi / He));
    for (int32_t j = 0; j < We; ++j) {
      const float* e = env + 3 * ((size_t)i * We + j);
      double lum = (0.2126 * (double)e[0] + 0.7152 * (double)e[1]) + 0.0722 * (double)e[2];
      double wij = lum * omega;
      w[(size_t)i * We + j] = wij;
      wmax = std::max(wmax, wij);
    }
  }
  uint64_t Q = 0;
  for (int32_t i = 0; i < He; ++i) {
    uint64_t rs = 0;
    for (int32_t j = 0; j < We; ++j) {
      size_t t = (size_t)i * We + j;
      double s = wmax > 0 ? std::floor(w[t] / wmax * 1048576.0) : 0.0;
      uint64_t qq = s < 1.0 ? 1 : (uint64_t)s;
      q[t] = qq;
      rs += qq;
      cdf_col[t] = rs;
    }
    Q += rs;
    cdf_row[i] = Q;
  }
  for (int32_t i = 0; i < He; ++i) {
    double omega = 2.0 * kPi / We * (std::cos(i * kPi / He) - std::cos((i + 1) * kPi / He));
    for (int32_t j = 0; j < We; ++j) {
      size_t t = (size_t)i * We + j;
      pdf[t] = (double)q[t] / ((double)Q * omega);
    }
  }
  *Qout = Q;
  if (wout) std::copy(w.begin(), w.end(), wout);
}

void ora_env_sample(const ora_tables* t, uint64_t x, double u2, double u3, int32_t* row, int32_t* col,
                    double* dir, double* pdf) {
  EnvSample s = env_sample(t, x, u2, u3);
  *row = (int32_t)(s.texel / t->We);
  *col = (int32_t)(s.texel % t->We);
  dir[0] = s.dir.x; dir[1] = s.dir.y; dir[2] = s.dir.z;
  *pdf = s.pdf;
}

void ora_brdf(const double a[3], double r, double m, const double n[3], const double wi[3], const double wo[3],
              double f_diel, double eps, uint32_t flags, double out[3]) {
  double aa[3] = {a[0], a[1], a[2]};
  if (flags & ORA_METALLIC_OFF) m = 0.0;
  brdf<double>(aa, r, m, V3<double>{n[0], n[1], n[2]}, D3{wi[0], wi[1], wi[2]}, D3{wo[0], wo[1], wo[2]}, f_diel, eps,
               flags, out);
}

double ora_ggx_D(double r, const double n[3], const double h[3]) {
  double alpha = r * r, alpha2 = std::max(alpha * alpha, 1e-12);
  D3 nn{n[0], n[1], n[2]}, hh{h[0], h[1], h[2]};
  D3 c = cross(nn, hh);
  return ggx_D<double>(alpha2, dot(nn, hh), dot(c, c));
}

double ora_smith_G1(double r, double c) {
  double alpha = r * r, alpha2 = std::max(alpha * alpha, 1e-12);
  return smith_G1<double>(alpha2, std::max(c, 0.0));
}

void ora_bilinear(int32_t Ht, int32_t Wt, const double* tex, int32_t C, double u, double v, double* out) {
  Taps tp = bilinear_taps(Ht, Wt, u, v);
  for (int c = 0; c < C; ++c) {
    out[c] = 0.0;
    for (int k = 0; k < 4; ++k) out[c] += tp.w[k] * tex[(size_t)tp.idx[k] * C + c];
  }
}

void ora_shading_normal(const ora_mesh* m, const double* vnrm, const double* ftan, int32_t f, const double b[3],
                        const double q[3], double ng[3], double ns[3]) {
  // one-texel 1x1 map holding q; query through the same code path as the renderer
  double tex[8] = {0, 0, 0, 0.5, 0, q[0], q[1], q[2]};
  ora_params_theta th{1, 1, tex, nullptr, 1, 1, tex, nullptr};
  ora_params p{};
  Scene S{m, nullptr, &th, nullptr, &p, {}};
  S.attr.vnrm.assign(vnrm, vnrm + 3 * (size_t)m->nV);
  S.attr.ftan.assign(ftan, ftan + 4 * (size_t)m->nF);
  Attr<double> A = query<double>(S, f, b);
  ng[0] = A.ng.x; ng[1] = A.ng.y; ng[2] = A.ng.z;
  ns[0] = A.ns.x; ns[1] = A.ns.y; ns[2] = A.ns.z;
}

ora_bvh* ora_bvh_build(const ora_mesh* m) {
  ora_bvh* B = new ora_bvh;
  std::vector<D3> cen(m->nF);
  for (int32_t f = 0; f < m->nF; ++f) {
    D3 p0 = vtx(m, m->tri[3 * f]), p1 = vtx(m, m->tri[3 * f + 1]), p2 = vtx(m, m->tri[3 * f + 2]);
    cen[f] = mul(1.0 / 3.0, (p0 + p1) + p2);
  }
  B->order.resize(m->nF);
  std::iota(B->order.begin(), B->order.end(), 0);
  B->nodes.reserve(2 * (size_t)m->nF / 4 + 8);
  if (m->nF > 0) build_rec(B, m, cen, 0, m->nF);
  return B;
}

void ora_bvh_free(ora_bvh* b) { delete b; }

void ora_trace_closest(const ora_mesh* m, const ora_bvh* b, int32_t n, const double* o, const double* d, double tmin,
                       const int32_t* skip, int32_t* hit, double* t, double* bary2) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < n; ++i) {
    Hit h = closest(m, b, D3{o[3 * i], o[3 * i + 1], o[3 * i + 2]}, D3{d[3 * i], d[3 * i + 1], d[3 * i + 2]}, tmin,
                    skip ? skip[i] : -1);
    hit[i] = h.id;
    t[i] = h.id >= 0 ? h.t : INFINITY;
    bary2[2 * i] = h.b1;
    bary2[2 * i + 1] = h.b2;
  }
}

void ora_trace_any(const ora_mesh* m, const ora_bvh* b, int32_t n, const double* o, const double* d, double tmin,
                   const int32_t* skip, uint8_t* hit) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < n; ++i)
    hit[i] = any_hit(m, b, D3{o[3 * i], o[3 * i + 1], o[3 * i + 2]}, D3{d[3 * i], d[3 * i + 1], d[3 * i + 2]}, tmin,
                     skip ? skip[i] : -1)
                 ? 1
                 : 0;
}

// Decision margins of one ray, brute force over all triangles except `skip`. A decision of the
// watertight test can only differ between two precisions where the ray passes close to a
// triangle's boundary (the edge functions are near zero there) or where a hit lies close to
// the start of the ray's range. Distances are measured in space along the part of the ray that
// can matter, s >= s0 = tmin |d| - tol (s = distance from the origin):
//  n_hits          number of triangles hit at t >= tmin
//  max_hit_margin  max over hit triangles of min(distance from the ray to the triangle's
//                  three edges, |t - tmin| |d|)          (small: every hit is fragile)
//  min_margin      min over all triangles of the distance from the ray to their edges, and
//                  over triangles whose interior the ray's line crosses, of |t - tmin| |d|
//                                                        (small: some near miss could become a hit)
// A triangle the ray does not come near contributes nothing small, whatever its plane does.
namespace {
// distance from point p to the segment a-b
double point_segment_dist(D3 p, D3 a, D3 b) {
  D3 ab = b - a;
  double l2 = dot(ab, ab);
  double w = l2 > 0 ? std::min(1.0, std::max(0.0, dot(p - a, ab) / l2)) : 0.0;
  return norm(p - (a + mul(w, ab)));
}
// distance from point p to the ray o + s u (u unit), s >= s0
double point_ray_dist(D3 p, D3 o, D3 u, double s0) {
  double s = std::max(s0, dot(p - o, u));
  return norm(p - (o + mul(s, u)));
}
// Minimum over s >= s0 and w in [0,1] of |o + s u - (a + w (b - a))|, u unit. The squared
// distance is a convex quadratic in (s, w), so the minimum over this half-strip is the
// unconstrained stationary point when it lies inside, and otherwise lies on one of the three
// boundary pieces (s = s0, w = 0, w = 1), each a point-to-segment or point-to-ray distance.
double ray_segment_dist(D3 o, D3 u, double s0, D3 a, D3 b) {
  D3 e = b - a, r = o - a;
  double best = std::min({point_segment_dist(o + mul(s0, u), a, b), point_ray_dist(a, o, u, s0),
                          point_ray_dist(b, o, u, s0)});
  // stationary point of |r + s u - w e|^2: [1, -u.e; -u.e, e.e] (s, w) = (-r.u, r.e)
  double ue = dot(u, e), ee = dot(e, e);
  double det = ee - ue * ue;
  if (det > 1e-300 * ee) {
    double ru = dot(r, u), re = dot(r, e);
    double s = (-ru * ee + ue * re) / det;
    double w = (re - ue * ru) / det;
    if (s >= s0 && w >= 0.0 && w <= 1.0) best = std::min(best, norm((o + mul(s, u)) - (a + mul(w, e))));
  }
  return best;
}
}  // namespace

void ora_ray_margins(const ora_mesh* m, const double o_[3], const double d_[3], double tmin, int32_t skip, double tol,
                     int32_t* n_hits, double* max_hit_margin, double* min_margin) {
  D3 o{o_[0], o_[1], o_[2]}, d{d_[0], d_[1], d_[2]};
  const double dl = norm(d);
  const D3 u = mul(1.0 / dl, d);
  const double s0 = tmin * dl - tol;
  int32_t nh = 0;
  double mx = 0.0, mn = INFINITY;
  for (int32_t f = 0; f < m->nF; ++f) {
    if (f == skip) continue;
    D3 p0 = vtx(m, m->tri[3 * f]), p1 = vtx(m, m->tri[3 * f + 1]), p2 = vtx(m, m->tri[3 * f + 2]);
    double edge = std::min({ray_segment_dist(o, u, s0, p0, p1), ray_segment_dist(o, u, s0, p1, p2),
                            ray_segment_dist(o, u, s0, p2, p0)});
    mn = std::min(mn, edge);
    D3 nrm = cross(p1 - p0, p2 - p0);
    double den = dot(nrm, d);
    if (den == 0.0) continue;
    double t = dot(nrm, p0 - o) / den;
    D3 x = o + mul(t, d);
    double a2 = dot(nrm, nrm);
    double b0 = dot(cross(p1 - x, p2 - x), nrm) / a2;
    double b1 = dot(cross(p2 - x, p0 - x), nrm) / a2;
    double b2 = dot(cross(p0 - x, p1 - x), nrm) / a2;
    if (!(b0 >= 0 && b1 >= 0 && b2 >= 0)) continue;  // the line misses the interior
    double dt = std::fabs(t - tmin) * dl;
    mn = std::min(mn, dt);
    if (t >= tmin) {
      ++nh;
      mx = std::max(mx, std::min(edge, dt));
    }
  }
  *n_hits = nh;
  *max_hit_margin = mx;
  *min_margin = mn;
}

void ora_sample_rays(const ora_mesh* m, const ora_bvh* b, const ora_camera* cam, const ora_params_theta* th,
                     const ora_tables* tab, const ora_params* p, int32_t n, const int64_t* pix, const int32_t* idx,
                     int32_t stream, double* o, double* d, double* c, int32_t* skip, uint8_t* valid) {
  Scene S{m, b, th, tab, p, {}};
  S.attr.vnrm.resize(3 * (size_t)m->nV);
  S.attr.ftan.resize(4 * (size_t)m->nF);
  vertex_normals(m, S.attr.vnrm.data());
  face_tangents(m, S.attr.ftan.data());
  const size_t HW = (size_t)cam->H * cam->W;
  std::vector<int32_t> ids(HW);
  std::vector<double> bary(3 * HW);
  ora_raster(m, cam, ids.data(), bary.data());
  const uint32_t view = (uint32_t)cam->view_id;
  for (int32_t i = 0; i < n; ++i) {
    valid[i] = 0;
    const int64_t q = pix[i];
    const int32_t f = ids[q];
    if (f < 0) continue;
    Attr<double> A = query<double>(S, f, &bary[3 * q]);
    D3 org = A.x, dir{0, 0, 0};
    double cc = 0;
    int32_t sk = f;
    if (stream == 0) {
      Draw dr = draw(p, (uint32_t)q, view, (uint32_t)idx[i], 0u);
      EnvSample es = env_sample(tab, dr.x, dr.u2, dr.u3);
      dir = es.dir;
      cc = dot(A.ns, dir);
    } else {
      const int32_t j = stream == 1 ? idx[i] : stream - 2;
      D3 b1, b2;
      onb(A.ng, &b1, &b2);
      Draw dr = draw(p, (uint32_t)q, view, (uint32_t)j, 1u);
      double rr = std::sqrt(dr.u2), phi = 2.0 * kPi * dr.u3;
      double lz = std::sqrt(std::max(0.0, 1.0 - dr.u2));
      D3 w = (mul(rr * std::cos(phi), b1) + mul(rr * std::sin(phi), b2)) + mul(lz, A.ng);
      if (stream == 1) {
        dir = w;
        cc = dot(A.ng, w);
      } else {
        Hit h = closest(m, b, A.x, w, p->tmin, f);
        if (h.id < 0) continue;
        D3 q0 = vtx(m, m->tri[3 * h.id]), q1 = vtx(m, m->tri[3 * h.id + 1]), q2 = vtx(m, m->tri[3 * h.id + 2]);
        if (!(dot(w, cross(q1 - q0, q2 - q0)) < 0.0)) continue;
        double by[3] = {1.0 - h.b1 - h.b2, h.b1, h.b2};
        Attr<double> Y = query<double>(S, h.id, by);
        Draw ds = draw(p, (uint32_t)q, view, (uint32_t)idx[i], (uint32_t)stream);
        EnvSample es = env_sample(tab, ds.x, ds.u2, ds.u3);
        org = Y.x;
        dir = es.dir;
        cc = dot(Y.ns, dir);
        sk = h.id;
      }
    }
    o[3 * i] = org.x; o[3 * i + 1] = org.y; o[3 * i + 2] = org.z;
    d[3 * i] = dir.x; d[3 * i + 1] = dir.y; d[3 * i + 2] = dir.z;
    c[i] = cc;
    skip[i] = sk;
    valid[i] = 1;
  }
}

int32_t ora_render(const ora_mesh* m, const ora_bvh* b, const ora_camera* cam, const ora_params_theta* th,
                   const ora_tables* tab, const ora_params* p, int32_t n_pix, const int64_t* pix, ora_out* out,
                   int32_t n_threads) {
  if (p->N_d < 0 || p->N_d > 64 || p->N_b < 0 || p->N_s < 0 || p->N_b * p->N_s > 64) return -1;
  Scene S{m, b, th, tab, p, {}};
  S.attr.vnrm.resize(3 * (size_t)m->nV);
  S.attr.ftan.resize(4 * (size_t)m->nF);
  vertex_normals(m, S.attr.vnrm.data());
  face_tangents(m, S.attr.ftan.data());
  const size_t HW = (size_t)cam->H * cam->W;
  std::vector<int32_t> ids(HW);
  std::vector<double> bary(3 * HW);
  ora_raster(m, cam, ids.data(), bary.data());
  const bool jvp = th->tex_dot || th->env_dot;
  const int32_t n = pix ? n_pix : (int32_t)HW;
  const int Nb = std::max(p->N_b, 1);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t i = 0; i < n; ++i) {
    int64_t q = pix ? pix[i] : i;
    int32_t f = ids[q];
    const double* bb = &bary[3 * q];
    out->tri_id[i] = f;
    for (int k = 0; k < 3; ++k) out->bary[3 * i + k] = bb[k];
    std::vector<int32_t> st(Nb, -1);
    std::vector<double> sb(2 * Nb, 0.0);
    uint64_t vis = 0, svis = 0;
    int32_t ns = 0;
    double Ld[3] = {0, 0, 0}, Li[3] = {0, 0, 0}, dLd[3] = {0, 0, 0}, dLi[3] = {0, 0, 0};
    if (f >= 0) {
      if (jvp) {
        Dual a[3], c[3];
        shade_pixel<Dual>(S, cam, (uint32_t)q, f, bb, a, c, &vis, st.data(), sb.data(), &svis, &ns);
        for (int k = 0; k < 3; ++k) { Ld[k] = a[k].v; dLd[k] = a[k].d; Li[k] = c[k].v; dLi[k] = c[k].d; }
      } else {
        shade_pixel<double>(S, cam, (uint32_t)q, f, bb, Ld, Li, &vis, st.data(), sb.data(), &svis, &ns);
      }
    }
    for (int k = 0; k < 3; ++k) {
      out->L_dir[3 * i + k] = Ld[k];
      if (out->L_ind) out->L_ind[3 * i + k] = Li[k];
      if (out->dL_dir) out->dL_dir[3 * i + k] = dLd[k];
      if (out->dL_ind) out->dL_ind[3 * i + k] = dLi[k];
    }
    out->vis[i] = vis;
    if (out->sec_vis) out->sec_vis[i] = svis;
    if (out->n_shadow) out->n_shadow[i] = ns;
    if (out->sec_tri && p->N_b > 0)
      for (int j = 0; j < p->N_b; ++j) {
        out->sec_tri[(size_t)i * p->N_b + j] = st[j];
        out->sec_bary[((size_t)i * p->N_b + j) * 2] = sb[2 * j];
        out->sec_bary[((size_t)i * p->N_b + j) * 2 + 1] = sb[2 * j + 1];
      }
  }
  return 0;
}

}  // extern "C"
