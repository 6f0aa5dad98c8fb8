// G-buffer raster: for every pixel the closest triangle f and its perspective-correct
// barycentrics b (the visible point of the Attribute Query).
//
// Bit-exact rules (shared with the CPU reference by specification only):
//  * clip = MVP [p,1] in FP64 without FMA; pixel x = ((x/w)+1)/2 W, y = (1-(y/w))/2 H,
//    z01 = ((z/w)+1)/2; vertices snapped with rint to 1/256 pixel (int64); a triangle with a
//    vertex at w <= 0, beyond +-2^30 sub-pixel units, or with non-finite depth is dropped.
//  * one sample at the pixel centre (256 px + 128); int64 edge functions; top-left fill rule
//    in y-down space (an edge owns its samples if dy < 0, or dy == 0 and dx > 0); both
//    windings rasterise; zero-area triangles never cover.
//  * depth z01 = (E0 z0 + E1 z1 + E2 z2) / A2 in FP64; fragments outside [0,1] discarded;
//    the 64-bit key (float bits of z01) << 32 | id is minimised with an atomic, so ties go to
//    the lower id whatever the launch order.
// Three kernels: clear the key buffer (the bary output, 8 bytes per pixel), one thread per
// (triangle, view) with a wave-cooperative loop for triangles covering many pixels, and a
// per-pixel resolve that recomputes the winner's barycentrics and overwrites the key.
#include <hip/hip_runtime.h>

#include "exm_internal.h"

namespace exm {
namespace {

constexpr int kThreads = 256;
constexpr int64_t kSmallPixels = 16;

struct Proj {
  int64_t X[3], Y[3];
  double z[3], w[3];
  bool ok;
};

__device__ __forceinline__ Proj project(const float* __restrict__ pos, const int32_t* __restrict__ tri, int32_t f,
                                        const double* M, int32_t H, int32_t W) {
#pragma clang fp contract(off)
  Proj P;
  P.ok = true;
  const double lim = 1073741824.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int32_t vi = tri[3 * f + k];
    const double x = pos[3 * vi], y = pos[3 * vi + 1], z = pos[3 * vi + 2];
    const double cx = ((M[0] * x + M[1] * y) + M[2] * z) + M[3];
    const double cy = ((M[4] * x + M[5] * y) + M[6] * z) + M[7];
    const double cz = ((M[8] * x + M[9] * y) + M[10] * z) + M[11];
    const double cw = ((M[12] * x + M[13] * y) + M[14] * z) + M[15];
    const double xs = ((((cx / cw) + 1.0) * 0.5) * (double)W) * 256.0;
    const double ys = (((1.0 - (cy / cw)) * 0.5) * (double)H) * 256.0;
    const double zz = ((cz / cw) + 1.0) * 0.5;
    if (!(cw > 0.0) || !(fabs(xs) <= lim && fabs(ys) <= lim) || !isfinite(zz)) P.ok = false;
    P.X[k] = P.ok ? (int64_t)rint(xs) : 0;
    P.Y[k] = P.ok ? (int64_t)rint(ys) : 0;
    P.z[k] = zz;
    P.w[k] = cw;
  }
  return P;
}

// coverage of sample (Px,Py); on success E[k] carries the original vertex labels, A2 > 0
__device__ __forceinline__ bool cover(const Proj& P, int64_t Px, int64_t Py, int64_t E[3], int64_t* A2) {
  int64_t a2 = (P.X[1] - P.X[0]) * (P.Y[2] - P.Y[0]) - (P.X[2] - P.X[0]) * (P.Y[1] - P.Y[0]);
  if (a2 == 0) return false;
  const bool swp = a2 < 0;
  if (swp) a2 = -a2;
  // slot s is opposite vertex o[s]; with a negative area vertices 1 and 2 trade places
  const int o0 = 0, o1 = swp ? 2 : 1, o2 = swp ? 1 : 2;
  const int ord[3] = {o0, o1, o2};
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int ia = ord[(s + 1) % 3], ib = ord[(s + 2) % 3];
    const int64_t dx = P.X[ib] - P.X[ia], dy = P.Y[ib] - P.Y[ia];
    const int64_t e = dx * (Py - P.Y[ia]) - dy * (Px - P.X[ia]);
    if (!(e > 0 || (e == 0 && (dy < 0 || (dy == 0 && dx > 0))))) return false;
    E[ord[s]] = e;
  }
  *A2 = a2;
  return true;
}

__device__ __forceinline__ int64_t ceil_px(int64_t v) {  // first pixel whose centre is >= v
  const int64_t t = v - 128;
  return t >= 0 ? (t + 255) / 256 : -((-t) / 256);
}
__device__ __forceinline__ int64_t floor_px(int64_t v) {  // last pixel whose centre is <= v
  const int64_t t = v - 128;
  return t >= 0 ? t / 256 : -((-t + 255) / 256);
}

__device__ __forceinline__ void fragment(const Proj& P, int32_t f, int64_t px, int64_t py, int32_t W,
                                         unsigned long long* __restrict__ keys) {
#pragma clang fp contract(off)
  int64_t E[3], A2;
  if (!cover(P, 256 * px + 128, 256 * py + 128, E, &A2)) return;
  const double z = (((double)E[0] * P.z[0] + (double)E[1] * P.z[1]) + (double)E[2] * P.z[2]) / (double)A2;
  if (!(z >= 0.0 && z <= 1.0)) return;
  float zf = (float)z;
  if (zf == 0.0f) zf = 0.0f;  // -0 -> +0
  const unsigned long long key = ((unsigned long long)__float_as_uint(zf) << 32) | (uint32_t)f;
  atomicMin(keys + py * W + px, key);
}

__global__ __launch_bounds__(kThreads) void k_clear(int64_t n, unsigned long long* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) keys[i] = ~0ull;
}

__global__ __launch_bounds__(kThreads) void k_raster(int32_t nF, const float* __restrict__ pos,
                                                     const int32_t* __restrict__ tri, RasterViews V,
                                                     unsigned long long* __restrict__ keys_all) {
  const int32_t view = blockIdx.y;
  const int32_t f = blockIdx.x * kThreads + threadIdx.x;
  const int32_t H = V.H, W = V.W;
  unsigned long long* keys = keys_all + (int64_t)view * H * W;
  Proj P;
  P.ok = false;
  int64_t x0 = 0, x1 = -1, y0 = 0, y1 = -1;
  if (f < nF) {
    P = project(pos, tri, f, V.mvp[view], H, W);
    if (P.ok) {
      const int64_t xmin = min(P.X[0], min(P.X[1], P.X[2])), xmax = max(P.X[0], max(P.X[1], P.X[2]));
      const int64_t ymin = min(P.Y[0], min(P.Y[1], P.Y[2])), ymax = max(P.Y[0], max(P.Y[1], P.Y[2]));
      x0 = max((int64_t)0, ceil_px(xmin));
      x1 = min((int64_t)W - 1, floor_px(xmax));
      y0 = max((int64_t)0, ceil_px(ymin));
      y1 = min((int64_t)H - 1, floor_px(ymax));
    }
  }
  const int64_t nx = x1 - x0 + 1, ny = y1 - y0 + 1;
  const int64_t npix = (P.ok && nx > 0 && ny > 0) ? nx * ny : 0;
  const bool big = npix > kSmallPixels;
  if (!big && npix > 0) {  // row by row: no 64-bit division per pixel
    for (int64_t yy = y0; yy <= y1; ++yy)
      for (int64_t xx = x0; xx <= x1; ++xx) fragment(P, f, xx, yy, W, keys);
  }
  // large triangles: the whole wave walks one triangle's pixels at a time
  unsigned long long mask = __ballot(big);
  const int lane = threadIdx.x & 63;
  while (mask) {
    const int src = __ffsll((long long)mask) - 1;
    mask &= mask - 1;
    Proj Q;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Q.X[k] = __shfl(P.X[k], src, 64);
      Q.Y[k] = __shfl(P.Y[k], src, 64);
      Q.z[k] = __shfl(P.z[k], src, 64);
    }
    const int32_t qf = __shfl(f, src, 64);
    const int64_t qx0 = __shfl(x0, src, 64), qy0 = __shfl(y0, src, 64);
    const int64_t qnx = __shfl(nx, src, 64), qn = __shfl(npix, src, 64);
    if (qn < ((int64_t)1 << 31)) {  // 32-bit division for the pixel of index k
      const uint32_t n32 = (uint32_t)qn, nx32 = (uint32_t)qnx;
      for (uint32_t k = lane; k < n32; k += 64) fragment(Q, qf, qx0 + k % nx32, qy0 + k / nx32, W, keys);
    } else {
      for (int64_t k = lane; k < qn; k += 64) fragment(Q, qf, qx0 + k % qnx, qy0 + k / qnx, W, keys);
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_resolve(const float* __restrict__ pos, const int32_t* __restrict__ tri,
                                                      RasterViews V, int32_t* __restrict__ tri_id,
                                                      float* __restrict__ bary) {
#pragma clang fp contract(off)
  // 32-bit pixel indices: the boundary holds nViews * H * W below 2^31
  const uint32_t HW = (uint32_t)V.H * (uint32_t)V.W;
  const uint32_t gid = blockIdx.x * kThreads + threadIdx.x;
  if (gid >= HW * (uint32_t)V.n) return;
  const uint32_t view = gid / HW;
  const uint32_t p = gid - view * HW, px = p % (uint32_t)V.W, py = p / (uint32_t)V.W;
  const unsigned long long key = reinterpret_cast<const unsigned long long*>(bary)[gid];
  float2 out = make_float2(0.f, 0.f);
  int32_t f = -1;
  if (key != ~0ull) {
    f = (int32_t)(uint32_t)key;
    const Proj P = project(pos, tri, f, V.mvp[view], V.H, V.W);
    int64_t E[3], A2;
    cover(P, 256 * (int64_t)px + 128, 256 * (int64_t)py + 128, E, &A2);
    const double q0 = (double)E[0] / P.w[0], q1 = (double)E[1] / P.w[1], q2 = (double)E[2] / P.w[2];
    const double s = (q0 + q1) + q2;
    out = make_float2((float)(q1 / s), (float)(q2 / s));
  }
  tri_id[gid] = f;
  reinterpret_cast<float2*>(bary)[gid] = out;
}

}  // namespace

hipError_t launch_raster(const exm_mesh* m, const RasterViews& v, int32_t* tri_id, float* bary, hipStream_t s) {
  const int64_t n = (int64_t)v.n * v.H * v.W;
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(bary);
  const unsigned nb = (unsigned)((n + kThreads - 1) / kThreads);
  {
    EXM_TIMED("raster_clear", s);
    k_clear<<<nb, kThreads, 0, s>>>(n, keys);
  }
  if (m->nF > 0) {
    dim3 grid((m->nF + kThreads - 1) / kThreads, v.n);
    {
      EXM_TIMED("raster", s);
      k_raster<<<grid, kThreads, 0, s>>>(m->nF, m->pos, m->tri, v, keys);
    }
  }
  {
    EXM_TIMED("raster_resolve", s);
    k_resolve<<<nb, kThreads, 0, s>>>(m->pos, m->tri, v, tri_id, bary);
  }
  return hipGetLastError();
}

}  // namespace exm
