// Indirect light evaluated at half resolution and brought to full resolution (the paper traces
// secondary rays at half resolution in both image dimensions and upsamples the indirect
// component; Implementation Details). Reading of the unstated filter: per axis the
// full-resolution pixel x sits at u = ((x + 1/2) n_half / n_full) - 1/2 in half-resolution pixel
// units (FP64, multiplication first), its two taps are floor(u) and floor(u) + 1 clamped to the
// edge with weights 1 - frac(u) and frac(u); of the four 2D taps only covered half-resolution
// pixels count and the weights are renormalised over them; a background pixel, or one with no
// covered tap, gets 0.
//
// Forward: one thread per full-resolution pixel (a gather). Adjoint: one thread per
// half-resolution pixel, gathering from every full-resolution pixel that has it among its taps,
// so that no atomics are needed and the result is deterministic.
#include <hip/hip_runtime.h>

#include "exm_internal.h"

namespace exm {
namespace {

constexpr int kThreads = 256;

struct Axis {
  int32_t i0, i1;
  float w0, w1;
};

__device__ __forceinline__ Axis up_axis(int32_t x, int32_t n_full, int32_t n_half) {
  const double u = ((double)x + 0.5) * (double)n_half / (double)n_full - 0.5;
  const double f0 = floor(u);
  const float fr = (float)(u - f0);
  const int32_t i = (int32_t)f0;
  Axis a;
  a.i0 = min(max(i, 0), n_half - 1);
  a.i1 = min(max(i + 1, 0), n_half - 1);
  a.w0 = 1.0f - fr;
  a.w1 = fr;
  return a;
}

// weight of half-resolution index i in the taps of an axis (clamped taps may coincide)
__device__ __forceinline__ float axis_weight(const Axis& a, int32_t i) {
  return (a.i0 == i ? a.w0 : 0.0f) + (a.i1 == i ? a.w1 : 0.0f);
}

// sum over the four 2D taps of w * covered
__device__ __forceinline__ float covered_weight(const Axis& ay, const Axis& ax, const int32_t* __restrict__ tri_h,
                                                int32_t Wh) {
  float s = 0.0f;
  if (tri_h[ay.i0 * Wh + ax.i0] >= 0) s += ay.w0 * ax.w0;
  if (tri_h[ay.i0 * Wh + ax.i1] >= 0) s += ay.w0 * ax.w1;
  if (tri_h[ay.i1 * Wh + ax.i0] >= 0) s += ay.w1 * ax.w0;
  if (tri_h[ay.i1 * Wh + ax.i1] >= 0) s += ay.w1 * ax.w1;
  return s;
}

__global__ __launch_bounds__(kThreads) void k_upsample(const int32_t* __restrict__ tri_half, int32_t Hh, int32_t Wh,
                                                       const float* __restrict__ L_half,
                                                       const int32_t* __restrict__ tri_id, int32_t H, int32_t W,
                                                       int32_t n_views, float* __restrict__ L) {
  const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t HW = (int64_t)H * W;
  if (gid >= HW * n_views) return;
  const int32_t v = (int32_t)(gid / HW);
  const int32_t y = (int32_t)((gid - v * HW) / W), x = (int32_t)(gid - v * HW - (int64_t)y * W);
  float o[3] = {0.f, 0.f, 0.f};
  if (tri_id[gid] >= 0) {
    const int32_t* th = tri_half + (int64_t)v * Hh * Wh;
    const float* lh = L_half + 3 * (int64_t)v * Hh * Wh;
    const Axis ay = up_axis(y, H, Hh), ax = up_axis(x, W, Wh);
    const int32_t ty[2] = {ay.i0, ay.i1}, tx[2] = {ax.i0, ax.i1};
    const float wy[2] = {ay.w0, ay.w1}, wx[2] = {ax.w0, ax.w1};
    float s = 0.0f;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int64_t k = (int64_t)ty[a] * Wh + tx[b];
        if (th[k] < 0) continue;
        const float w = wy[a] * wx[b];
        s += w;
        o[0] += w * lh[3 * k];
        o[1] += w * lh[3 * k + 1];
        o[2] += w * lh[3 * k + 2];
      }
    if (s > 0.0f) {
      const float inv = 1.0f / s;
      o[0] *= inv;
      o[1] *= inv;
      o[2] *= inv;
    } else {
      o[0] = o[1] = o[2] = 0.0f;
    }
  }
  L[3 * gid] = o[0];
  L[3 * gid + 1] = o[1];
  L[3 * gid + 2] = o[2];
}

// dL_half[k] = sum over covered full-resolution pixels p with k among their taps of
// w_k(p) / S(p) * lambda * dI(p)
__global__ __launch_bounds__(kThreads) void k_upsample_bwd(const int32_t* __restrict__ tri_half, int32_t Hh,
                                                           int32_t Wh, const int32_t* __restrict__ tri_id, int32_t H,
                                                           int32_t W, int32_t n_views, float lambda,
                                                           const float* __restrict__ dI, float* __restrict__ dL_half) {
  const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t HWh = (int64_t)Hh * Wh;
  if (gid >= HWh * n_views) return;
  const int32_t v = (int32_t)(gid / HWh);
  const int32_t i = (int32_t)((gid - v * HWh) / Wh), j = (int32_t)(gid - v * HWh - (int64_t)i * Wh);
  const int32_t* th = tri_half + (int64_t)v * HWh;
  float acc[3] = {0.f, 0.f, 0.f};
  if (th[(int64_t)i * Wh + j] >= 0) {
    // full-resolution rows and columns that can have i (j) among their taps, with a margin
    const int32_t y0 = max(0, (int32_t)floor((double)(i - 1) * H / Hh) - 2);
    const int32_t y1 = min(H - 1, (int32_t)ceil((double)(i + 2) * H / Hh) + 2);
    const int32_t x0 = max(0, (int32_t)floor((double)(j - 1) * W / Wh) - 2);
    const int32_t x1 = min(W - 1, (int32_t)ceil((double)(j + 2) * W / Wh) + 2);
    const int64_t base = (int64_t)v * H * W;
    for (int32_t y = y0; y <= y1; ++y) {
      const Axis ay = up_axis(y, H, Hh);
      const float wyi = axis_weight(ay, i);
      if (wyi == 0.0f) continue;
      for (int32_t x = x0; x <= x1; ++x) {
        const Axis ax = up_axis(x, W, Wh);
        const float wxj = axis_weight(ax, j);
        if (wxj == 0.0f) continue;
        const int64_t p = base + (int64_t)y * W + x;
        if (tri_id[p] < 0) continue;
        const float s = covered_weight(ay, ax, th, Wh);
        if (!(s > 0.0f)) continue;
        const float f = wyi * wxj / s * lambda;
        acc[0] += f * dI[3 * p];
        acc[1] += f * dI[3 * p + 1];
        acc[2] += f * dI[3 * p + 2];
      }
    }
  }
  dL_half[3 * gid] = acc[0];
  dL_half[3 * gid + 1] = acc[1];
  dL_half[3 * gid + 2] = acc[2];
}

}  // namespace

hipError_t launch_upsample(const int32_t* tri_half, int32_t Hh, int32_t Wh, const float* L_half, const int32_t* tri_id,
                           int32_t H, int32_t W, int32_t n_views, float* L, hipStream_t s) {
  const int64_t n = (int64_t)H * W * n_views;
  {
    EXM_TIMED("upsample", s);
    k_upsample<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(tri_half, Hh, Wh, L_half, tri_id, H, W,
                                                                              n_views, L);
  }
  return hipGetLastError();
}

hipError_t launch_upsample_bwd(const int32_t* tri_half, int32_t Hh, int32_t Wh, const int32_t* tri_id, int32_t H,
                               int32_t W, int32_t n_views, float lambda, const float* dI, float* dL_half,
                               hipStream_t s) {
  const int64_t n = (int64_t)Hh * Wh * n_views;
  {
    EXM_TIMED("upsample_bwd", s);
    k_upsample_bwd<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(tri_half, Hh, Wh, tri_id, H, W,
                                                                                  n_views, lambda, dI, dL_half);
  }
  return hipGetLastError();
}

}  // namespace exm
