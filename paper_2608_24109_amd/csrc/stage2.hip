// The Stage-II objective (Stage-II Optimization, Eq. 21-24) and the optimiser step, on the device.
//
// Readings of what the paper leaves open (stated once more in include/exm.h):
//   L_img = lambda_log * mean |log(1 + I_hat) - log(1 + I)| + lambda_ssim * (1 - mean SSIM),
//     lambda_ssim = 0.2, lambda_log = 0.8, means over pixels and channels of a view; SSIM of
//     Wang et al. 2004 per channel on the sRGB curve of the radiance clamped to [0, 1], 11-tap
//     Gaussian window (sigma 1.5), zero padding, C1 = 0.01^2, C2 = 0.03^2.
//   TV(P_hat): for the map groups A, R, N (and M when metallic is optimised), the sum over
//     right/down neighbour pairs of visible pixels of the group's channel-mean |difference| of
//     the screen projection (the bilinear query of Eq. 10), over the view's pixel count.
//   TV(E): the same over env texels with phi wrapping, over He * We. Chroma: squared distance of
//     the per-channel texel mean of E from its grey mean (Eq. 24).
//
// The SSIM gradient uses the derivatives of SSIM with respect to the local moments
// (mu_x, E[x^2], E[xy]) and the fact that the zero-padded Gaussian blur is its own transpose:
//   dS/dx = blur(dS/dmu_x) + 2 x blur(dS/dE[x^2]) + y blur(dS/dE[xy]).
#include <hip/hip_runtime.h>

#include "exm_device.h"
#include "exm_internal.h"

namespace exm {
namespace {

constexpr int kThreads = 256;
constexpr int kTaps = 11;
constexpr float kC1 = 1e-4f, kC2 = 9e-4f;
constexpr float kLambdaSsim = 0.2f, kLambdaLog = 0.8f;

struct Gauss {
  float g[kTaps];
};

constexpr int32_t kTvRows = 4;

// Kernels that also sum into an FP64 scalar run as grid-stride loops over at most this many
// blocks, so that the scalar takes one atomic per block and not one per 256 pixels (ten
// thousand same-address atomics per 1600^2 view serialise).
constexpr unsigned kReduceBlocks = 1024;

__device__ __forceinline__ void block_add(double v, double* out) {
  __shared__ double red[kThreads];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0.0) atomicAdd(out, red[0]);
}

__device__ __forceinline__ float srgb(float v) {
  v = fminf(fmaxf(v, 0.0f), 1.0f);
  return v <= 0.0031308f ? 12.92f * v : 1.055f * powf(v, 1.0f / 2.4f) - 0.055f;
}
__device__ __forceinline__ float srgb_d(float v) {
  if (!(v > 0.0f && v < 1.0f)) return 0.0f;
  return v <= 0.0031308f ? 12.92f : 1.055f / 2.4f * powf(v, 1.0f / 2.4f - 1.0f);
}
__device__ __forceinline__ float sgn(float x) { return (float)((x > 0.0f) - (x < 0.0f)); }

__global__ void k_fill_zero_f64(double* p, int32_t n) {
  if ((int32_t)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

// ---- screen projection of the maps --------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_project(MeshView M, TexView T, int64_t n_px,
                                                      const int32_t* __restrict__ tri_id,
                                                      const float* __restrict__ bary, float* __restrict__ P) {
  const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (gid >= n_px) return;
  float ch[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const int32_t f = tri_id[gid];
  if (f >= 0) {
    const float2 b = reinterpret_cast<const float2*>(bary)[gid];
    int32_t tap[4];
    float w[4];
    surface_taps(M, T, f, b.x, b.y, tap, w);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float4* tp = reinterpret_cast<const float4*>(T.tex + (int64_t)tap[k] * 8);
      const float4 lo = tp[0], hi = tp[1];
      ch[0] += w[k] * lo.x;
      ch[1] += w[k] * lo.y;
      ch[2] += w[k] * lo.z;
      ch[3] += w[k] * lo.w;
      ch[4] += w[k] * hi.x;
      ch[5] += w[k] * hi.y;
      ch[6] += w[k] * hi.z;
      ch[7] += w[k] * hi.w;
    }
  }
  float4* o = reinterpret_cast<float4*>(P + 8 * gid);
  o[0] = make_float4(ch[0], ch[1], ch[2], ch[3]);
  o[1] = make_float4(ch[4], ch[5], ch[6], ch[7]);
}

__global__ __launch_bounds__(kThreads) void k_project_bwd(MeshView M, TexView T, int64_t n_px,
                                                          const int32_t* __restrict__ tri_id,
                                                          const float* __restrict__ bary,
                                                          const float* __restrict__ dP, float* __restrict__ dtex) {
  const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (gid >= n_px) return;
  const int32_t f = tri_id[gid];
  if (f < 0) return;
  const float2 b = reinterpret_cast<const float2*>(bary)[gid];
  int32_t tap[4];
  float w[4];
  surface_taps(M, T, f, b.x, b.y, tap, w);
  const float* g = dP + 8 * gid;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (w[k] == 0.0f) continue;
    float* dst = dtex + (int64_t)tap[k] * 8;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (g[c] != 0.0f) unsafeAtomicAdd(dst + c, w[k] * g[c]);
  }
}

// ---- image loss -------------------------------------------------------------------------

// planes of one view: x, y, x^2, y^2, xy for 3 channels (15), their blur (15), a temporary (15)
// and the 9 planes of moment derivatives with their blur and temporary
struct ImgWs {
  float* mom;   // [15][H][W]
  float* bmom;  // [15][H][W]
  float* tmp;   // [15][H][W]
  float* dmo;   // [9][H][W]
  float* bdmo;  // [9][H][W]
};

__global__ __launch_bounds__(kThreads) void k_img_prep(const float* __restrict__ a, const float* __restrict__ b,
                                                       int64_t HW, float scale, ImgWs w, float* __restrict__ dA,
                                                       double* __restrict__ loss) {
  double l1 = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < HW; p += (int64_t)gridDim.x * kThreads) {
    const float inv_n = 1.0f / (3.0f * (float)HW);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float va = a[3 * p + c], vb = b[3 * p + c];
      const float d = log1pf(va) - log1pf(vb);
      l1 += fabsf(d);
      dA[3 * p + c] = scale * kLambdaLog * sgn(d) / (1.0f + va) * inv_n;
      const float x = srgb(va), y = srgb(vb);
      w.mom[(0 * 3 + c) * HW + p] = x;
      w.mom[(1 * 3 + c) * HW + p] = y;
      w.mom[(2 * 3 + c) * HW + p] = x * x;
      w.mom[(3 * 3 + c) * HW + p] = y * y;
      w.mom[(4 * 3 + c) * HW + p] = x * y;
    }
  }
  l1 *= (double)scale * kLambdaLog / (3.0 * (double)HW);
  block_add(l1, loss);
}

// horizontal then vertical pass of the Gaussian over planes of H x W (zero padding); grid
// (x blocks, rows, planes), so no index division
// The horizontal pass stages kSegH pixels of a row and their halo in LDS; each thread then
// writes kPerThreadH consecutive outputs.
constexpr int kPerThreadH = 4;
constexpr int kSegH = kThreads * kPerThreadH;

__global__ __launch_bounds__(kThreads) void k_blur_h(const float* __restrict__ in, float* __restrict__ out, int32_t H,
                                                     int32_t W, Gauss g) {
  __shared__ float seg[kSegH + kTaps - 1];
  const int32_t x0 = blockIdx.x * kSegH;
  const int64_t row = ((int64_t)blockIdx.z * H + blockIdx.y) * W;
  const float* r = in + row;
  for (int32_t i = threadIdx.x; i < kSegH + kTaps - 1; i += kThreads) {
    const int32_t xx = x0 - kTaps / 2 + i;
    seg[i] = (xx >= 0 && xx < W) ? r[xx] : 0.0f;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPerThreadH; ++q) {
    const int32_t j = threadIdx.x * kPerThreadH + q;  // output x0 + j, taps seg[j .. j + 10]
    if (x0 + j >= W) break;
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kTaps; ++k) s += g.g[k] * seg[j + k];
    out[row + x0 + j] = s;
  }
}

// The vertical pass walks a strip of kRowsV rows per block with the 11-row window in registers,
// so each input row is read once per strip (one block per row would spread a column's rows over
// the XCDs and fetch every row eleven times). Taps outside the image add zero, which leaves the
// sum of the in-image taps unchanged.
constexpr int kRowsV = 64;

__global__ __launch_bounds__(kThreads) void k_blur_v(const float* __restrict__ in, float* __restrict__ out, int32_t H,
                                                     int32_t W, Gauss g) {
  const int32_t x = blockIdx.x * kThreads + threadIdx.x;
  if (x >= W) return;
  const int32_t y0 = blockIdx.y * kRowsV, y1 = min(H, y0 + kRowsV);
  const float* col = in + (int64_t)blockIdx.z * H * W + x;
  float* ocol = out + (int64_t)blockIdx.z * H * W + x;
  float win[kTaps];
  win[0] = 0.0f;
#pragma unroll
  for (int k = 0; k < kTaps - 1; ++k) {
    const int32_t yy = y0 - kTaps / 2 + k;
    win[k + 1] = (yy >= 0 && yy < H) ? col[(int64_t)yy * W] : 0.0f;
  }
  for (int32_t y = y0; y < y1; y += 4) {
    float nxt[4];  // the next four rows in flight together
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int32_t yy = y + q + kTaps / 2;
      nxt[q] = yy < H ? col[(int64_t)yy * W] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (y + q >= y1) break;
#pragma unroll
      for (int k = 0; k < kTaps - 1; ++k) win[k] = win[k + 1];
      win[kTaps - 1] = nxt[q];
      float s = 0.0f;
#pragma unroll
      for (int k = 0; k < kTaps; ++k) s += g.g[k] * win[k];
      ocol[(int64_t)(y + q) * W] = s;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_ssim_terms(ImgWs w, int64_t HW, float scale, double* __restrict__ loss) {
  double ssum = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < HW; p += (int64_t)gridDim.x * kThreads) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float mx = w.bmom[(0 * 3 + c) * HW + p], my = w.bmom[(1 * 3 + c) * HW + p];
      const float sxx = w.bmom[(2 * 3 + c) * HW + p] - mx * mx;
      const float syy = w.bmom[(3 * 3 + c) * HW + p] - my * my;
      const float sxy = w.bmom[(4 * 3 + c) * HW + p] - mx * my;
      const float a1 = 2.0f * mx * my + kC1, a2 = 2.0f * sxy + kC2;
      const float b1 = mx * mx + my * my + kC1, b2 = sxx + syy + kC2;
      const float ib = 1.0f / (b1 * b2);
      const float S = a1 * a2 * ib;
      ssum += S;
      w.dmo[(0 * 3 + c) * HW + p] = 2.0f * my * (a2 - a1) * ib - 2.0f * mx * S * (b2 - b1) * ib;
      w.dmo[(1 * 3 + c) * HW + p] = -S / b2;
      w.dmo[(2 * 3 + c) * HW + p] = 2.0f * a1 * ib;
    }
  }
  // loss += scale * lambda_ssim * (1 - sum S / N): the constant part once per view
  double v = -(double)scale * kLambdaSsim * ssum / (3.0 * (double)HW);
  if (blockIdx.x == 0 && threadIdx.x == 0) v += (double)scale * kLambdaSsim;
  block_add(v, loss);
}

__global__ __launch_bounds__(kThreads) void k_img_grad(const float* __restrict__ a, int64_t HW, float scale, ImgWs w,
                                                       float* __restrict__ dA) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= HW) return;
  const float inv_n = 1.0f / (3.0f * (float)HW);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float x = w.mom[(0 * 3 + c) * HW + p], y = w.mom[(1 * 3 + c) * HW + p];
    const float dx = (w.bdmo[(0 * 3 + c) * HW + p] + 2.0f * x * w.bdmo[(1 * 3 + c) * HW + p] +
                      y * w.bdmo[(2 * 3 + c) * HW + p]) * inv_n;
    dA[3 * p + c] -= scale * kLambdaSsim * dx * srgb_d(a[3 * p + c]);
  }
}

// ---- total variation --------------------------------------------------------------------

// per-channel weight of the material TV: scale / (group size * H * W) for the channels of the
// active groups (A, R, N, and M when the metallic map is optimised), 0 elsewhere
struct TvWeights {
  float w[8];
};

// grid (column blocks, bands of kTvRows rows, views): one thread per pixel and row of the band,
// no index division, one atomic per block for the loss
__global__ __launch_bounds__(kThreads) void k_tv_screen(const float* __restrict__ P, const int32_t* __restrict__ tri,
                                                        int32_t H, int32_t W, TvWeights cw,
                                                        double* __restrict__ loss, float* __restrict__ dP) {
  const int64_t HW = (int64_t)H * W;
  double l = 0.0;
  const int32_t x = blockIdx.x * kThreads + threadIdx.x;
  const int32_t y_end = min(H, (int32_t)(blockIdx.y + 1) * kTvRows);
  for (int32_t y = blockIdx.y * kTvRows; y < y_end && x < W; ++y) {
    const int64_t gid = (int64_t)blockIdx.z * HW + (int64_t)y * W + x;
    float g[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (tri[gid] >= 0) {
      const float4 p0 = reinterpret_cast<const float4*>(P)[2 * gid];
      const float4 p1 = reinterpret_cast<const float4*>(P)[2 * gid + 1];
      const float pp[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
      const int64_t nb[4] = {x + 1 < W ? gid + 1 : -1, x > 0 ? gid - 1 : -1, y + 1 < H ? gid + W : -1,
                             y > 0 ? gid - W : -1};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (nb[q] < 0 || tri[nb[q]] < 0) continue;
        const float4 q0 = reinterpret_cast<const float4*>(P)[2 * nb[q]];
        const float4 q1 = reinterpret_cast<const float4*>(P)[2 * nb[q] + 1];
        const float pq[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const float d = pp[c] - pq[c];
          g[c] += cw.w[c] * sgn(d);
          if (q == 0 || q == 2) l += (double)cw.w[c] * fabsf(d);  // each pair once (right, down)
        }
      }
    }
    float4* o = reinterpret_cast<float4*>(dP + 8 * gid);
    o[0] = make_float4(g[0], g[1], g[2], g[3]);
    o[1] = make_float4(g[4], g[5], g[6], g[7]);
  }
  block_add(l, loss);
}

// channel sums of E into acc[0..2] (FP64)
__global__ __launch_bounds__(kThreads) void k_env_sum(const float* __restrict__ E, int64_t n, double* __restrict__ acc) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double v = t < n ? (double)E[3 * t + c] : 0.0;
    block_add(v, acc + c);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void k_env_reg(const float* __restrict__ E, int32_t He, int32_t We, float w_tv,
                                                      float w_chroma, const double* __restrict__ acc,
                                                      double* __restrict__ loss, double* __restrict__ dE) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t n = (int64_t)He * We;
  double l = 0.0;
  if (t < n) {
    const int32_t i = (int32_t)(t / We), j = (int32_t)(t - (int64_t)i * We);
    const int64_t r = (int64_t)i * We + (j + 1 < We ? j + 1 : 0);   // right (phi wraps)
    const int64_t lft = (int64_t)i * We + (j > 0 ? j - 1 : We - 1);  // left
    const double wt = (double)w_tv / (3.0 * (double)n);
    const double m[3] = {acc[0] / (double)n, acc[1] / (double)n, acc[2] / (double)n};
    const double mu = (m[0] + m[1] + m[2]) / 3.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float e = E[3 * t + c];
      double g = wt * (sgn(e - E[3 * r + c]) + sgn(e - E[3 * lft + c]));
      l += wt * fabs((double)E[3 * r + c] - (double)e);
      if (i + 1 < He) {
        g += wt * sgn(e - E[3 * (t + We) + c]);
        l += wt * fabs((double)E[3 * (t + We) + c] - (double)e);
      }
      if (i > 0) g += wt * sgn(e - E[3 * (t - We) + c]);
      g += (double)w_chroma * 2.0 * (m[c] - mu) / (double)n;
      dE[3 * t + c] += g;
    }
    if (t == 0) {
      double ch = 0.0;
      for (int c = 0; c < 3; ++c) ch += (m[c] - mu) * (m[c] - mu);
      l += (double)w_chroma * ch;
    }
  }
  block_add(l, loss);
}

// ---- optimiser ----------------------------------------------------------------------------

struct Bounds {
  float lo[8], hi[8];
};

// Adam coefficients, each formed in double and rounded once (1 - beta2 rounded from the float
// beta2 would be off by 1e-5 relative).
struct AdamCoef {
  float lr, b1, b2, omb1, omb2, eps, c1, c2;
};

template <typename G>
__global__ __launch_bounds__(kThreads) void k_adam(float* __restrict__ prm, const G* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                   int32_t n_chan, Bounds bd, AdamCoef k) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const float g = (float)grad[i];
  const float mi = k.b1 * m[i] + k.omb1 * g;
  const float vi = k.b2 * v[i] + k.omb2 * (g * g);
  m[i] = mi;
  v[i] = vi;
  const int32_t c = (int32_t)(i % n_chan);
  const float p = prm[i] - k.lr * (mi * k.c1) / (sqrtf(vi * k.c2) + k.eps);
  prm[i] = fminf(fmaxf(p, bd.lo[c]), bd.hi[c]);
}

Gauss gauss_taps() {
  Gauss g;
  double w[kTaps], s = 0.0;
  for (int k = 0; k < kTaps; ++k) {
    const double x = k - (kTaps - 1) / 2.0;
    w[k] = exp(-x * x / (2.0 * 1.5 * 1.5));
    s += w[k];
  }
  for (int k = 0; k < kTaps; ++k) g.g[k] = (float)(w[k] / s);
  return g;
}

unsigned nblk(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

MeshView mesh_view(const exm_mesh* m);

size_t image_loss_ws_bytes(int32_t H, int32_t W) { return (size_t)(15 * 3 + 9 * 2) * H * W * sizeof(float); }

hipError_t launch_project(const exm_mesh* m, const exm_material* mat, int64_t n_px, const int32_t* tri_id,
                          const float* bary, float* P, hipStream_t s) {
  EXM_TIMED("project_maps", s);
  k_project<<<nblk(n_px), kThreads, 0, s>>>(mesh_view(m), TexView{mat->Ht, mat->Wt, mat->tex}, n_px, tri_id, bary, P);
  return hipGetLastError();
}

hipError_t launch_project_bwd(const exm_mesh* m, const exm_material* mat, int64_t n_px, const int32_t* tri_id,
                              const float* bary, const float* dP, float* dtex, hipStream_t s) {
  EXM_TIMED("project_maps_bwd", s);
  k_project_bwd<<<nblk(n_px), kThreads, 0, s>>>(mesh_view(m), TexView{mat->Ht, mat->Wt, mat->tex}, n_px, tri_id, bary,
                                                dP, dtex);
  return hipGetLastError();
}

hipError_t launch_image_loss(const float* a, const float* b, int32_t n_views, int32_t H, int32_t W, float scale,
                             double* loss, float* dA, void* ws, hipStream_t s) {
  const int64_t HW = (int64_t)H * W;
  float* q = static_cast<float*>(ws);
  ImgWs w{q, q + 15 * HW, q + 30 * HW, q + 45 * HW, q + 54 * HW};
  float* tmp9 = w.tmp;  // the 9-plane pass reuses the first planes of tmp
  const Gauss g = gauss_taps();
  for (int32_t v = 0; v < n_views; ++v) {
    const float* av = a + 3 * v * HW;
    const float* bv = b + 3 * v * HW;
    float* dv = dA + 3 * v * HW;
    const unsigned segs = (unsigned)((W + kSegH - 1) / kSegH);
    const dim3 g15(segs, (unsigned)H, 15), g9(segs, (unsigned)H, 9);
    const unsigned strips = (unsigned)((H + kRowsV - 1) / kRowsV);
    const dim3 v15(nblk(W), strips, 15), v9(nblk(W), strips, 9);
    {
      EXM_TIMED("image_loss_prep", s);
      k_img_prep<<<std::min(nblk(HW), kReduceBlocks), kThreads, 0, s>>>(av, bv, HW, scale, w, dv, loss);
    }
    {
      EXM_TIMED("image_loss_blur_h", s);
      k_blur_h<<<g15, kThreads, 0, s>>>(w.mom, w.tmp, H, W, g);
    }
    {
      EXM_TIMED("image_loss_blur_v", s);
      k_blur_v<<<v15, kThreads, 0, s>>>(w.tmp, w.bmom, H, W, g);
    }
    {
      EXM_TIMED("image_loss_ssim", s);
      k_ssim_terms<<<std::min(nblk(HW), kReduceBlocks), kThreads, 0, s>>>(w, HW, scale, loss);
    }
    {
      EXM_TIMED("image_loss_blur_h", s);
      k_blur_h<<<g9, kThreads, 0, s>>>(w.dmo, tmp9, H, W, g);
    }
    {
      EXM_TIMED("image_loss_blur_v", s);
      k_blur_v<<<v9, kThreads, 0, s>>>(tmp9, w.bdmo, H, W, g);
    }
    {
      EXM_TIMED("image_loss_grad", s);
      k_img_grad<<<nblk(HW), kThreads, 0, s>>>(av, HW, scale, w, dv);
    }
  }
  return hipGetLastError();
}

hipError_t launch_tv_screen(const float* P, const int32_t* tri, int32_t n_views, int32_t H, int32_t W, int32_t metallic,
                            float scale, double* loss, float* dP, hipStream_t s) {
  TvWeights cw;
  const int32_t a[4] = {0, 3, 5, 4}, b[4] = {3, 4, 8, 5};  // A, R, N, M
  for (int c = 0; c < 8; ++c) cw.w[c] = 0.0f;
  for (int k = 0; k < (metallic ? 4 : 3); ++k)
    for (int c = a[k]; c < b[k]; ++c) cw.w[c] = scale / ((float)(b[k] - a[k]) * (float)((int64_t)H * W));
  EXM_TIMED("tv_screen", s);
  const dim3 grid(nblk(W), (unsigned)((H + kTvRows - 1) / kTvRows), (unsigned)n_views);
  k_tv_screen<<<grid, kThreads, 0, s>>>(P, tri, H, W, cw, loss, dP);
  return hipGetLastError();
}

hipError_t launch_env_regularizers(const float* E, int32_t He, int32_t We, float w_tv, float w_chroma, double* loss,
                                   double* dE, double* acc3, hipStream_t s) {
  const int64_t n = (int64_t)He * We;
  EXM_TIMED("env_regularizers", s);
  k_fill_zero_f64<<<1, 32, 0, s>>>(acc3, 3);
  k_env_sum<<<nblk(n), kThreads, 0, s>>>(E, n, acc3);
  k_env_reg<<<nblk(n), kThreads, 0, s>>>(E, He, We, w_tv, w_chroma, acc3, loss, dE);
  return hipGetLastError();
}

hipError_t launch_adam(float* prm, const void* grad, bool grad_f64, float* m, float* v, int64_t n, int32_t n_chan,
                       const float* lo, const float* hi, double lr, double b1, double b2, double eps, int32_t t,
                       hipStream_t s) {
  Bounds bd;
  for (int c = 0; c < 8; ++c) {
    bd.lo[c] = c < n_chan ? lo[c] : 0.0f;
    bd.hi[c] = c < n_chan ? hi[c] : 0.0f;
  }
  AdamCoef k;
  k.lr = (float)lr;
  k.b1 = (float)b1;
  k.b2 = (float)b2;
  k.omb1 = (float)(1.0 - b1);
  k.omb2 = (float)(1.0 - b2);
  k.eps = (float)eps;
  k.c1 = (float)(1.0 / (1.0 - pow(b1, t)));
  k.c2 = (float)(1.0 / (1.0 - pow(b2, t)));
  EXM_TIMED("adam", s);
  if (grad_f64)
    k_adam<double><<<nblk(n), kThreads, 0, s>>>(prm, static_cast<const double*>(grad), m, v, n, n_chan, bd, k);
  else
    k_adam<float><<<nblk(n), kThreads, 0, s>>>(prm, static_cast<const float*>(grad), m, v, n, n_chan, bd, k);
  return hipGetLastError();
}

}  // namespace exm
