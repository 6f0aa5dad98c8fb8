// Per-asset preparation of the fixed carrier: area-weighted vertex normals (for the
// interpolated geometry normal n_g) and per-face UV tangent frames (the tangent frame on the
// current face that carries the tangent-space normal map to world space; Attribute Query).
#include <hip/hip_runtime.h>

#include "exm_internal.h"

namespace exm {
namespace {

// sum of (P1-P0) x (P2-P0) over incident faces, accumulated in FP64
__global__ __launch_bounds__(256) void k_face_normals(int32_t nF, const float* __restrict__ pos,
                                                      const int32_t* __restrict__ tri, double* __restrict__ acc) {
  const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nF) return;
  const int32_t i0 = tri[3 * f], i1 = tri[3 * f + 1], i2 = tri[3 * f + 2];
  const double ax = pos[3 * i0], ay = pos[3 * i0 + 1], az = pos[3 * i0 + 2];
  const double e1x = pos[3 * i1] - ax, e1y = pos[3 * i1 + 1] - ay, e1z = pos[3 * i1 + 2] - az;
  const double e2x = pos[3 * i2] - ax, e2y = pos[3 * i2 + 1] - ay, e2z = pos[3 * i2 + 2] - az;
  const double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  const int32_t v[3] = {i0, i1, i2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    unsafeAtomicAdd(acc + 3 * (int64_t)v[k], nx);
    unsafeAtomicAdd(acc + 3 * (int64_t)v[k] + 1, ny);
    unsafeAtomicAdd(acc + 3 * (int64_t)v[k] + 2, nz);
  }
}

__global__ __launch_bounds__(256) void k_zero_f64(int64_t n, double* __restrict__ a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

__global__ __launch_bounds__(256) void k_vertex_normalize(int32_t nV, const double* acc, double* vnrm) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nV) return;
  const double x = acc[3 * v], y = acc[3 * v + 1], z = acc[3 * v + 2];
  const double l = sqrt(x * x + y * y + z * z);
  const double s = l > 0.0 ? 1.0 / l : 0.0;
  vnrm[3 * v] = x * s;
  vnrm[3 * v + 1] = y * s;
  vnrm[3 * v + 2] = z * s;
}

// tangent T = (e1 dv2 - e2 dv1)/det, bitangent B = (e2 du1 - e1 du2)/det,
// handedness = sign(((e1 x e2) x T) . B) (0 -> +1); |det| < 1e-20 -> T = 0
__global__ __launch_bounds__(256) void k_face_tangents(int32_t nF, const float* __restrict__ pos,
                                                       const int32_t* __restrict__ tri, const float* __restrict__ uv,
                                                       const int32_t* __restrict__ tri_uv, float4* __restrict__ ftan) {
  const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nF) return;
  const int32_t i0 = tri[3 * f], i1 = tri[3 * f + 1], i2 = tri[3 * f + 2];
  const int32_t t0 = tri_uv[3 * f], t1 = tri_uv[3 * f + 1], t2 = tri_uv[3 * f + 2];
  double e1[3], e2[3];
  for (int a = 0; a < 3; ++a) {
    e1[a] = (double)pos[3 * i1 + a] - (double)pos[3 * i0 + a];
    e2[a] = (double)pos[3 * i2 + a] - (double)pos[3 * i0 + a];
  }
  const double d1u = (double)uv[2 * t1] - uv[2 * t0], d1v = (double)uv[2 * t1 + 1] - uv[2 * t0 + 1];
  const double d2u = (double)uv[2 * t2] - uv[2 * t0], d2v = (double)uv[2 * t2 + 1] - uv[2 * t0 + 1];
  const double det = d1u * d2v - d2u * d1v;
  if (fabs(det) < 1e-20) {
    ftan[f] = make_float4(0.f, 0.f, 0.f, 1.f);
    return;
  }
  const double id = 1.0 / det;
  double T[3], B[3];
  for (int a = 0; a < 3; ++a) {
    T[a] = (e1[a] * d2v - e2[a] * d1v) * id;
    B[a] = (e2[a] * d1u - e1[a] * d2u) * id;
  }
  const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  const double nt[3] = {n[1] * T[2] - n[2] * T[1], n[2] * T[0] - n[0] * T[2], n[0] * T[1] - n[1] * T[0]};
  const double hs = nt[0] * B[0] + nt[1] * B[1] + nt[2] * B[2];
  ftan[f] = make_float4((float)T[0], (float)T[1], (float)T[2], hs < 0.0 ? -1.f : 1.f);
}

}  // namespace

// The FP64 normal sums accumulate in vnrm itself, which is then normalised in place.
hipError_t launch_mesh_prepare(const exm_mesh* m, hipStream_t s) {
  const int64_t n = 3 * (int64_t)m->nV;
  k_zero_f64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, m->vnrm);
  if (m->nF > 0) k_face_normals<<<(m->nF + 255) / 256, 256, 0, s>>>(m->nF, m->pos, m->tri, m->vnrm);
  k_vertex_normalize<<<(m->nV + 255) / 256, 256, 0, s>>>(m->nV, m->vnrm, m->vnrm);
  if (m->nF > 0)
    k_face_tangents<<<(m->nF + 255) / 256, 256, 0, s>>>(m->nF, m->pos, m->tri, m->uv, m->tri_uv,
                                                        reinterpret_cast<float4*>(m->ftan));
  return hipGetLastError();
}

}  // namespace exm
