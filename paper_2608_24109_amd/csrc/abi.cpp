// C ABI of the render pass: argument validation (before any launch), error state, view
// chunking, and BVH ownership. Every entry point returns an exm_status and only enqueues
// work on the caller's stream.
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "exm_internal.h"

namespace exm {

namespace {
thread_local std::string g_last_error;

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// gfx950 check, cached per device
std::mutex g_dev_mu;
std::vector<int> g_dev_ok;  // -1 unknown, 0 no, 1 yes

// calls still to fail on purpose (exm_inject_failures), process-wide
std::atomic<int32_t> g_inject{0};

exm_status check_device() {
  // an injected failure is taken by the first call that reaches this point, after its
  // arguments were validated and before anything is enqueued
  for (int32_t n = g_inject.load(); n > 0;)
    if (g_inject.compare_exchange_weak(n, n - 1)) return fail(EXM_E_HIP, "injected failure (exm_inject_failures)");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(EXM_E_HIP, "no current HIP device");
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if ((int)g_dev_ok.size() <= dev) g_dev_ok.resize(dev + 1, -1);
  if (g_dev_ok[dev] < 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(EXM_E_HIP, "hipGetDeviceProperties failed");
    g_dev_ok[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
  }
  if (!g_dev_ok[dev]) return fail(EXM_E_UNSUPPORTED, "device is not gfx950 (MI355X)");
  return EXM_OK;
}

exm_status check_mesh(const exm_mesh* m, bool need_prepared) {
  if (!m) return fail(EXM_E_INVAL, "mesh is NULL");
  if (m->nV <= 0 || m->nF < 0 || m->nUV <= 0) return fail(EXM_E_INVAL, "mesh sizes must be nV > 0, nF >= 0, nUV > 0");
  if (m->nF >= (1 << 27)) return fail(EXM_E_INVAL, "mesh has too many triangles (limit 2^27 - 1)");
  // per-face arrays may be NULL for a mesh without triangles
  if (!m->pos || !m->uv || (m->nF > 0 && (!m->tri || !m->tri_uv)))
    return fail(EXM_E_INVAL, "mesh array pointer is NULL");
  if (need_prepared) {
    if (!m->vnrm || (m->nF > 0 && !m->ftan)) return fail(EXM_E_INVAL, "mesh vnrm/ftan are NULL (run exm_mesh_prepare)");
    if (!aligned(m->ftan, 16) || !aligned(m->vnrm, 8)) return fail(EXM_E_INVAL, "mesh ftan must be 16-byte and vnrm 8-byte aligned");
  }
  return EXM_OK;
}

exm_status check_cams(const exm_camera* c, int32_t n) {
  if (!c) return fail(EXM_E_INVAL, "cameras are NULL");
  if (n <= 0) return fail(EXM_E_INVAL, "nViews must be > 0");
  for (int32_t i = 0; i < n; ++i) {
    if (c[i].H != c[0].H || c[i].W != c[0].W) return fail(EXM_E_INVAL, "all views of a call must share H and W");
    for (int k = 0; k < 16; ++k)
      if (!std::isfinite(c[i].mvp[k])) return fail(EXM_E_INVAL, "camera matrix is not finite");
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(c[i].eye[k])) return fail(EXM_E_INVAL, "camera eye is not finite");
  }
  if (c[0].H <= 0 || c[0].W <= 0) return fail(EXM_E_INVAL, "H and W must be > 0");
  if ((int64_t)c[0].H * c[0].W * n >= ((int64_t)1 << 31))
    return fail(EXM_E_INVAL, "nViews * H * W must be < 2^31");
  return EXM_OK;
}

exm_status check_material(const exm_material* t) {
  if (!t || !t->tex) return fail(EXM_E_INVAL, "material is NULL");
  if (t->Ht <= 0 || t->Wt <= 0 || (int64_t)t->Ht * t->Wt >= ((int64_t)1 << 31))
    return fail(EXM_E_INVAL, "material map size must be > 0 and Ht*Wt < 2^31");
  if (!aligned(t->tex, 16)) return fail(EXM_E_INVAL, "material map must be 16-byte aligned");
  return EXM_OK;
}

exm_status check_env_dims(int32_t He, int32_t We) {
  if (He < 1 || We < 2 || (int64_t)He * We > ((int64_t)1 << 24))
    return fail(EXM_E_INVAL, "env size must satisfy He >= 1, We >= 2, He*We <= 2^24");
  return EXM_OK;
}

exm_status check_env(const exm_env* e) {
  if (!e || !e->env || !e->cdf_row || !e->cdf_col || !e->pdf || !e->guide || !e->rec)
    return fail(EXM_E_INVAL, "env or its tables are NULL");
  if (!aligned(e->rec, 16) || !aligned(e->cdf_row, 8) || !aligned(e->cdf_col, 8) || !aligned(e->guide, 4))
    return fail(EXM_E_INVAL, "env tables are misaligned (rec 16 B, cdf 8 B, guide 4 B)");
  return check_env_dims(e->He, e->We);
}

exm_status check_params(const exm_params* p, bool indirect) {
  if (!p) return fail(EXM_E_INVAL, "params are NULL");
  if (p->N_d < 0 || p->N_d > 64) return fail(EXM_E_INVAL, "N_d must be in [0, 64]");
  if (indirect) {
    if (p->N_b < 0 || p->N_b > 64 || p->N_s < 0 || (int64_t)p->N_b * p->N_s > 64)
      return fail(EXM_E_INVAL, "N_b, N_s must be >= 0 with N_b <= 64 and N_b * N_s <= 64");
  }
  if (!std::isfinite(p->tmin) || p->tmin < 0.f) return fail(EXM_E_INVAL, "tmin must be finite and >= 0");
  if (!std::isfinite(p->eps) || p->eps < 0.f) return fail(EXM_E_INVAL, "eps must be finite and >= 0");
  if (!std::isfinite(p->f_diel)) return fail(EXM_E_INVAL, "f_diel must be finite");
  if (p->flags & ~0x3Fu) return fail(EXM_E_INVAL, "unknown flag bits");
  return EXM_OK;
}

exm_status check_gbuffer(const int32_t* tri_id, const float* bary) {
  if (!tri_id || !bary) return fail(EXM_E_INVAL, "G-buffer pointer is NULL");
  if (!aligned(bary, 8)) return fail(EXM_E_INVAL, "bary must be 8-byte aligned");
  return EXM_OK;
}

#define EXM_TRY(x)                        \
  do {                                    \
    exm_status _s = (x);                  \
    if (_s != EXM_OK) return _s;          \
  } while (0)

}  // namespace

ShadeViews shade_views(const exm_camera* c, int32_t first, int32_t n) {
  ShadeViews v;
  std::memset(&v, 0, sizeof(v));
  v.n = n;
  v.H = c[0].H;
  v.W = c[0].W;
  for (int32_t i = 0; i < n; ++i) {
    v.view_id[i] = c[first + i].view_id;
    for (int k = 0; k < 3; ++k) v.eye[i][k] = (float)c[first + i].eye[k];
  }
  return v;
}

exm_status fail(exm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

exm_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return EXM_OK;
}

}  // namespace exm

using namespace exm;

extern "C" {

const char* exm_last_error(void) { return g_last_error.c_str(); }

void exm_inject_failures(int32_t n) { g_inject.store(n > 0 ? n : 0); }

exm_status exm_mesh_prepare(const exm_mesh* m, hipStream_t stream) {
  EXM_TRY(check_mesh(m, true));
  EXM_TRY(check_device());
  hipError_t e = launch_mesh_prepare(m, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_mesh_prepare: ") + hipGetErrorString(e));
  return EXM_OK;
}

exm_status exm_build_bvh(const float* pos_host, int32_t nV, const int32_t* tri_host, int32_t nF, exm_bvh** out,
                         hipStream_t stream) {
  if (!out) return fail(EXM_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!pos_host || (nF > 0 && !tri_host)) return fail(EXM_E_INVAL, "host mesh arrays are NULL");
  if (nV <= 0 || nF < 0) return fail(EXM_E_INVAL, "bad mesh sizes");
  if (nF > kMaxBvhTris)
    return fail(EXM_E_UNSUPPORTED, "exm_build_bvh: more than 2^25 triangles (the BVH depth bound of the traversal stack)");
  for (int64_t i = 0; i < 3 * (int64_t)nF; ++i)
    if (tri_host[i] < 0 || tri_host[i] >= nV) return fail(EXM_E_INVAL, "triangle vertex index out of range");
  for (int64_t i = 0; i < 3 * (int64_t)nV; ++i)
    if (!std::isfinite(pos_host[i])) return fail(EXM_E_INVAL, "vertex position is not finite");
  EXM_TRY(check_device());
  HostBvh hb{};
  std::string err;
  if (!build_bvh_host(pos_host, nV, tri_host, nF, &hb, &err)) return fail(EXM_E_NOMEM, err);
  if (hb.depth > kMaxDepth) {
    free_bvh_host(&hb);
    return fail(EXM_E_UNSUPPORTED, "exm_build_bvh: BVH deeper than the traversal stack");
  }
  if (hb.depth4 > kMaxDepth4) {  // follows from the binary bound; checked because the stack relies on it
    free_bvh_host(&hb);
    return fail(EXM_E_UNSUPPORTED, "exm_build_bvh: 4-wide BVH deeper than the traversal stack");
  }
  exm_bvh* b = new exm_bvh;
  b->n_nodes = hb.n_nodes4;
  b->n_tris = hb.n_tris;
  b->depth = hb.depth;
  const size_t nb = sizeof(BvhNode4) * (size_t)std::max(1, hb.n_nodes4);
  const size_t tb = sizeof(BvhTri) * (size_t)std::max(1, hb.n_tris);
  if (hipMalloc(&b->nodes, nb) != hipSuccess || hipMalloc(&b->tris, tb) != hipSuccess) {
    if (b->nodes) (void)hipFree(b->nodes);
    free_bvh_host(&hb);
    delete b;
    (void)hipGetLastError();
    return fail(EXM_E_NOMEM, "hipMalloc of the BVH failed");
  }
  b->bytes = nb + tb;
  // synchronous copies: the host arrays are freed right after
  hipError_t e1 = hipMemcpyAsync(b->nodes, hb.nodes4, sizeof(BvhNode4) * (size_t)hb.n_nodes4, hipMemcpyHostToDevice, stream);
  hipError_t e2 = hipMemcpyAsync(b->tris, hb.tris, sizeof(BvhTri) * (size_t)hb.n_tris, hipMemcpyHostToDevice, stream);
  hipError_t e3 = hipStreamSynchronize(stream);
  free_bvh_host(&hb);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
    (void)hipFree(b->nodes);
    (void)hipFree(b->tris);
    delete b;
    return fail(EXM_E_HIP, "BVH upload failed");
  }
  *out = b;
  return EXM_OK;
}

exm_status exm_free_bvh(exm_bvh* b) {
  if (!b) return EXM_OK;
  hipError_t e1 = hipFree(b->nodes), e2 = hipFree(b->tris);
  delete b;
  if (e1 != hipSuccess || e2 != hipSuccess) return fail(EXM_E_HIP, "hipFree of the BVH failed");
  return EXM_OK;
}

size_t exm_bvh_device_bytes(const exm_bvh* b) { return b ? b->bytes : 0; }

size_t exm_env_guide_len(int32_t He, int32_t We) {
  if (He < 1 || We < 2) return 0;
  return env_guide_len(He, We);
}

exm_status exm_build_env_sampler(const float* env, int32_t He, int32_t We, uint64_t* cdf_row, uint64_t* cdf_col,
                                 float* pdf, uint32_t* guide, float* rec, hipStream_t stream) {
  if (!env || !cdf_row || !cdf_col || !pdf || !guide || !rec)
    return fail(EXM_E_INVAL, "env sampler pointer is NULL");
  EXM_TRY(check_env_dims(He, We));
  if (!aligned(pdf, 8) || !aligned(cdf_row, 8) || !aligned(cdf_col, 8) || !aligned(rec, 16) || !aligned(guide, 4))
    return fail(EXM_E_INVAL, "env tables are misaligned (cdf and pdf 8 B, rec 16 B, guide 4 B)");
  EXM_TRY(check_device());
  hipError_t e = launch_env_sampler(env, He, We, cdf_row, cdf_col, pdf, guide, rec, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_build_env_sampler: ") + hipGetErrorString(e));
  return EXM_OK;
}

exm_status exm_raster_gbuffer(const exm_mesh* m, const exm_camera* cams, int32_t nViews, int32_t* tri_id, float* bary,
                              hipStream_t stream) {
  EXM_TRY(check_mesh(m, false));
  EXM_TRY(check_cams(cams, nViews));
  EXM_TRY(check_gbuffer(tri_id, bary));
  EXM_TRY(check_device());
  const int64_t HW = (int64_t)cams[0].H * cams[0].W;
  for (int32_t v0 = 0; v0 < nViews; v0 += kViewsPerLaunch) {
    RasterViews rv;
    std::memset(&rv, 0, sizeof(rv));
    rv.n = std::min(kViewsPerLaunch, nViews - v0);
    rv.H = cams[0].H;
    rv.W = cams[0].W;
    for (int32_t i = 0; i < rv.n; ++i) std::memcpy(rv.mvp[i], cams[v0 + i].mvp, sizeof(double) * 16);
    hipError_t e = launch_raster(m, rv, tri_id + v0 * HW, bary + 2 * v0 * HW, stream);
    if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_raster_gbuffer: ") + hipGetErrorString(e));
  }
  return EXM_OK;
}

// ws == nullptr with static_scratch: the pass runs in the library's device scratch (no allocation)
static exm_status shade_fwd_impl(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat, const exm_env* env,
                                 const exm_camera* cams, int32_t nViews, const int32_t* tri_id, const float* bary,
                                 const exm_params* p, float* L_dir, uint64_t* vis, void* ws, size_t ws_bytes,
                                 uint64_t* counters, hipStream_t stream, bool static_scratch = false) {
  EXM_TRY(check_mesh(m, true));
  if (!bvh) return fail(EXM_E_INVAL, "bvh is NULL");
  EXM_TRY(check_material(mat));
  EXM_TRY(check_env(env));
  EXM_TRY(check_cams(cams, nViews));
  EXM_TRY(check_gbuffer(tri_id, bary));
  EXM_TRY(check_params(p, false));
  if (!L_dir || !vis) return fail(EXM_E_INVAL, "output pointer is NULL");
  if (static_scratch) {
    if (shade_fwd_ws_min(p->N_d) > kNoAllocScratchBytes)
      return fail(EXM_E_INVAL, "exm_shade_fwd_noalloc: the smallest pixel chunk needs more than the 64 MiB scratch");
  } else if (!ws || !aligned(ws, 256) || ws_bytes < shade_fwd_ws_min(p->N_d)) {
    return fail(EXM_E_INVAL, "workspace must be 256-byte aligned and at least exm_shade_fwd_workspace_min bytes");
  }
  EXM_TRY(check_device());
  if (static_scratch) {
    const hipError_t e = noalloc_scratch(&ws);
    if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_shade_fwd_noalloc: scratch lookup: ") + hipGetErrorString(e));
    if (!aligned(ws, 256)) return fail(EXM_E_HIP, "exm_shade_fwd_noalloc: scratch is not 256-byte aligned");
    ws_bytes = kNoAllocScratchBytes;
  }
  const int64_t HW = (int64_t)cams[0].H * cams[0].W;
  for (int32_t v0 = 0; v0 < nViews; v0 += kViewsPerLaunch) {
    const int32_t n = std::min(kViewsPerLaunch, nViews - v0);
    hipError_t e = launch_shade_fwd(m, bvh, mat, env, shade_views(cams, v0, n), tri_id + v0 * HW, bary + 2 * v0 * HW, p,
                                    L_dir + 3 * v0 * HW, vis + v0 * HW, ws, ws_bytes,
                                    reinterpret_cast<unsigned long long*>(counters), stream);
    if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_shade_fwd: ") + hipGetErrorString(e));
  }
  return EXM_OK;
}

static exm_status trace_indirect_impl(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat,
                                      const exm_env* env, const exm_camera* cams, int32_t nViews,
                                      const int32_t* tri_id, const float* bary, const exm_params* p, float* L_ind,
                                      exm_sec_rec* sec_rec, uint64_t* sec_vis, void* ws, size_t ws_bytes,
                                      uint64_t* counters, hipStream_t stream) {
  EXM_TRY(check_mesh(m, true));
  if (!bvh) return fail(EXM_E_INVAL, "bvh is NULL");
  EXM_TRY(check_material(mat));
  EXM_TRY(check_env(env));
  EXM_TRY(check_cams(cams, nViews));
  EXM_TRY(check_gbuffer(tri_id, bary));
  EXM_TRY(check_params(p, true));
  if (!L_ind || !sec_vis || (!sec_rec && p->N_b > 0)) return fail(EXM_E_INVAL, "output pointer is NULL");
  if (!ws || !aligned(ws, 256) || ws_bytes < trace_indirect_ws_min(p->N_b, p->N_s))
    return fail(EXM_E_INVAL, "workspace must be 256-byte aligned and at least exm_trace_indirect_workspace_min bytes");
  EXM_TRY(check_device());
  const int64_t HW = (int64_t)cams[0].H * cams[0].W;
  for (int32_t v0 = 0; v0 < nViews; v0 += kViewsPerLaunch) {
    const int32_t n = std::min(kViewsPerLaunch, nViews - v0);
    hipError_t e = launch_trace_indirect(m, bvh, mat, env, shade_views(cams, v0, n), tri_id + v0 * HW,
                                         bary + 2 * v0 * HW, p, L_ind + 3 * v0 * HW,
                                         sec_rec ? sec_rec + v0 * HW * p->N_b : nullptr, sec_vis + v0 * HW, ws,
                                         ws_bytes, reinterpret_cast<unsigned long long*>(counters), stream);
    if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_trace_indirect: ") + hipGetErrorString(e));
  }
  return EXM_OK;
}

size_t exm_shade_fwd_workspace_size(int32_t nViews, int32_t H, int32_t W, int32_t N_d) {
  if (nViews <= 0 || H <= 0 || W <= 0 || N_d < 0 || N_d > 64) return 0;
  return shade_fwd_ws_bytes((int64_t)std::min(nViews, kViewsPerLaunch) * H * W, N_d);
}

size_t exm_shade_fwd_workspace_min(int32_t N_d) { return (N_d < 0 || N_d > 64) ? 0 : shade_fwd_ws_min(N_d); }

exm_status exm_shade_fwd(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat, const exm_env* env,
                         const exm_camera* cams, int32_t nViews, const int32_t* tri_id, const float* bary,
                         const exm_params* p, float* L_dir, uint64_t* vis, void* ws, size_t ws_bytes,
                         hipStream_t stream) {
  return shade_fwd_impl(m, bvh, mat, env, cams, nViews, tri_id, bary, p, L_dir, vis, ws, ws_bytes, nullptr, stream);
}

size_t exm_shade_fwd_batch_workspace_size(const exm_request* reqs, int32_t n_req, int32_t N_d) {
  if (!reqs || n_req <= 0 || N_d < 0 || N_d > 64) return 0;
  for (int32_t i = 0; i < n_req; ++i)
    if (reqs[i].cam.H <= 0 || reqs[i].cam.W <= 0 || (int64_t)reqs[i].cam.H * reqs[i].cam.W > ((int64_t)1 << 26)) return 0;
  return shade_fwd_batch_ws_bytes(reqs, n_req, N_d);
}

exm_status exm_shade_fwd_batch(const exm_request* reqs, int32_t n_req, const exm_params* p, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
  if (!reqs || n_req <= 0) return fail(EXM_E_INVAL, "exm_shade_fwd_batch: no requests");
  EXM_TRY(check_params(p, false));
  for (int32_t i = 0; i < n_req; ++i) {
    const exm_request& r = reqs[i];
    EXM_TRY(check_mesh(r.mesh, true));
    if (!r.bvh) return fail(EXM_E_INVAL, "exm_shade_fwd_batch: bvh is NULL");
    EXM_TRY(check_material(r.mat));
    EXM_TRY(check_env(r.env));
    EXM_TRY(check_cams(&r.cam, 1));
    if ((int64_t)r.cam.H * r.cam.W > ((int64_t)1 << 26)) return fail(EXM_E_INVAL, "exm_shade_fwd_batch: view too large");
    EXM_TRY(check_gbuffer(r.tri_id, r.bary));
    if (!r.L_dir || !r.vis) return fail(EXM_E_INVAL, "exm_shade_fwd_batch: output pointer is NULL");
    if (!std::isfinite(r.tmin) || r.tmin < 0.f) return fail(EXM_E_INVAL, "exm_shade_fwd_batch: tmin must be finite and >= 0");
  }
  if (!ws || !aligned(ws, 256) || ws_bytes < shade_fwd_batch_ws_bytes(reqs, n_req, p->N_d))
    return fail(EXM_E_INVAL, "workspace must be 256-byte aligned and at least exm_shade_fwd_batch_workspace_size bytes");
  EXM_TRY(check_device());
  for (int32_t i0 = 0; i0 < n_req; i0 += kMaxFrames) {
    const int32_t n = std::min(kMaxFrames, n_req - i0);
    const hipError_t e = launch_shade_fwd_batch(reqs + i0, n, p, ws, ws_bytes, nullptr, stream);
    if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_shade_fwd_batch: ") + hipGetErrorString(e));
  }
  return EXM_OK;
}

exm_status exm_shade_fwd_noalloc(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat, const exm_env* env,
                                 const exm_camera* cams, int32_t nViews, const int32_t* tri_id, const float* bary,
                                 const exm_params* p, float* L_dir, uint64_t* vis, hipStream_t stream) {
  return shade_fwd_impl(m, bvh, mat, env, cams, nViews, tri_id, bary, p, L_dir, vis, nullptr, 0, nullptr, stream, true);
}

exm_status exm_shade_fwd_counted(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat, const exm_env* env,
                                 const exm_camera* cams, int32_t nViews, const int32_t* tri_id, const float* bary,
                                 const exm_params* p, float* L_dir, uint64_t* vis, void* ws, size_t ws_bytes,
                                 uint64_t* counters, hipStream_t stream) {
  if (!counters || !aligned(counters, 8)) return fail(EXM_E_INVAL, "counters must be an 8-byte aligned device array");
  return shade_fwd_impl(m, bvh, mat, env, cams, nViews, tri_id, bary, p, L_dir, vis, ws, ws_bytes, counters, stream);
}

size_t exm_trace_indirect_workspace_size(int32_t nViews, int32_t H, int32_t W, int32_t N_b, int32_t N_s) {
  if (nViews <= 0 || H <= 0 || W <= 0 || N_b < 0 || N_s < 0 || (int64_t)N_b * N_s > 64 || N_b > 64) return 0;
  return trace_indirect_ws_bytes((int64_t)std::min(nViews, kViewsPerLaunch) * H * W, N_b, N_s);
}

size_t exm_trace_indirect_workspace_min(int32_t N_b, int32_t N_s) {
  if (N_b < 0 || N_s < 0 || (int64_t)N_b * N_s > 64 || N_b > 64) return 0;
  return trace_indirect_ws_min(N_b, N_s);
}

exm_status exm_trace_indirect(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat, const exm_env* env,
                              const exm_camera* cams, int32_t nViews, const int32_t* tri_id, const float* bary,
                              const exm_params* p, float* L_ind, exm_sec_rec* sec_rec, uint64_t* sec_vis, void* ws,
                              size_t ws_bytes, hipStream_t stream) {
  return trace_indirect_impl(m, bvh, mat, env, cams, nViews, tri_id, bary, p, L_ind, sec_rec, sec_vis, ws, ws_bytes,
                             nullptr, stream);
}

exm_status exm_trace_indirect_counted(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat,
                                      const exm_env* env, const exm_camera* cams, int32_t nViews,
                                      const int32_t* tri_id, const float* bary, const exm_params* p, float* L_ind,
                                      exm_sec_rec* sec_rec, uint64_t* sec_vis, void* ws, size_t ws_bytes,
                                      uint64_t* counters, hipStream_t stream) {
  if (!counters || !aligned(counters, 8)) return fail(EXM_E_INVAL, "counters must be an 8-byte aligned device array");
  return trace_indirect_impl(m, bvh, mat, env, cams, nViews, tri_id, bary, p, L_ind, sec_rec, sec_vis, ws, ws_bytes,
                             counters, stream);
}

size_t exm_shade_bwd_workspace_size(int32_t nViews, int32_t H, int32_t W, int32_t N_d, int32_t He, int32_t We) {
  if (nViews <= 0 || H <= 0 || W <= 0 || N_d < 0 || N_d > 64 || He < 1 || We < 2) return 0;
  const int32_t n = std::min(nViews, kViewsPerLaunch);
  return shade_bwd_ws_bytes((int64_t)n * H * W, N_d, He, We);
}

size_t exm_shade_bwd_workspace_min(int32_t N_d, int32_t He, int32_t We) {
  if (N_d < 0 || N_d > 64 || He < 1 || We < 2) return 0;
  return shade_bwd_ws_min(N_d, He, We);
}

size_t exm_trace_bwd_workspace_size(int32_t nViews, int32_t H, int32_t W, int32_t N_b, int32_t N_s, int32_t He,
                                    int32_t We) {
  if (nViews <= 0 || H <= 0 || W <= 0 || N_b < 0 || N_s < 0 || (int64_t)N_b * N_s > 64 || He < 1 || We < 2) return 0;
  const int32_t n = std::min(nViews, kViewsPerLaunch);
  return trace_bwd_ws_bytes((int64_t)n * H * W, N_b, N_s, He, We);
}

size_t exm_trace_bwd_workspace_min(int32_t N_b, int32_t N_s, int32_t He, int32_t We) {
  if (N_b < 0 || N_s < 0 || (int64_t)N_b * N_s > 64 || He < 1 || We < 2) return 0;
  return trace_bwd_ws_min(N_b, N_s, He, We);
}

exm_status exm_shade_bwd(const exm_mesh* m, const exm_material* mat, const exm_env* env, const exm_camera* cams,
                         int32_t nViews, const int32_t* tri_id, const float* bary, const exm_params* p, const float* dI,
                         const uint64_t* vis, const float* dquery, float* dtex, double* denv, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
  EXM_TRY(check_mesh(m, true));
  EXM_TRY(check_material(mat));
  EXM_TRY(check_env(env));
  EXM_TRY(check_cams(cams, nViews));
  EXM_TRY(check_gbuffer(tri_id, bary));
  EXM_TRY(check_params(p, false));
  if (!dI || !vis || !dtex || !denv) return fail(EXM_E_INVAL, "gradient pointer is NULL");
  if (dquery && !aligned(dquery, 16)) return fail(EXM_E_INVAL, "dquery must be 16-byte aligned");
  if (!aligned(dtex, 16)) return fail(EXM_E_INVAL, "dtex must be 16-byte aligned");
  if (!ws || !aligned(ws, 256) || ws_bytes < shade_bwd_ws_min(p->N_d, env->He, env->We))
    return fail(EXM_E_INVAL, "workspace must be 256-byte aligned and at least exm_shade_bwd_workspace_min bytes");
  EXM_TRY(check_device());
  const int64_t HW = (int64_t)cams[0].H * cams[0].W;
  for (int32_t v0 = 0; v0 < nViews; v0 += kViewsPerLaunch) {
    const int32_t n = std::min(kViewsPerLaunch, nViews - v0);
    hipError_t e = launch_shade_bwd(m, mat, env, shade_views(cams, v0, n), tri_id + v0 * HW, bary + 2 * v0 * HW, p,
                                    dI + 3 * v0 * HW, vis + v0 * HW, dquery ? dquery + 8 * v0 * HW : nullptr, dtex,
                                    denv, ws, ws_bytes, stream);
    if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_shade_bwd: ") + hipGetErrorString(e));
  }
  return EXM_OK;
}

exm_status exm_trace_bwd(const exm_mesh* m, const exm_material* mat, const exm_env* env, const exm_camera* cams,
                         int32_t nViews, const int32_t* tri_id, const float* bary, const exm_params* p,
                         float lambda_ind, const float* dI, const exm_sec_rec* sec_rec, const uint64_t* sec_vis,
                         float* dtex, double* denv, void* ws, size_t ws_bytes, hipStream_t stream) {
  EXM_TRY(check_mesh(m, true));
  EXM_TRY(check_material(mat));
  EXM_TRY(check_env(env));
  EXM_TRY(check_cams(cams, nViews));
  EXM_TRY(check_gbuffer(tri_id, bary));
  EXM_TRY(check_params(p, true));
  if (!std::isfinite(lambda_ind)) return fail(EXM_E_INVAL, "lambda_ind must be finite");
  if (!dI || !sec_vis || !dtex || !denv || (!sec_rec && p->N_b > 0)) return fail(EXM_E_INVAL, "pointer is NULL");
  if (!ws || !aligned(ws, 256) || ws_bytes < trace_bwd_ws_min(p->N_b, p->N_s, env->He, env->We))
    return fail(EXM_E_INVAL, "workspace must be 256-byte aligned and at least exm_trace_bwd_workspace_min bytes");
  EXM_TRY(check_device());
  const int64_t HW = (int64_t)cams[0].H * cams[0].W;
  for (int32_t v0 = 0; v0 < nViews; v0 += kViewsPerLaunch) {
    const int32_t n = std::min(kViewsPerLaunch, nViews - v0);
    hipError_t e = launch_trace_bwd(m, mat, env, shade_views(cams, v0, n), tri_id + v0 * HW, bary + 2 * v0 * HW, p,
                                    lambda_ind, dI + 3 * v0 * HW, sec_rec ? sec_rec + v0 * HW * p->N_b : nullptr,
                                    sec_vis + v0 * HW, dtex, denv, ws, ws_bytes, stream);
    if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_trace_bwd: ") + hipGetErrorString(e));
  }
  return EXM_OK;
}

static exm_status check_upsample(const int32_t* tri_h, int32_t Hh, int32_t Wh, const int32_t* tri, int32_t H,
                                 int32_t W, int32_t n) {
  if (!tri_h || !tri) return fail(EXM_E_INVAL, "G-buffer pointer is NULL");
  if (n < 1 || H < 1 || W < 1 || Hh < 1 || Wh < 1 || Hh > H || Wh > W || (int64_t)H * W > (1 << 26))
    return fail(EXM_E_INVAL, "need 1 <= Hh <= H, 1 <= Wh <= W, nViews >= 1 and H * W <= 2^26");
  return EXM_OK;
}

exm_status exm_upsample_indirect(const int32_t* tri_h, int32_t Hh, int32_t Wh, const float* L_half, const int32_t* tri,
                                 int32_t H, int32_t W, int32_t n, float* L_ind, hipStream_t stream) {
  EXM_TRY(check_upsample(tri_h, Hh, Wh, tri, H, W, n));
  if (!L_half || !L_ind) return fail(EXM_E_INVAL, "radiance pointer is NULL");
  EXM_TRY(check_device());
  hipError_t e = launch_upsample(tri_h, Hh, Wh, L_half, tri, H, W, n, L_ind, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_upsample_indirect: ") + hipGetErrorString(e));
  return EXM_OK;
}

exm_status exm_upsample_indirect_bwd(const int32_t* tri_h, int32_t Hh, int32_t Wh, const int32_t* tri, int32_t H,
                                     int32_t W, int32_t n, float lambda_ind, const float* dI, float* dL_half,
                                     hipStream_t stream) {
  EXM_TRY(check_upsample(tri_h, Hh, Wh, tri, H, W, n));
  if (!dI || !dL_half) return fail(EXM_E_INVAL, "gradient pointer is NULL");
  if (!std::isfinite(lambda_ind)) return fail(EXM_E_INVAL, "lambda_ind must be finite");
  EXM_TRY(check_device());
  hipError_t e = launch_upsample_bwd(tri_h, Hh, Wh, tri, H, W, n, lambda_ind, dI, dL_half, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_upsample_indirect_bwd: ") + hipGetErrorString(e));
  return EXM_OK;
}

static exm_status check_view_dims(int32_t n, int32_t H, int32_t W) {
  if (n < 1 || H < 1 || W < 1 || (int64_t)H * W > (1 << 26)) return fail(EXM_E_INVAL, "bad view dimensions");
  return EXM_OK;
}

exm_status exm_project_maps(const exm_mesh* m, const exm_material* mat, int32_t n, int32_t H, int32_t W,
                            const int32_t* tri_id, const float* bary, float* P, hipStream_t stream) {
  EXM_TRY(check_mesh(m, true));
  EXM_TRY(check_material(mat));
  EXM_TRY(check_view_dims(n, H, W));
  EXM_TRY(check_gbuffer(tri_id, bary));
  if (!P || !aligned(P, 16)) return fail(EXM_E_INVAL, "P must be a 16-byte aligned device pointer");
  EXM_TRY(check_device());
  hipError_t e = launch_project(m, mat, (int64_t)n * H * W, tri_id, bary, P, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_project_maps: ") + hipGetErrorString(e));
  return EXM_OK;
}

exm_status exm_project_maps_bwd(const exm_mesh* m, const exm_material* mat, int32_t n, int32_t H, int32_t W,
                                const int32_t* tri_id, const float* bary, const float* dP, float* dtex,
                                hipStream_t stream) {
  EXM_TRY(check_mesh(m, true));
  EXM_TRY(check_material(mat));
  EXM_TRY(check_view_dims(n, H, W));
  EXM_TRY(check_gbuffer(tri_id, bary));
  if (!dP || !dtex) return fail(EXM_E_INVAL, "gradient pointer is NULL");
  EXM_TRY(check_device());
  hipError_t e = launch_project_bwd(m, mat, (int64_t)n * H * W, tri_id, bary, dP, dtex, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_project_maps_bwd: ") + hipGetErrorString(e));
  return EXM_OK;
}

size_t exm_image_loss_workspace_size(int32_t H, int32_t W) {
  if (H < 1 || W < 1 || (int64_t)H * W > (1 << 26)) return 0;
  return image_loss_ws_bytes(H, W);
}

exm_status exm_image_loss(const float* a, const float* b, int32_t n, int32_t H, int32_t W, float scale, double* loss,
                          float* dA, void* ws, size_t ws_bytes, hipStream_t stream) {
  EXM_TRY(check_view_dims(n, H, W));
  if (H > 65535) return fail(EXM_E_INVAL, "H must be at most 65535");
  if (!a || !b || !loss || !dA) return fail(EXM_E_INVAL, "pointer is NULL");
  if (!std::isfinite(scale)) return fail(EXM_E_INVAL, "scale must be finite");
  if (!ws || !aligned(ws, 256) || ws_bytes < image_loss_ws_bytes(H, W))
    return fail(EXM_E_INVAL, "workspace must be 256-byte aligned and at least exm_image_loss_workspace_size bytes");
  EXM_TRY(check_device());
  hipError_t e = launch_image_loss(a, b, n, H, W, scale, loss, dA, ws, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_image_loss: ") + hipGetErrorString(e));
  return EXM_OK;
}

exm_status exm_tv_screen(const float* P, const int32_t* tri_id, int32_t n, int32_t H, int32_t W, int32_t metallic,
                         float scale, double* loss, float* dP, hipStream_t stream) {
  EXM_TRY(check_view_dims(n, H, W));
  if (n > 65535) return fail(EXM_E_INVAL, "at most 65535 views per call");
  if (!P || !tri_id || !loss || !dP) return fail(EXM_E_INVAL, "pointer is NULL");
  if (!aligned(dP, 16) || !aligned(P, 16)) return fail(EXM_E_INVAL, "P and dP must be 16-byte aligned");
  if (!std::isfinite(scale)) return fail(EXM_E_INVAL, "scale must be finite");
  EXM_TRY(check_device());
  hipError_t e = launch_tv_screen(P, tri_id, n, H, W, metallic, scale, loss, dP, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_tv_screen: ") + hipGetErrorString(e));
  return EXM_OK;
}

exm_status exm_env_regularizers(const float* E, int32_t He, int32_t We, float w_tv, float w_chroma, double* loss,
                                double* dE, double* acc3, hipStream_t stream) {
  EXM_TRY(check_env_dims(He, We));
  if (!E || !loss || !dE || !acc3) return fail(EXM_E_INVAL, "pointer is NULL");
  if (!std::isfinite(w_tv) || !std::isfinite(w_chroma)) return fail(EXM_E_INVAL, "weights must be finite");
  EXM_TRY(check_device());
  hipError_t e = launch_env_regularizers(E, He, We, w_tv, w_chroma, loss, dE, acc3, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_env_regularizers: ") + hipGetErrorString(e));
  return EXM_OK;
}

exm_status exm_adam_step(float* prm, const void* grad, int32_t grad_is_f64, float* m, float* v, int64_t n,
                         int32_t n_chan, const float* lo, const float* hi, double lr, double b1, double b2, double eps,
                         int32_t t, hipStream_t stream) {
  if (!prm || !grad || !m || !v || !lo || !hi) return fail(EXM_E_INVAL, "pointer is NULL");
  if (n < 0 || n_chan < 1 || n_chan > 8 || n % n_chan != 0) return fail(EXM_E_INVAL, "n must be a multiple of n_chan <= 8");
  if (t < 1 || !(b1 >= 0.0 && b1 < 1.0) || !(b2 >= 0.0 && b2 < 1.0) || !(eps > 0.0) || !std::isfinite(lr))
    return fail(EXM_E_INVAL, "need t >= 1, 0 <= beta < 1, eps > 0, finite lr");
  for (int32_t c = 0; c < n_chan; ++c)
    if (!(lo[c] <= hi[c])) return fail(EXM_E_INVAL, "bounds need lo <= hi");
  if (n == 0) return EXM_OK;
  EXM_TRY(check_device());
  hipError_t e = launch_adam(prm, grad, grad_is_f64 != 0, m, v, n, n_chan, lo, hi, lr, b1, b2, eps, t, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_adam_step: ") + hipGetErrorString(e));
  return EXM_OK;
}

static exm_status check_topo_params(const exm_topo_params* p) {
  if (!p) return fail(EXM_E_INVAL, "params pointer is NULL");
  if (!(p->beta_g >= 0.0 && p->beta_g <= 1.0) || !std::isfinite(p->w_g) || !std::isfinite(p->w_k) ||
      !std::isfinite(p->tau_degen) || !(p->tau_uv >= 0.0 && std::isfinite(p->tau_uv)) ||
      !(p->split_fraction >= 0.0 && p->split_fraction <= 1.0) || p->max_faces < 0 || (p->flags & ~3u))
    return fail(EXM_E_INVAL, "topology params out of range");
  return EXM_OK;
}

static exm_status check_topo_mesh(const exm_topo_mesh* m) {
  if (!m || !m->pos || !m->G || !m->uv || !m->tri || !m->tri_uv) return fail(EXM_E_INVAL, "mesh pointer is NULL");
  if (m->nV < 0 || m->nF < 0 || m->nUV < 0 || m->nF > (1 << 26) || m->nV > (1 << 26) || m->nUV > (1 << 27))
    return fail(EXM_E_INVAL, "mesh counts out of range");
  if (m->nV > m->capV || m->nF > m->capF || m->nUV > m->capUV) return fail(EXM_E_INVAL, "counts exceed capacities");
  if (m->nF > 0 && (m->nV < 3 || m->nUV < 1)) return fail(EXM_E_INVAL, "faces need vertices and UVs");
  return EXM_OK;
}

exm_status exm_vertex_grad_ema(float* G, const float* grad, int32_t nV, double beta, hipStream_t stream) {
  if (!G || !grad) return fail(EXM_E_INVAL, "pointer is NULL");
  if (nV < 0 || !(beta >= 0.0 && beta <= 1.0)) return fail(EXM_E_INVAL, "need nV >= 0 and 0 <= beta <= 1");
  if (nV == 0) return EXM_OK;
  EXM_TRY(check_device());
  hipError_t e = launch_grad_ema(G, grad, nV, beta, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_vertex_grad_ema: ") + hipGetErrorString(e));
  return EXM_OK;
}

exm_status exm_face_render_counts(const int32_t* tri_id, int64_t n_px, int32_t nF, int32_t* counts,
                                  hipStream_t stream) {
  if (!tri_id || !counts) return fail(EXM_E_INVAL, "pointer is NULL");
  if (n_px < 0 || nF < 0) return fail(EXM_E_INVAL, "negative size");
  if (n_px == 0) return EXM_OK;
  EXM_TRY(check_device());
  hipError_t e = launch_face_counts(tri_id, n_px, nF, counts, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_face_render_counts: ") + hipGetErrorString(e));
  return EXM_OK;
}

size_t exm_topology_workspace_size(int32_t nV, int32_t nF, int32_t nUV, const exm_topo_params* p) {
  if (!p || nV < 0 || nF < 0 || nUV < 0) return 0;
  return topology_ws_bytes(nV, nF, nUV, p);
}

exm_status exm_topology_scores(const exm_topo_mesh* m, const exm_topo_params* p, double* S, double* K, double* D,
                               double* area, void* ws, size_t ws_bytes, hipStream_t stream) {
  EXM_TRY(check_topo_mesh(m));
  EXM_TRY(check_topo_params(p));
  if (!S || !K || !D || !area || !ws) return fail(EXM_E_INVAL, "output or workspace pointer is NULL");
  if (ws_bytes < topology_ws_bytes(m->nV, m->nF, m->nUV, p)) return fail(EXM_E_NOMEM, "workspace too small");
  if (!aligned(ws, 256)) return fail(EXM_E_INVAL, "workspace must be 256-byte aligned");
  EXM_TRY(check_device());
  bool ok = true;
  hipError_t e = topology_check_indices(m, ws, &ok, stream);
  if (e == hipSuccess && !ok) return fail(EXM_E_INVAL, "a face or UV index is out of range");
  if (e == hipSuccess) e = launch_topology_scores(m, p, S, K, D, area, ws, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_topology_scores: ") + hipGetErrorString(e));
  return EXM_OK;
}

exm_status exm_topology_round(exm_topo_mesh* m, const int32_t* c_rend, const exm_topo_params* p, void* ws,
                              size_t ws_bytes, exm_topo_stats* stats, hipStream_t stream) {
  EXM_TRY(check_topo_mesh(m));
  EXM_TRY(check_topo_params(p));
  if (!ws || !stats) return fail(EXM_E_INVAL, "workspace or stats pointer is NULL");
  const int64_t K = topology_split_count(m->nF, p);
  if ((int64_t)m->nV + K > m->capV || (int64_t)m->nF + 2 * K > m->capF || (int64_t)m->nUV + 2 * K > m->capUV)
    return fail(EXM_E_INVAL, "capacities must hold nV + K vertices, nF + 2K faces and nUV + 2K UVs");
  if (ws_bytes < topology_ws_bytes(m->nV, m->nF, m->nUV, p)) return fail(EXM_E_NOMEM, "workspace too small");
  if (!aligned(ws, 256)) return fail(EXM_E_INVAL, "workspace must be 256-byte aligned");
  EXM_TRY(check_device());
  bool ok = true;
  hipError_t e = topology_check_indices(m, ws, &ok, stream);
  if (e == hipSuccess && !ok) return fail(EXM_E_INVAL, "a face or UV index is out of range");
  if (e == hipSuccess) e = launch_topology_round(m, c_rend, p, ws, stats, stream);
  if (e != hipSuccess) return fail(EXM_E_HIP, std::string("exm_topology_round: ") + hipGetErrorString(e));
  return EXM_OK;
}

}  // extern "C"
