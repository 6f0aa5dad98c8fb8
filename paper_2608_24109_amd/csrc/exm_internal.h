// Internal declarations shared by the host ABI layer and the kernel files.
#pragma once
#include <stdint.h>

#include <string>

#include "../../include/exm.h"

namespace exm {

// 64-byte BVH2 node: boxes of both children and their references.
//   ref >= 0              internal node index
//   ref <  0, != INT_MIN  leaf: v = ~ref, triangles [v >> 4, (v >> 4) + (v & 15))
//   ref == INT_MIN        empty
struct alignas(64) BvhNode {
  float lo0[3], hi0[3];
  float lo1[3], hi1[3];
  int32_t c0, c1;
  int32_t pad[2];
};
static_assert(sizeof(BvhNode) == 64, "node layout");

// 128-byte 4-wide node (one cache line) for the traversal: the child boxes by axis, so that seven
// 16-byte loads fetch the node, then the child references (internal: node index; leaf:
// ~(first * 16 + count) into the triangle records; empty slot: kEmptyChild). Collapsed from the
// binary tree two levels at a time, so a tree of depth <= kMaxDepth gives 4-wide depth <= 12.
struct alignas(128) BvhNode4 {
  float lo_x[4], lo_y[4], lo_z[4];
  float hi_x[4], hi_y[4], hi_z[4];
  int32_t child[4];
  int32_t pad[4];
};
static_assert(sizeof(BvhNode4) == 128, "wide node layout");
constexpr int32_t kEmptyChild = (int32_t)0x80000000;

// 48-byte triangle record in leaf order (vertices copied, original id kept)
struct alignas(16) BvhTri {
  float v0[3], v1[3], v2[3];
  int32_t id;
  int32_t pad[2];
};
static_assert(sizeof(BvhTri) == 48, "triangle layout");

constexpr int kMaxDepth = 24;  // builder guarantee for the binary tree
constexpr int kMaxDepth4 = (kMaxDepth + 1) / 2;  // of the 4-wide tree collapsed from it
// the traversal defers at most three children per 4-wide node on its path: 36 references plus the
// bottom sentinel; the first kStackLds entries live in LDS (25 KB per 256-lane block, so six
// blocks fit a CU), the rest, which only deep stacks reach, in a per-lane private array
constexpr int kStack = 3 * kMaxDepth4 + 1;
constexpr int kStackLds = 25;
constexpr int kStackOvf = kStack - kStackLds;
// The builder's depth bound holds while need(nF) <= kMaxDepth, i.e. for at most 2 * 2^kMaxDepth
// triangles (2^25); larger meshes would put leaves below the bound and overflow the stack.
constexpr int64_t kMaxBvhTris = (int64_t)2 << kMaxDepth;

// Views per launch: camera data travels in kernel arguments.
constexpr int kViewsPerLaunch = 8;
// Requests per launch of a batched pass (their descriptors travel in kernel arguments too).
constexpr int kMaxFrames = 8;

struct RasterViews {
  int32_t n, H, W;
  double mvp[kViewsPerLaunch][16];
};

struct ShadeViews {
  int32_t n, H, W;
  int32_t view_id[kViewsPerLaunch];
  float eye[kViewsPerLaunch][3];
};

}  // namespace exm

struct exm_bvh {
  exm::BvhNode4* nodes = nullptr;  // 4-wide nodes, root at 0
  exm::BvhTri* tris = nullptr;
  int32_t n_nodes = 0, n_tris = 0;
  int32_t depth = 0;  // of the binary tree it was collapsed from
  size_t bytes = 0;
};

namespace exm {

// Layout of the cutpoint ("guide") tables. A CDF a[0..n) with total T = a[n-1] is cut into at
// most n buckets of 2^s keys, s the smallest shift with (T - 1) >> s < n; entry g holds the
// first index whose CDF value exceeds g << s (clamped to n - 1), for g in [0, n]. A key t in
// bucket g = t >> s then has its answer in [entry g, entry g + 1], so the search runs over
// that range only and returns the same index as a search over the whole array.
//   guide[0]                          row shift
//   guide[1 .. He + 1]                row entries
//   guide[He + 2 .. 2 He + 2)         shift of each row's column CDF
//   guide[2 He + 2 + i (We + 1) + g]  column entries of row i
// and, when We < kCdf32MaxW (a row total is at most We * 2^20 < 2^32), compact copies that the
// pick reads instead (fewer bytes per probe, tables that fit an L2 together):
//   guide[He (We + 3) + 2 + i We + j]               cdf_col[i][j] as 32 bits
//   16-bit entry i (We + 1) + g of the words after  column entry g of row i
//   16-bit entry i We + j of the words after        (cdf_col[i][j] - 1) mod 2^16
// The last table decides a probe of a row whose column shift s is at most 16 on its own: a probe
// inside key t's bucket g = t >> s reads a value c with g 2^s < c <= (g + 1) 2^s, so c <= t holds
// exactly when (c - 1) mod 2^s < t mod 2^s.
constexpr int32_t kCdf32MaxW = 4096;
__host__ __device__ inline size_t env_cdf32_offset(int32_t He, int32_t We) { return (size_t)He * (size_t)(We + 3) + 2; }
__host__ __device__ inline size_t env_col16_offset(int32_t He, int32_t We) {
  return env_cdf32_offset(He, We) + (size_t)He * (size_t)We;
}
__host__ __device__ inline size_t env_cdf16_offset(int32_t He, int32_t We) {
  return env_col16_offset(He, We) + ((size_t)He * (size_t)(We + 1) + 1) / 2;
}
inline size_t env_guide_len(int32_t He, int32_t We) {
  if (We >= kCdf32MaxW) return env_cdf32_offset(He, We);
  return env_cdf16_offset(He, We) + ((size_t)He * (size_t)We + 1) / 2;
}

// Brackets one kernel launch with HIP events on its stream when timing is enabled
// (exm_timing_enable); names are string literals.
class KernelTimer {
 public:
  KernelTimer(const char* name, hipStream_t s);
  ~KernelTimer();
  KernelTimer(const KernelTimer&) = delete;
  KernelTimer& operator=(const KernelTimer&) = delete;

 private:
  const char* name_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr;
};
#define EXM_TIMED(name, stream) ::exm::KernelTimer exm_kernel_timer_(name, stream)

// error reporting (thread-local last error)
exm_status fail(exm_status s, const std::string& msg);
exm_status check_launch(const char* what);

// host launchers (defined in the .hip files); arguments already validated
hipError_t launch_mesh_prepare(const exm_mesh* m, hipStream_t s);
hipError_t launch_env_sampler(const float* env, int32_t He, int32_t We, uint64_t* cdf_row, uint64_t* cdf_col,
                              float* pdf, uint32_t* guide, float* rec, hipStream_t s);
hipError_t launch_upsample(const int32_t* tri_half, int32_t Hh, int32_t Wh, const float* L_half, const int32_t* tri_id,
                           int32_t H, int32_t W, int32_t n_views, float* L, hipStream_t s);
hipError_t launch_upsample_bwd(const int32_t* tri_half, int32_t Hh, int32_t Wh, const int32_t* tri_id, int32_t H,
                               int32_t W, int32_t n_views, float lambda, const float* dI, float* dL_half,
                               hipStream_t s);
size_t image_loss_ws_bytes(int32_t H, int32_t W);
hipError_t launch_project(const exm_mesh* m, const exm_material* mat, int64_t n_px, const int32_t* tri_id,
                          const float* bary, float* P, hipStream_t s);
hipError_t launch_project_bwd(const exm_mesh* m, const exm_material* mat, int64_t n_px, const int32_t* tri_id,
                              const float* bary, const float* dP, float* dtex, hipStream_t s);
hipError_t launch_image_loss(const float* a, const float* b, int32_t n_views, int32_t H, int32_t W, float scale,
                             double* loss, float* dA, void* ws, hipStream_t s);
hipError_t launch_tv_screen(const float* P, const int32_t* tri, int32_t n_views, int32_t H, int32_t W, int32_t metallic,
                            float scale, double* loss, float* dP, hipStream_t s);
hipError_t launch_env_regularizers(const float* E, int32_t He, int32_t We, float w_tv, float w_chroma, double* loss,
                                   double* dE, double* acc3, hipStream_t s);
hipError_t launch_adam(float* prm, const void* grad, bool grad_f64, float* m, float* v, int64_t n, int32_t n_chan,
                       const float* lo, const float* hi, double lr, double b1, double b2, double eps, int32_t t,
                       hipStream_t s);
hipError_t launch_raster(const exm_mesh* m, const RasterViews& v, int32_t* tri_id, float* bary, hipStream_t s);
int32_t topology_split_count(int32_t nF, const exm_topo_params* p);
hipError_t topology_check_indices(const exm_topo_mesh* m, void* ws, bool* ok, hipStream_t s);
size_t topology_ws_bytes(int32_t nV, int32_t nF, int32_t nUV, const exm_topo_params* p);
hipError_t launch_grad_ema(float* G, const float* grad, int32_t nV, double beta, hipStream_t s);
hipError_t launch_face_counts(const int32_t* tri_id, int64_t n_px, int32_t nF, int32_t* counts, hipStream_t s);
hipError_t launch_topology_scores(const exm_topo_mesh* m, const exm_topo_params* p, double* S, double* K, double* D,
                                  double* area, void* ws, hipStream_t s);
hipError_t launch_topology_round(exm_topo_mesh* m, const int32_t* c_rend, const exm_topo_params* p, void* ws,
                                 exm_topo_stats* st, hipStream_t s);
hipError_t launch_shade_fwd(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat, const exm_env* env,
                            const ShadeViews& v, const int32_t* tri_id, const float* bary, const exm_params* p,
                            float* L_dir, uint64_t* vis, void* ws, size_t ws_bytes, unsigned long long* counters,
                            hipStream_t s);
size_t shade_fwd_ws_bytes(int64_t n_pix, int32_t N_d);
// a batch of at most 8 requests in one launch sequence (gen, trace, finalize)
hipError_t launch_shade_fwd_batch(const exm_request* r, int32_t n, const exm_params* p, void* ws, size_t ws_bytes,
                                  unsigned long long* counters, hipStream_t s);
size_t shade_fwd_batch_ws_bytes(const exm_request* r, int32_t n, int32_t N_d);
ShadeViews shade_views(const exm_camera* c, int32_t first, int32_t n);
size_t shade_fwd_ws_min(int32_t N_d);
// Scratch of exm_shade_fwd_noalloc: a device array of this many bytes per GPU; noalloc_scratch
// gives the current device's address (looked up once per device).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
hipError_t noalloc_scratch(void** ptr);
hipError_t launch_shade_bwd(const exm_mesh* m, const exm_material* mat, const exm_env* env, const ShadeViews& v,
                            const int32_t* tri_id, const float* bary, const exm_params* p, const float* dI,
                            const uint64_t* vis, const float* dquery, float* dtex, double* denv, void* ws,
                            size_t ws_bytes, hipStream_t s);
size_t shade_bwd_ws_bytes(int64_t n_pix, int32_t N_d, int32_t He, int32_t We);
size_t shade_bwd_ws_min(int32_t N_d, int32_t He, int32_t We);
hipError_t launch_trace_indirect(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat, const exm_env* env,
                                 const ShadeViews& v, const int32_t* tri_id, const float* bary, const exm_params* p,
                                 float* L_ind, exm_sec_rec* sec_rec, uint64_t* sec_vis, void* ws, size_t ws_bytes,
                                 unsigned long long* counters, hipStream_t s);
size_t trace_indirect_ws_bytes(int64_t n_pix, int32_t N_b, int32_t N_s);
size_t trace_indirect_ws_min(int32_t N_b, int32_t N_s);
hipError_t launch_trace_bwd(const exm_mesh* m, const exm_material* mat, const exm_env* env, const ShadeViews& v,
                            const int32_t* tri_id, const float* bary, const exm_params* p, float lambda_ind,
                            const float* dI, const exm_sec_rec* sec_rec, const uint64_t* sec_vis, float* dtex,
                            double* denv, void* ws, size_t ws_bytes, hipStream_t s);
size_t trace_bwd_ws_bytes(int64_t n_pix, int32_t N_b, int32_t N_s, int32_t He, int32_t We);
size_t trace_bwd_ws_min(int32_t N_b, int32_t N_s, int32_t He, int32_t We);

// host SAH builder (bvh_build.cpp): fills node/triangle arrays in host memory
struct HostBvh {
  BvhNode* nodes;    // the binary tree (host only)
  BvhNode4* nodes4;  // the 4-wide tree the traversal reads (root at 0)
  BvhTri* tris;
  int32_t n_nodes, n_nodes4, n_tris, root_is_leaf, depth, depth4;
};
bool build_bvh_host(const float* pos, int32_t nV, const int32_t* tri, int32_t nF, HostBvh* out, std::string* err);
void free_bvh_host(HostBvh* b);

}  // namespace exm
