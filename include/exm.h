/* exm: MI355X-native differentiable UV-PBR render pass (Stage II of ExMesh++).
 *
 * The pass renders a fixed mesh-UV carrier with optimisable UV-space PBR maps and an
 * equirectangular environment map (UV-PBR Asset Decomposition section):
 *   raster G-buffer -> bilinear UV queries (Eq. 10-11) -> GGX/Lambert shading under env
 *   importance sampling with shadow rays (Eq. 12-17) -> one-bounce diffuse indirect (Eq. 18-19)
 *   -> hand-written adjoint scatter into the maps and the env map.
 *
 * Conventions for every call:
 *  - Array pointers are DEVICE pointers owned by the caller, except those marked _host.
 *  - Calls only enqueue work on `stream` and return; results are valid after the stream
 *    synchronises. The library allocates no device memory except inside exm_build_bvh; passes
 *    that buffer rays take a caller-owned workspace.
 *  - Gradient outputs ACCUMULATE (+=); the caller zeroes them.
 *  - Shapes, null pointers, sizes and host-readable values are validated before any launch;
 *    a failed check returns EXM_E_INVAL and enqueues nothing. A HIP launch or runtime error
 *    returns EXM_E_HIP. exm_last_error() gives a thread-local message for the last non-OK
 *    status of the calling thread.
 *  - All views of one call share H and W. At most 64 direct samples per pixel (one u64 of
 *    visibility bits) and at most 64 secondary light samples (N_b * N_s <= 64).
 *  - Random numbers: Philox4x32-10 keyed by (seed_lo ^ seed_hi, iteration_lo) with counter
 *    (pixel = y*W + x, view_id, sample, stream); stream 0 = direct sample, 1 = secondary
 *    direction, 2+j = light sample of secondary ray j. Results are independent of how views
 *    are batched into calls.
 */
#ifndef EXM_H
#define EXM_H
#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EXM_OK = 0,
  EXM_E_INVAL = -1,       /* bad argument; nothing was enqueued */
  EXM_E_HIP = -2,         /* HIP runtime / launch error */
  EXM_E_NOMEM = -3,       /* allocation failed (exm_build_bvh only) */
  EXM_E_UNSUPPORTED = -4, /* no gfx950 device / feature */
} exm_status;

/* Thread-local text of the last non-OK status returned on this thread. */
const char* exm_last_error(void);

/* Test hook for failure handling (not a paper operation): the next n calls that would reach the
 * device fail with EXM_E_HIP and the message "injected failure (exm_inject_failures)" after
 * validating their arguments, enqueuing nothing; n <= 0 clears the count. Process-wide, taken
 * by whichever thread calls first. Lets a caller exercise its error paths (a failed request in
 * the relight service) without a faulty device. */
void exm_inject_failures(int32_t n);

/* Shading flags (exm_params.flags). METALLIC_OFF fixes m = 0 (dielectric model; UV-PBR Asset
 * Decomposition section, and the Implementation details of the Experiments). DIFFUSE_ONLY /
 * SPECULAR_ONLY drop f_s / f_d of Eq. 13 (tests). NO_VIS sets Vis = 1 (tests).
 * NO_SECONDARY_MATERIAL is the "No Secondary Material" ablation of the Ablation Study
 * (Indirect Lighting): the maps are not queried at secondary hits, which are shaded as a grey
 * Lambertian (albedo 0.5, metallic 0) with the interpolated geometric normal; the adjoint then
 * sends nothing to the maps at secondary hits. MAP_GRAD_ATOMIC makes the adjoints add the map
 * gradient with one atomic per tap and channel at any map size, instead of the tiled reduction
 * used for maps of at most 16,384 tiles of 64x32 texels (tests compare the two paths). */
enum {
  EXM_METALLIC_OFF = 1u << 0,
  EXM_DIFFUSE_ONLY = 1u << 1,
  EXM_SPECULAR_ONLY = 1u << 2,
  EXM_NO_VIS = 1u << 3,
  EXM_NO_SECONDARY_MATERIAL = 1u << 4,
  EXM_MAP_GRAD_ATOMIC = 1u << 5,
};

/* Fixed mesh-UV carrier M = (V, F), UV set U and face-corner UV index Phi (UV-PBR Asset
 * Decomposition section). Counter-clockwise triangles are front facing. */
typedef struct {
  int32_t nV, nF, nUV;
  const float* pos;      /* [nV,3] */
  const int32_t* tri;    /* [nF,3] vertex indices */
  const float* uv;       /* [nUV,2] (u, v), row 0 of a map is v in [0, 1/Ht) */
  const int32_t* tri_uv; /* [nF,3] UV indices (Phi) */
  double* vnrm;          /* [nV,3] unit vertex normals (FP64), written by exm_mesh_prepare */
  float* ftan;           /* [nF,4] face tangent xyz + handedness, written by exm_mesh_prepare */
} exm_mesh;

/* One view. Host memory; clip = mvp * [p, 1] (row-major, OpenGL clip space, y up);
 * view_id is the RNG counter word of the view (a request id when serving). */
typedef struct {
  double mvp[16];
  double eye[3];
  int32_t H, W;
  int32_t view_id;
} exm_camera;

/* Packed UV-space material maps {A, R, M_met, N}: [Ht,Wt,8] float =
 * (a.r, a.g, a.b, roughness, metallic, n.x, n.y, n.z); n is the tangent-space normal. */
typedef struct {
  int32_t Ht, Wt;
  const float* tex;
} exm_material;

/* Learnable lat-long environment map E ([He,We,3], E >= 0; row 0 at theta = 0, +Y up,
 * phi from +X toward +Z) and its importance-sampling tables from exm_build_env_sampler. */
typedef struct {
  int32_t He, We;
  const float* env;
  const uint64_t* cdf_row; /* [He] */
  const uint64_t* cdf_col; /* [He,We] */
  const float* pdf;        /* [He,We] solid-angle density of the texel */
  const uint32_t* guide;   /* [exm_env_guide_len(He,We)] cutpoint tables over the CDFs */
  const float* rec;        /* [He,We,4] per texel (E.r, E.g, E.b, 1/pdf); 16-byte aligned */
} exm_env;

/* Estimator parameters. N_d direct env samples (Eq. 17), N_b secondary rays (Eq. 19), N_s
 * light samples per secondary hit (Eq. 18); hyperparameter table defaults are 8 / 16 / 4.
 * f_diel = F_dielectric of Eq. 16 (0.04), eps = epsilon of Eq. 15 (1e-6), tmin = ray start
 * distance (world units) for shadow and secondary rays. */
typedef struct {
  int32_t N_d, N_b, N_s;
  uint64_t seed, iteration;
  float f_diel, eps, tmin;
  uint32_t flags;
} exm_params;

/* One secondary-ray record per (pixel, j): triangle id (-1: miss or back face) and
 * barycentrics (b1, b2) of the hit. */
typedef struct {
  int32_t tri;
  float b1, b2;
} exm_sec_rec;

typedef struct exm_bvh exm_bvh; /* opaque; device resident; owned by the library */

/* Area-weighted vertex normals and per-face UV tangent frames of the carrier (tangent frame
 * "interpolated on the current face", Attribute Query). Writes m->vnrm and m->ftan. */
exm_status exm_mesh_prepare(const exm_mesh* m, hipStream_t stream);

/* Binned-SAH BVH over the fixed triangles, built on the host as a binary tree, collapsed to
 * 4-wide nodes (128 bytes each) and uploaded on `stream` (ray queries for visibility and
 * secondary hits: Direct Illumination, One-Bounce Indirect Illumination). Host inputs; *out
 * receives a handle. At most 2^25 triangles: the builder bounds the binary depth at 24 (the wide
 * depth at 12) so that the traversal's stack cannot overflow, which holds up to that size;
 * larger meshes return EXM_E_UNSUPPORTED before anything is read. Returns EXM_E_NOMEM if device
 * memory runs out. exm_free_bvh waits for the stream work that uses the BVH to be done by the
 * caller. */
exm_status exm_build_bvh(const float* pos_host, int32_t nV, const int32_t* tri_host, int32_t nF,
                         exm_bvh** out, hipStream_t stream);
exm_status exm_free_bvh(exm_bvh* bvh);
/* Device bytes held by the BVH (for admission by HBM footprint). 0 for NULL. */
size_t exm_bvh_device_bytes(const exm_bvh* bvh);

/* Importance-sampling distribution over env texels proportional to luminance times texel
 * solid angle (Direct Illumination). Integer tables: q_ij = max(1, floor(w_ij / max w *
 * 2^20)); cdf_row = inclusive prefix of row totals; cdf_col = inclusive prefix inside a row;
 * pdf_ij = q_ij / (Q Omega_i). A texel is picked by inverting these CDFs (row, then column).
 * Also written, as functions of the tables and the map: `guide`, cutpoint tables that narrow
 * each inversion to a few entries without changing its result (Chen and Asau's guide-table
 * method), followed for We < 4096 by compact copies that the pick reads (cdf_col in uint32,
 * a row total being below 2^32 there; the column cutpoints in uint16; (cdf_col - 1) mod 2^16
 * in uint16, which decides a search step in rows whose cutpoint buckets hold at most 2^16
 * keys), and `rec`, the packed per-texel record (E, 1/pdf) read by the pick. All outputs
 * are caller-owned device buffers; cdf_row, cdf_col 8-byte, rec 16-byte aligned. The tables
 * describe the map at the time of the call: rebuild them after the map changes. Needs
 * He >= 1, 2 <= We, He*We <= 2^24; uses no workspace. */
size_t exm_env_guide_len(int32_t He, int32_t We); /* uint32 entries of `guide` */
exm_status exm_build_env_sampler(const float* env, int32_t He, int32_t We, uint64_t* cdf_row,
                                 uint64_t* cdf_col, float* pdf, uint32_t* guide, float* rec,
                                 hipStream_t stream);

/* G-buffer (Attribute Query: face f and barycentrics b of the visible point): per pixel the
 * closest triangle under a top-left fill rule at the pixel centre, id -1 for background, and
 * perspective-correct barycentrics (b1, b2). tri_id [nViews,H,W] int32, bary [nViews,H,W,2]
 * float (8-byte aligned; also used as the depth buffer during the call). */
exm_status exm_raster_gbuffer(const exm_mesh* m, const exm_camera* cams_host, int32_t nViews,
                              int32_t* tri_id, float* bary, hipStream_t stream);

/* Direct light, Eq. 17: L_dir [nViews,H,W,3] float (overwritten) and vis [nViews,H,W] u64,
 * bit k = sample k had n_s . w > 0 and was unoccluded. Needs exm_mesh_prepare.
 * ws: caller-owned device workspace (256-byte aligned) holding the shadow rays of a chunk of
 * pixels; exm_shade_fwd_workspace_size gives the bytes that hold one launch's pixels at once
 * (at most 8 views per launch), any size >= exm_shade_fwd_workspace_min works by processing
 * pixels in chunks. The workspace is scratch: its contents are undefined after the call, and
 * calls sharing one workspace must be ordered on one stream. */
size_t exm_shade_fwd_workspace_size(int32_t nViews, int32_t H, int32_t W, int32_t N_d);
size_t exm_shade_fwd_workspace_min(int32_t N_d);
exm_status exm_shade_fwd(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat,
                         const exm_env* env, const exm_camera* cams_host, int32_t nViews,
                         const int32_t* tri_id, const float* bary, const exm_params* p,
                         float* L_dir, uint64_t* vis, void* ws, size_t ws_bytes, hipStream_t stream);

/* Batched direct pass for serving (relighting of exported assets, Computational Efficiency): one
 * launch sequence (env sampling and shading, shadow-ray traversal, finalisation) over the pixels
 * of several requests, each with its own asset (mesh, BVH, maps), env map and view. Per request:
 * the same outputs, bit for bit, as exm_shade_fwd of that request alone with p and tmin: the
 * random numbers are keyed by cam.view_id (the request id), so a result does not depend on the
 * batch it runs in. At most 8 requests share one launch sequence; more are run 8 at a time. */
typedef struct {
  const exm_mesh* mesh;     /* prepared by exm_mesh_prepare */
  const exm_bvh* bvh;
  const exm_material* mat;
  const exm_env* env;       /* with its tables from exm_build_env_sampler */
  exm_camera cam;           /* the request's view (host); view_id keys its random numbers */
  float tmin;               /* ray start distance of the asset (world units); replaces p->tmin */
  const int32_t* tri_id;    /* [H,W] G-buffer of the view (exm_raster_gbuffer) */
  const float* bary;        /* [H,W,2] */
  float* L_dir;             /* [H,W,3] out */
  uint64_t* vis;            /* [H,W] out */
} exm_request;

/* ws: device workspace (256-byte aligned) of at least exm_shade_fwd_batch_workspace_size bytes for
 * these requests (the ray records of up to 8 requests at once; no chunking). reqs is host memory;
 * p applies to every request except its tmin. */
size_t exm_shade_fwd_batch_workspace_size(const exm_request* reqs_host, int32_t n_req, int32_t N_d);
exm_status exm_shade_fwd_batch(const exm_request* reqs_host, int32_t n_req, const exm_params* p, void* ws,
                               size_t ws_bytes, hipStream_t stream);

/* exm_shade_fwd without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * outputs, bit for bit, computed in a device scratch array of 64 MiB that the library holds on
 * each GPU it runs on until the process ends (looked up on the first call on a device). It
 * allocates nothing: any image size works, the pixels run in chunks of what fits in the
 * scratch (at N_d = 64 about 35,000 pixels per chunk, at N_d = 8 about 260,000). Every call on
 * one GPU shares that GPU's scratch: calls that overlap on one GPU (on different streams or
 * from several threads) race; order them on one stream. */
exm_status exm_shade_fwd_noalloc(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat,
                                 const exm_env* env, const exm_camera* cams_host, int32_t nViews,
                                 const int32_t* tri_id, const float* bary, const exm_params* p,
                                 float* L_dir, uint64_t* vis, hipStream_t stream);

/* One-bounce diffuse indirect, Eq. 18-19: L_ind [nViews,H,W,3] (overwritten), sec_rec
 * [nViews,H,W,N_b], sec_vis [nViews,H,W] u64 (bit j*N_s+s). ws: ray workspace as for
 * exm_shade_fwd, sized by exm_trace_indirect_workspace_size / _min. */
size_t exm_trace_indirect_workspace_size(int32_t nViews, int32_t H, int32_t W, int32_t N_b,
                                         int32_t N_s);
size_t exm_trace_indirect_workspace_min(int32_t N_b, int32_t N_s);
exm_status exm_trace_indirect(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat,
                              const exm_env* env, const exm_camera* cams_host, int32_t nViews,
                              const int32_t* tri_id, const float* bary, const exm_params* p,
                              float* L_ind, exm_sec_rec* sec_rec, uint64_t* sec_vis, void* ws,
                              size_t ws_bytes, hipStream_t stream);

/* Measurement variants: the same work and outputs as exm_shade_fwd / exm_trace_indirect, plus
 * work counts accumulated (+=) into the caller's device array `counters` (u64):
 *   exm_shade_fwd_counted      [4]: shadow rays traced, BVH nodes visited, triangles tested,
 *                                   env samples drawn
 *   exm_trace_indirect_counted [6]: secondary rays, their node visits and triangle tests,
 *                                   secondary light shadow rays, their node visits and tests
 * The counts are the traversal work of the ray queries (Direct Illumination visibility,
 * One-Bounce Indirect Illumination secondary hits) on this BVH. */
exm_status exm_shade_fwd_counted(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat,
                                 const exm_env* env, const exm_camera* cams_host, int32_t nViews,
                                 const int32_t* tri_id, const float* bary, const exm_params* p,
                                 float* L_dir, uint64_t* vis, void* ws, size_t ws_bytes,
                                 uint64_t* counters, hipStream_t stream);
exm_status exm_trace_indirect_counted(const exm_mesh* m, const exm_bvh* bvh, const exm_material* mat,
                                      const exm_env* env, const exm_camera* cams_host, int32_t nViews,
                                      const int32_t* tri_id, const float* bary, const exm_params* p,
                                      float* L_ind, exm_sec_rec* sec_rec, uint64_t* sec_vis, void* ws,
                                      size_t ws_bytes, uint64_t* counters, hipStream_t stream);

/* Adjoint of the direct pass for upstream dI [nViews,H,W,3]: dtex [Ht,Wt,8] += d/dtex,
 * denv [He,We,3] += d/dE (double). Discrete choices (ids, texel picks, vis bits) and the
 * sampling pdf are held fixed. dquery [nViews,H,W,8] (or NULL) is a gradient with respect to
 * the eight queried map values of Eq. 10 at each visible pixel (such as the adjoint of a loss on
 * the screen projection of the maps); it is added to the pixel's map adjoint before the one
 * scatter into dtex, which gives what exm_project_maps_bwd would add. Part of the additions into
 * dtex are plain read-modify-writes (a texel tile summed by one block): calls that add into the
 * same dtex must not run concurrently (issue them on one stream, or order them with events).
 * dtex must be 16-byte aligned (EXM_E_INVAL otherwise). */
exm_status exm_shade_bwd(const exm_mesh* m, const exm_material* mat, const exm_env* env,
                         const exm_camera* cams_host, int32_t nViews, const int32_t* tri_id,
                         const float* bary, const exm_params* p, const float* dI,
                         const uint64_t* vis, const float* dquery, float* dtex, double* denv, void* ws,
                         size_t ws_bytes, hipStream_t stream);

/* Adjoint of the indirect pass for upstream lambda_ind * dI (Eq. 20): into the materials at
 * the primary and the secondary points and into E at the secondary light samples. The map
 * gradient is added as exm_shade_bwd adds its own (tiles summed by one block each, with plain
 * read-modify-writes): calls that add into the same dtex must not run concurrently. */
exm_status exm_trace_bwd(const exm_mesh* m, const exm_material* mat, const exm_env* env,
                         const exm_camera* cams_host, int32_t nViews, const int32_t* tri_id,
                         const float* bary, const exm_params* p, float lambda_ind,
                         const float* dI, const exm_sec_rec* sec_rec, const uint64_t* sec_vis,
                         float* dtex, double* denv, void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace of the adjoints (device memory, 256-byte aligned, caller-owned): two 16-byte
 * records per env sample of the pixels in flight (N_d per pixel for exm_shade_bwd, N_b * N_s
 * for exm_trace_bwd) plus the bucket tables of the env map's binned reduction; two 64-byte
 * map-gradient records per surface point in flight (the pixel's for exm_shade_bwd, the pixel's
 * and its N_b secondary points' for exm_trace_bwd) and the tables of their tile sort (about
 * 0.3 MB). _size is what
 * the views of one launch (at most 8) take at once; any size from _min up works, the pixels
 * then run in chunks. 0 for invalid arguments. */
size_t exm_shade_bwd_workspace_size(int32_t nViews, int32_t H, int32_t W, int32_t N_d, int32_t He,
                                    int32_t We);
size_t exm_shade_bwd_workspace_min(int32_t N_d, int32_t He, int32_t We);
size_t exm_trace_bwd_workspace_size(int32_t nViews, int32_t H, int32_t W, int32_t N_b, int32_t N_s,
                                    int32_t He, int32_t We);
size_t exm_trace_bwd_workspace_min(int32_t N_b, int32_t N_s, int32_t He, int32_t We);

/* Half-resolution indirect light (Implementation Details: secondary rays are evaluated at half
 * resolution in both image dimensions and the indirect component is upsampled to full
 * resolution). The caller renders the indirect pass on a half-resolution G-buffer of the same
 * cameras (tri_id_half [nViews,Hh,Wh]) and exm_upsample_indirect writes the full-resolution
 * L_ind [nViews,H,W,3] from L_half [nViews,Hh,Wh,3]: per axis the pixel x sits at
 * u = ((x + 1/2) Hh / H) - 1/2 half-resolution pixels, bilinear over the two clamped taps;
 * only covered half-resolution taps count and the weights are renormalised over them; 0 for
 * background pixels and pixels without a covered tap. exm_upsample_indirect_bwd writes (does
 * not accumulate) dL_half = U^T (lambda_ind * dI), the transpose of that map, ready to be the
 * upstream gradient of exm_trace_bwd on the half-resolution buffers with lambda_ind = 1.
 * Needs 1 <= Hh <= H, 1 <= Wh <= W. */
exm_status exm_upsample_indirect(const int32_t* tri_id_half, int32_t Hh, int32_t Wh, const float* L_half,
                                 const int32_t* tri_id, int32_t H, int32_t W, int32_t nViews, float* L_ind,
                                 hipStream_t stream);
exm_status exm_upsample_indirect_bwd(const int32_t* tri_id_half, int32_t Hh, int32_t Wh, const int32_t* tri_id,
                                     int32_t H, int32_t W, int32_t nViews, float lambda_ind, const float* dI,
                                     float* dL_half, hipStream_t stream);

/* ---- Stage-II objective and optimiser step (Stage-II Optimization, Eq. 21-24) ----
 * Readings of what the paper leaves open: L_img = 0.8 * mean |log(1 + I_hat) - log(1 + I)| +
 * 0.2 * (1 - mean SSIM) (D-SSIM weight 0.2 from the hyperparameter table, the log-L1 weight its
 * complement; means over pixels and channels of a view); SSIM per channel (Wang et al. 2004) of
 * the sRGB curve of the radiance clamped to [0, 1], 11-tap Gaussian window of sigma 1.5, zero
 * padding, C1 = 1e-4, C2 = 9e-4. TV(P_hat) (Eq. 23): for the groups A, R, N (and M when metallic
 * is optimised) the sum over right/down pairs of visible pixels of the group's channel-mean
 * |difference| of the screen projection, divided by H * W. TV(E): the same over env texels
 * with phi wrapping, divided by He * We. Chroma (Eq. 24): squared distance of the per-channel
 * texel mean of E from its grey mean. Losses ACCUMULATE into a device double; gradients as
 * stated per call. */

/* Screen projection of the packed map: P [nViews,H,W,8] = the bilinear query (Eq. 10) at every
 * visible pixel, 0 elsewhere; _bwd: dtex += its adjoint for dP [nViews,H,W,8]. */
exm_status exm_project_maps(const exm_mesh* m, const exm_material* mat, int32_t nViews, int32_t H, int32_t W,
                            const int32_t* tri_id, const float* bary, float* P, hipStream_t stream);
exm_status exm_project_maps_bwd(const exm_mesh* m, const exm_material* mat, int32_t nViews, int32_t H, int32_t W,
                                const int32_t* tri_id, const float* bary, const float* dP, float* dtex,
                                hipStream_t stream);
/* scale * L_img of each view (I_hat, I [nViews,H,W,3]) into *loss; dI_hat = scale * dL_img/dI_hat
 * (written). Workspace: exm_image_loss_workspace_size(H, W) bytes, 256-byte aligned. H <= 65535. */
size_t exm_image_loss_workspace_size(int32_t H, int32_t W);
exm_status exm_image_loss(const float* I_hat, const float* I, int32_t nViews, int32_t H, int32_t W, float scale,
                          double* loss, float* dI_hat, void* ws, size_t ws_bytes, hipStream_t stream);
/* scale * L_mat of the projections P [nViews,H,W,8] (visibility from tri_id) into *loss;
 * dP = its gradient (written). metallic != 0 adds the M group. */
exm_status exm_tv_screen(const float* P, const int32_t* tri_id, int32_t nViews, int32_t H, int32_t W,
                         int32_t metallic, float scale, double* loss, float* dP, hipStream_t stream);
/* w_tv * TV(E) + w_chroma * L_chroma into *loss; dE [He,We,3] += gradient (double). acc3 is a
 * device scratch of 3 doubles. */
exm_status exm_env_regularizers(const float* E, int32_t He, int32_t We, float w_tv, float w_chroma, double* loss,
                                double* dE, double* acc3, hipStream_t stream);
/* One Adam step (Kingma and Ba 2015) on n values laid out with n_chan channels (<= 8): m, v
 * updated, param -= lr * m_hat / (sqrt(v_hat) + eps) for step t >= 1, then clamped to
 * [lo[c], hi[c]] (lo, hi host arrays of n_chan): the projection that keeps E non-negative and
 * the material channels in range. grad is float, or double when grad_is_f64. The moments and
 * the parameter are updated in float; the coefficients (beta, 1 - beta, the bias corrections)
 * are formed in double on the host and rounded once. */
exm_status exm_adam_step(float* param, const void* grad, int32_t grad_is_f64, float* m, float* v, int64_t n,
                         int32_t n_chan, const float* lo_host, const float* hi_host, double lr, double beta1,
                         double beta2, double eps, int32_t t, hipStream_t stream);

/* ---- Stage-I topology operations (Vertex Splitting, Vertex Merging, UV Maintenance; Eq. 1-6) --
 * A mesh being refined lives in caller-owned device arrays of fixed capacity; a round rewrites
 * them in place and updates the counts. */
typedef struct {
  int32_t nV, nF, nUV;          /* current counts (updated by exm_topology_round) */
  int32_t capV, capF, capUV;    /* capacities of the arrays below */
  float* pos;                   /* [capV,3] vertex positions */
  float* G;                     /* [capV] per-vertex EMA of the position-gradient norm (Eq. 1) */
  float* uv;                    /* [capUV,2] UV coordinates */
  int32_t* tri;                 /* [capF,3] faces (vertex indices) */
  int32_t* tri_uv;              /* [capF,3] face-corner UV indices (Phi) */
} exm_topo_mesh;

#define EXM_TOPO_NO_SPLIT (1u << 0) /* merging only */
#define EXM_TOPO_NO_MERGE (1u << 1) /* splitting only */

typedef struct {
  double beta_g;                /* EMA coefficient of Eq. 1 (0.95) */
  double w_g, w_k;              /* split-score weights of Eq. 3 (0.6, 0.4) */
  double tau_degen;             /* degeneracy threshold of Eq. 4 (0.05) */
  double tau_uv;                /* UV seam threshold of Eq. 6 (UV units) */
  double split_fraction;        /* share of the faces selected per splitting round */
  int32_t max_faces;            /* face budget (200K) */
  uint32_t flags;               /* EXM_TOPO_NO_SPLIT, EXM_TOPO_NO_MERGE */
} exm_topo_params;

typedef struct {
  int32_t split_selected, split_invalid, split_conflict, splits;
  int32_t merge_candidates, merge_conflict, merges, faces_deleted;
  int32_t mis_iterations;       /* parallel passes of the conflict resolution */
} exm_topo_stats;

/* Eq. 1: G[v] = beta G[v] + (1 - beta) |grad[v]| for nV vertices; grad [nV,3] float. Evaluated in
 * FP64 and rounded to float. */
exm_status exm_vertex_grad_ema(float* G, const float* grad, int32_t nV, double beta, hipStream_t stream);
/* C_rend of the merging criterion: counts[f] += number of pixels of a G-buffer (n_px ids, -1 for
 * background) whose visible face is f (f < nF). Accumulates over calls (views). */
exm_status exm_face_render_counts(const int32_t* tri_id, int64_t n_px, int32_t nF, int32_t* counts,
                                  hipStream_t stream);
/* Workspace of a round (and of exm_topology_scores) on a mesh of these counts. */
size_t exm_topology_workspace_size(int32_t nV, int32_t nF, int32_t nUV, const exm_topo_params* p);
/* Per-face terms of the criteria (FP64, [nF] each): S_f of Eq. 3 (with K_f of Eq. 2 and the face
 * mean of G), K_f, D_f of Eq. 4 and the face area. */
exm_status exm_topology_scores(const exm_topo_mesh* m, const exm_topo_params* p, double* S, double* K, double* D,
                               double* area, void* ws, size_t ws_bytes, hipStream_t stream);
/* One round of vertex splitting then vertex merging with the UV updates of Eq. 5-6 and the index
 * compaction after merging, on the criteria of the mesh at the start of the round. c_rend [nF]
 * is the render count of every face (NULL: every face counts as rendered). The arrays of *m are
 * rewritten in place and its counts updated; the capacities must hold nV + K vertices,
 * nF + 2K faces and nUV + 2K UVs, K = min(floor(split_fraction nF), floor((max_faces - nF)/2)).
 * Synchronous: it waits on `stream` (the conflict resolution reads a counter back per pass) and
 * fills *stats (host). Deterministic: the result does not depend on thread scheduling. */
exm_status exm_topology_round(exm_topo_mesh* m, const int32_t* c_rend, const exm_topo_params* p, void* ws,
                              size_t ws_bytes, exm_topo_stats* stats, hipStream_t stream);

/* Measurement hooks. With timing enabled, every kernel the library launches is bracketed by
 * two HIP events recorded on its launch stream (no events exist while it is off).
 * exm_timing_enable clears the records; exm_timing_collect waits for the recorded events and
 * adds their elapsed times to per-kernel totals, read back by index (0 <= i < count); names
 * stay valid until the next enable. */
exm_status exm_timing_enable(int32_t on);
exm_status exm_timing_collect(void);
int32_t exm_timing_count(void);
const char* exm_timing_name(int32_t i);
double exm_timing_total_ms(int32_t i);
int64_t exm_timing_launches(int32_t i);

#ifdef __cplusplus
}
#endif
#endif
