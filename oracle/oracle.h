/* FP64 CPU oracle of the Stage-II UV-PBR render pass.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load this library. The product path (the HIP library) never calls it, links
 * it or shares code with it; the two share only the input arrays.
 *
 * Every quantity is computed in double precision, in the order the paper states it:
 *   attribute query                      UV-PBR Asset Decomposition, Attribute Query (Eq. 10-11)
 *   BRDF f_r = f_d + f_s                 Direct Illumination (Eq. 13-16)
 *   env importance sampling, estimator   Direct Illumination (Eq. 17)
 *   one-bounce diffuse indirect          One-Bounce Indirect Illumination (Eq. 18-19)
 * Readings of what the paper leaves open (projection, fill rule, D/G/F variants, sampler
 * quantisation, RNG stream, t_min) are listed with each function below.
 */
#ifndef EXM_ORACLE_H
#define EXM_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORA_METALLIC_OFF = 1u << 0,
  ORA_DIFFUSE_ONLY = 1u << 1,
  ORA_SPECULAR_ONLY = 1u << 2,
  ORA_NO_VIS = 1u << 3,
  /* "No Secondary Material" ablation (Ablation Study, Indirect Lighting): no material query at
     secondary hits; read here as a grey Lambertian (albedo ORA_SECONDARY_ALBEDO, metallic 0)
     with the interpolated geometric normal */
  ORA_NO_SECONDARY_MATERIAL = 1u << 4,
};
#define ORA_SECONDARY_ALBEDO 0.5

typedef struct {
  int32_t nV, nF, nUV;
  const float* pos;      /* [nV,3] */
  const int32_t* tri;    /* [nF,3], counter-clockwise = front */
  const float* uv;       /* [nUV,2] */
  const int32_t* tri_uv; /* [nF,3] */
} ora_mesh;

typedef struct {
  double mvp[16]; /* row-major, OpenGL clip space */
  double eye[3];
  int32_t H, W;
  int32_t view_id; /* RNG counter word 1 */
} ora_camera;

typedef struct {
  int32_t He, We;
  uint64_t Q;
  const uint64_t* cdf_row; /* [He]   inclusive prefix of row totals */
  const uint64_t* cdf_col; /* [He,We] inclusive prefix within each row */
  const uint64_t* q;       /* [He,We] quantised weights */
} ora_tables;

typedef struct {
  int32_t N_d, N_b, N_s;
  uint64_t seed, iteration;
  double f_diel, eps, tmin;
  uint32_t flags;
} ora_params;

typedef struct {
  int32_t Ht, Wt;
  const double* tex;     /* [Ht,Wt,8] */
  const double* tex_dot; /* JVP direction for tex, or NULL */
  int32_t He, We;
  const double* env;     /* [He,We,3] */
  const double* env_dot; /* JVP direction for env, or NULL */
} ora_params_theta;

typedef struct {
  /* per listed pixel */
  int32_t* tri_id;   /* [n] */
  double* bary;      /* [n,3] perspective-correct b0,b1,b2 */
  double* L_dir;     /* [n,3] */
  double* L_ind;     /* [n,3] */
  double* dL_dir;    /* [n,3] JVP tangent (NULL unless a direction was given) */
  double* dL_ind;    /* [n,3] */
  uint64_t* vis;     /* [n] bit k = visibility of direct sample k */
  int32_t* sec_tri;  /* [n,N_b] -1 = no valid secondary hit */
  double* sec_bary;  /* [n,N_b,2] */
  uint64_t* sec_vis; /* [n] bit j*N_s+s */
  int32_t* n_shadow; /* [n] shadow rays traced (direct) */
} ora_out;

/* ---- mesh attributes (Attribute Query) ---- */
void ora_vertex_normals(const ora_mesh* m, double* vnrm /* [nV,3] */);
void ora_face_tangents(const ora_mesh* m, double* ftan /* [nF,4] */);

/* ---- raster: per-pixel closest triangle + perspective-correct barycentrics ---- */
void ora_raster(const ora_mesh* m, const ora_camera* cam, int32_t* tri_id /* [H*W] */,
                double* bary /* [H*W,3] */);
/* per-pixel number of triangles whose coverage test passes (depth ignored) */
void ora_coverage_count(const ora_mesh* m, const ora_camera* cam, int32_t* count /* [H*W] */);

/* ---- env importance sampling tables ---- */
void ora_env_tables(int32_t He, int32_t We, const float* env, uint64_t* q, uint64_t* cdf_row,
                    uint64_t* cdf_col, double* pdf, uint64_t* Q, double* w /* [He,We] or NULL */);
/* sample the table with a 64-bit target word and two uniforms */
void ora_env_sample(const ora_tables* t, uint64_t x, double u2, double u3, int32_t* row,
                    int32_t* col, double* dir /* [3] */, double* pdf);

/* ---- counter-based RNG ---- */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* ---- BRDF (Eq. 13-16) and its pieces, for closed-form checks ---- */
void ora_brdf(const double a[3], double r, double m, const double n[3], const double wi[3],
              const double wo[3], double f_diel, double eps, uint32_t flags, double out[3]);
double ora_ggx_D(double r, const double n[3], const double h[3]);
double ora_smith_G1(double r, double c);

/* ---- attribute query at a surface point (Eq. 10-11) ---- */
void ora_bilinear(int32_t Ht, int32_t Wt, const double* tex, int32_t C, double u, double v,
                  double* out /* [C] */);
void ora_shading_normal(const ora_mesh* m, const double* vnrm, const double* ftan, int32_t f,
                        const double b[3], const double q[3], double ng[3], double ns[3]);

/* ---- rays: BVH (median split) and brute force ---- */
typedef struct ora_bvh ora_bvh;
ora_bvh* ora_bvh_build(const ora_mesh* m);
void ora_bvh_free(ora_bvh* b);
/* closest hit: t >= tmin, skipping triangle `skip`; hit id -1 = miss. bvh may be NULL (brute) */
void ora_trace_closest(const ora_mesh* m, const ora_bvh* b, int32_t n, const double* o,
                       const double* d, double tmin, const int32_t* skip, int32_t* hit,
                       double* t, double* bary2);
void ora_trace_any(const ora_mesh* m, const ora_bvh* b, int32_t n, const double* o,
                   const double* d, double tmin, const int32_t* skip, uint8_t* hit);
/* decision margins of one ray (brute force): see oracle.cpp */
void ora_ray_margins(const ora_mesh* m, const double o[3], const double d[3], double tmin,
                     int32_t skip, double tol, int32_t* n_hits, double* max_hit_margin,
                     double* min_margin);

/* The oracle's own ray of one estimator sample, for flip accounting: for pixel pix[i] and
 * index idx[i] of stream `stream` (0 = direct sample k, 1 = secondary direction j,
 * 2+j = light sample idx of secondary ray j): origin, direction, the clamped cosine's
 * argument (n_s.w for 0 and 2+j, n_g.w for 1) and the triangle the ray skips.
 * valid[i] = 0 when the ray does not exist (background pixel, or no valid secondary hit). */
void ora_sample_rays(const ora_mesh* m, const ora_bvh* b, const ora_camera* cam, const ora_params_theta* th,
                     const ora_tables* tab, const ora_params* p, int32_t n, const int64_t* pix,
                     const int32_t* idx, int32_t stream, double* o, double* d, double* c, int32_t* skip,
                     uint8_t* valid);

/* ---- the render pass, for a list of pixels of one view ---- */
int32_t ora_render(const ora_mesh* m, const ora_bvh* b, const ora_camera* cam,
                   const ora_params_theta* th, const ora_tables* tab, const ora_params* p,
                   int32_t n_pix, const int64_t* pix /* NULL = all H*W pixels in order */,
                   ora_out* out, int32_t n_threads);

#ifdef __cplusplus
}
#endif
#endif
