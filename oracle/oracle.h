/* FP64 CPU oracle for the hybrid surface-volumetric marcher.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow and written to be checked against
 * the paper by eye: brute-force intersection over every triangle, one sample
 * at a time, no acceleration structure, no blocking or fusion.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may call it; the
 * product path never does.  It shares no code with the HIP library.
 *
 * Every function cites the passage of "Dynamic Mesh-Aware Radiance Fields"
 * (Qiao, Gao et al., ICCV 2023) it follows.  Where the paper is silent the
 * reading used is stated at the function.
 */
#ifndef MESHRF_ORACLE_H
#define MESHRF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_levels, feats, log2_table;
  const int32_t* res;        /* [n_levels] grid resolution per level        */
  const float* table;        /* [n_levels][2^log2_table][feats]              */
  int32_t d_in, d_hidden, d_out;          /* density MLP widths               */
  int32_t c_in, c_hidden, c_layers, sh;   /* colour MLP widths, SH components */
  const float* mlp;          /* flat weights, forward order, [out][in]       */
  double density_offset;
  double aabb_min[3], aabb_max[3];
  /* placement of the field in the world (a moving NeRF object): a world point
   * p is looked up at R^T (p - c), a direction d at R^T d.  pose = [R | c]
   * row-major 3x4, R a rotation.  has_pose = 0: the field's frame is the world. */
  int32_t has_pose;
  double pose[12];
} orc_field;

typedef struct {
  int32_t nv, nf;
  const float* vertices;     /* [nv][3] */
  const int32_t* indices;    /* [nf][3] */
  const int32_t* mat_ids;    /* [nf]    */
  int32_t n_mat;
  const float* materials;    /* [n_mat][8]: kind, ior, albedo rgb, emitted radiance rgb */
} orc_mesh;

typedef struct {
  double t_near, t_far;
  int32_t n_samples;
  int32_t max_bounces;
  int32_t rr_after;          /* -1 = no Russian roulette */
  double t_min_throughput;
  uint32_t seed;
  double tie_eps;            /* world-space edge margin / relative t gap of a geometric tie */
  double tie_rel;            /* relative band of a scalar decision (Fresnel, roulette, cut-off) */
  /* optional occupancy grid (the oracle's own, see orc_build_occupancy) */
  int32_t occ_res;
  const uint8_t* occ;        /* [res^3] 0/1, x fastest */
  /* optional proposal sampler */
  const orc_field* proposal; /* density-only field (d_out = 1, c_layers = 0) */
  int32_t n_prop;            /* proposal intervals */
  int32_t n_fine;            /* fine samples drawn from the proposal */
  /* optional shadow mask per field sample (Sec. 3.1 "Shadow rays"): a ray from
   * the sample to each light; each light a mesh blocks multiplies the
   * sample's emitted radiance by shadow_mask */
  int32_t sample_shadows;
  double shadow_mask;
  /* optional light sampling toward emitting triangles (Eq. 12's L_e read as
   * area lights): at every diffuse hit one point on one emitting triangle,
   * chosen with probability proportional to its summed emitted radiance and
   * uniformly by area on it; a path that reaches an emitter straight after a
   * diffuse scatter then adds no L_e there (the light sample stands for it) */
  int32_t sample_emitters;
  /* optional several fields in one scene (uniform sampler only): when
   * n_fields > 0 the field argument of orc_render is ignored and these are
   * marched together; field_occ[k] (or NULL) is field k's occupancy grid of
   * resolution field_occ_res[k] */
  int32_t n_fields;
  const orc_field* const* fields;
  const uint8_t* const* field_occ;
  const int32_t* field_occ_res;
  /* with several fields, the proposal sampler: field k's own proposal (the
   * boxes must not overlap; each field is marched on its own range in the
   * order the ray enters the boxes) */
  const orc_field* const* field_proposals;
  /* optional, to check the outcomes of tie rays: force_hits [n][max_bounces+1]
   * names per segment the triangle (-1 none) to take instead of the closest
   * hit, taken when single precision can reach it (a hit or near miss no
   * farther than the first certain hit, or no hit when none is certain), else
   * the ray is marked invalid; flip [n]: bit k takes the other branch of the
   * ray's k-th flagged scalar decision (occupancy, shadow visibility, Fresnel,
   * roulette, cut-off, emitter choice, in path order) */
  const int32_t* force_hits;
  const uint32_t* flip;
  /* with sample_emitters: grid intervals per segment length for the optical
   * depth along a light sample's shadow segment (0 = n_samples) */
  int32_t light_depth_samples;
} orc_opts;

typedef struct {
  double* radiance;          /* [n][3] */
  double* throughput;        /* [n][3] */
  int32_t* bounces;          /* [n]    */
  int32_t* hit_ids;          /* [n][max_bounces+1], -1 = miss / not reached */
  uint8_t* tie;              /* [n] */
  int64_t* samples;          /* [n] field evaluations per ray (optional) */
  int32_t* segments;         /* [n] marched segments per ray (optional) */
  uint8_t* invalid;          /* [n] a forced hit was not reachable (optional) */
  int32_t* n_flagged;        /* [n] flagged scalar decisions met on the path (optional) */
} orc_out;

/* ---- building blocks, exposed for the pin tests ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int orc_hash_index(int32_t res, int32_t log2_table, const int64_t v[3], uint32_t* idx);
void orc_hash_encode(const orc_field* f, const double xhat[3], double* feat);
void orc_sh(int32_t n, const double d[3], double* out);
void orc_field_eval(const orc_field* f, const double p[3], const double d[3],
                    double* sigma, double rgb[3], double* raw /*[d_out] or NULL*/);
int orc_intersect(const double o[3], const double d[3], const double v0[3],
                  const double v1[3], const double v2[3], double* t, double bary[3]);
int orc_closest_hit(const orc_mesh* m, const double o[3], const double d[3], double t_max,
                    double tie_eps, double* t_hit, double bary[3], int* tie);
void orc_scatter(const float* mat, const double d[3], const double n[3], const double u[4],
                 double nd[3], double side[3], double wgt[3], double* R_out);
double orc_fresnel(double cos_i, double eta_i, double eta_t);
void orc_rays_from_camera(const float* cam /*[12]*/, double* o, double* d /*[W*H][3]*/);

/* ---- whole-path renders ---- */
int orc_render(const orc_field* f, const orc_mesh* m, int64_t n, const float* origins,
               const float* dirs, const int64_t* ray_ids, const int32_t* max_bounces,
               const float* lights, int32_t n_lights, const orc_opts* opt, orc_out* out,
               int32_t n_threads);
void orc_field_batch(const orc_field* f, int64_t n, const float* x, const float* d,
                     double* sigma, double* rgb, double* feat, double* raw, int32_t n_threads);
void orc_build_occupancy(const orc_field* f, int32_t res, double thresh, uint8_t* bits,
                         double* margin, int32_t n_threads);

/* ---- proposal sampler and its loss (proposal forward / backward) ---- */
void orc_proposal_weights(const orc_field* p, const double o[3], const double d[3],
                          double lo, double hi, int32_t n, double* w);
void orc_proposal_edges(const double* w, int32_t np, int32_t nf, double lo, double hi,
                        double* edges);
void orc_proposal_targets(const orc_field* f, int64_t n, const float* origins, const float* dirs,
                          double t_near, double t_far, int32_t n_samples, int32_t n_bins,
                          double* lohi, double* target);
double orc_proposal_loss(const orc_field* p, int64_t n_seg, const float* o, const float* d,
                         const float* lohi, const float* target, int32_t n_bins,
                         double* g_table, double* g_mlp, int32_t n_threads);
/* probabilistic tolerance (Higham and Mary) on the rounding error of an
   implementation of orc_proposal_loss's gradient in a format of unit
   roundoff u; K: roundings folded into one node of the chain, lambda: the
   confidence parameter; for tests */
void orc_proposal_grad_bound(const orc_field* p, int64_t n_seg, const float* o, const float* d,
                             const float* lohi, const float* target, int32_t n_bins, double u, double K,
                             double lambda, double* b_table, double* b_mlp);

#ifdef __cplusplus
}
#endif
#endif
