/* FP64 CPU oracle for the hybrid surface-volumetric marcher.
 *
 * TEST INFRASTRUCTURE ONLY -- see oracle.h.  Plain loops in double precision,
 * brute force over every triangle, one sample at a time.
 *
 * Paper: "Dynamic Mesh-Aware Radiance Fields" (Qiao, Gao et al., ICCV 2023).
 *   Sec. 3.1 "Surface Rendering Equation", Eq. 1-4: surface transport, the
 *       ray-casting function t(p, w) and the path throughput recursion.
 *   Sec. 3.1 "Volumetric Rendering Equation", Eq. 8-9: emission-absorption
 *       volume rendering with transmittance T(t) = exp(-int sigma).
 *   Sec. 3.1 "Unifying color space": the field emits linear HDR radiance.
 *   Sec. 3.1 "Shadow rays" and "Hybrid Rendering Algorithm", Eq. 10-13 and
 *       Algorithm 1: per-segment march, then BSDF sampling at the surface hit,
 *       termination on escape / low throughput / bounce limit.
 * The radiance field itself is an Instant-NGP hash grid + small MLPs (Sec. 3.3);
 * its definition follows Mueller et al. 2022 (multiresolution hash encoding).
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11). */
/* The paper only says rays are "randomly cast" (Sec. 3.1, surface LTE); the  */
/* generator is keyed by the seed and counted by (ray id, segment, purpose). */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u01(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

enum { RNG_GLASS = 0, RNG_DIFFUSE = 1, RNG_RR = 2, RNG_EMITTER = 3 };

static void draw(uint32_t seed, int64_t ray, int seg, int purpose, double u[4]) {
  uint32_t ctr[4] = {(uint32_t)ray, (uint32_t)seg, (uint32_t)purpose, 0u};
  uint32_t key[2] = {seed, 0u};
  uint32_t o[4];
  orc_philox4x32_10(ctr, key, o);
  for (int i = 0; i < 4; ++i) u[i] = u01(o[i]);
}

/* ------------------------------------------------------------------------- */
/* Multiresolution hash encoding (Instant-NGP field of Sec. 3.3).            */
/* Level l has grid resolution N_l; a vertex v in {0..N_l}^3 is stored at    */
/* the dense index vx + vy(N+1) + vz(N+1)^2 when (N+1)^3 <= T, otherwise at  */
/* the spatial hash (vx*1 ^ vy*2654435761 ^ vz*805459861) mod T (uint32).     */
/* ------------------------------------------------------------------------- */
int orc_hash_index(int32_t res, int32_t log2_table, const int64_t v[3], uint32_t* idx) {
  int64_t T = (int64_t)1 << log2_table;
  int64_t n1 = (int64_t)res + 1;
  if (n1 * n1 * n1 <= T) {
    *idx = (uint32_t)(v[0] + v[1] * n1 + v[2] * n1 * n1);
    return 1;
  }
  uint32_t h = (uint32_t)v[0] ^ ((uint32_t)v[1] * 2654435761u) ^ ((uint32_t)v[2] * 805459861u);
  *idx = h & (uint32_t)(T - 1);
  return 0;
}

/* xhat in [0,1]^3 (clamped); features level-major, trilinear over 8 corners. */
void orc_hash_encode(const orc_field* f, const double xhat_in[3], double* feat) {
  int64_t T = (int64_t)1 << f->log2_table;
  double xhat[3];
  for (int k = 0; k < 3; ++k) xhat[k] = fmin(fmax(xhat_in[k], 0.0), 1.0);
  for (int l = 0; l < f->n_levels; ++l) {
    int32_t N = f->res[l];
    int64_t v0[3];
    double w[3];
    for (int k = 0; k < 3; ++k) {
      double xl = xhat[k] * (double)N;
      double fl = floor(xl);
      if (fl > (double)(N - 1)) fl = (double)(N - 1);
      v0[k] = (int64_t)fl;
      w[k] = xl - fl;
    }
    for (int c = 0; c < f->feats; ++c) feat[l * f->feats + c] = 0.0;
    for (int corner = 0; corner < 8; ++corner) {
      int64_t v[3];
      double wt = 1.0;
      for (int k = 0; k < 3; ++k) {
        int bit = (corner >> k) & 1;
        v[k] = v0[k] + bit;
        wt *= bit ? w[k] : (1.0 - w[k]);
      }
      uint32_t idx;
      orc_hash_index(N, f->log2_table, v, &idx);
      const float* e = f->table + ((int64_t)l * T + idx) * f->feats;
      for (int c = 0; c < f->feats; ++c) feat[l * f->feats + c] += wt * (double)e[c];
    }
  }
}

/* Real spherical harmonics, orthonormal, degrees l <= 3 (n = 1, 4, 9 or 16
 * components), in Sloan's "Efficient Spherical Harmonic Evaluation" ordering. */
void orc_sh(int32_t n, const double d[3], double* o) {
  double x = d[0], y = d[1], z = d[2];
  double xx = x * x, yy = y * y, zz = z * z;
  o[0] = 0.28209479177387814;
  if (n <= 1) return;
  o[1] = -0.48860251190291987 * y;
  o[2] = 0.48860251190291987 * z;
  o[3] = -0.48860251190291987 * x;
  if (n <= 4) return;
  o[4] = 1.0925484305920792 * x * y;
  o[5] = -1.0925484305920792 * y * z;
  o[6] = 0.31539156525252005 * (3.0 * zz - 1.0);
  o[7] = -1.0925484305920792 * x * z;
  o[8] = 0.54627421529603959 * (xx - yy);
  if (n <= 9) return;
  o[9] = -0.59004358992664352 * y * (3.0 * xx - yy);
  o[10] = 2.8906114426405538 * x * y * z;
  o[11] = -0.45704579946446572 * y * (5.0 * zz - 1.0);
  o[12] = 0.3731763325901154 * z * (5.0 * zz - 3.0);
  o[13] = -0.45704579946446572 * x * (5.0 * zz - 1.0);
  o[14] = 1.4453057213202769 * z * (xx - yy);
  o[15] = -0.59004358992664352 * x * (xx - 3.0 * yy);
}

static double softplus(double x) { return fmax(x, 0.0) + log1p(exp(-fabs(x))); }

/* y[out] = W[out][in] x[in] */
static void matvec(const float* W, int out, int in, const double* x, double* y) {
  for (int i = 0; i < out; ++i) {
    double s = 0.0;
    for (int j = 0; j < in; ++j) s += (double)W[(int64_t)i * in + j] * x[j];
    y[i] = s;
  }
}

static void relu(double* x, int n) {
  for (int i = 0; i < n; ++i) x[i] = x[i] > 0.0 ? x[i] : 0.0;
}

#define MAXW 256

/* The radiance field: density sigma = softplus(raw0 + offset) from the density
 * MLP on the hash features; colour = exp(colour MLP(raw ++ SH(d))), linear HDR
 * radiance (Sec. 3.1 "Unifying color space"). */
void orc_field_eval(const orc_field* f, const double p[3], const double d[3], double* sigma,
                    double rgb[3], double* raw_out) {
  double xhat[3], feat[MAXW], h[MAXW], raw[MAXW] = {0}, cin[MAXW], h2[MAXW], out[4];
  for (int k = 0; k < 3; ++k) xhat[k] = (p[k] - f->aabb_min[k]) / (f->aabb_max[k] - f->aabb_min[k]);
  int nfeat = f->n_levels * f->feats;
  for (int i = 0; i < f->d_in; ++i) feat[i] = 0.0;
  orc_hash_encode(f, xhat, feat);
  (void)nfeat;
  const float* w = f->mlp;
  matvec(w, f->d_hidden, f->d_in, feat, h);
  w += (int64_t)f->d_hidden * f->d_in;
  relu(h, f->d_hidden);
  matvec(w, f->d_out, f->d_hidden, h, raw);
  w += (int64_t)f->d_out * f->d_hidden;
  *sigma = softplus(raw[0] + f->density_offset);
  if (raw_out)
    for (int i = 0; i < f->d_out; ++i) raw_out[i] = raw[i];
  if (f->c_layers <= 0 || !rgb) return;
  for (int i = 0; i < f->c_in; ++i) cin[i] = 0.0;
  for (int i = 0; i < f->d_out; ++i) cin[i] = raw[i];
  orc_sh(f->sh, d, cin + f->d_out);
  matvec(w, f->c_hidden, f->c_in, cin, h);
  w += (int64_t)f->c_hidden * f->c_in;
  relu(h, f->c_hidden);
  for (int layer = 1; layer < f->c_layers; ++layer) {
    matvec(w, f->c_hidden, f->c_hidden, h, h2);
    w += (int64_t)f->c_hidden * f->c_hidden;
    relu(h2, f->c_hidden);
    memcpy(h, h2, sizeof(double) * f->c_hidden);
  }
  matvec(w, 3, f->c_hidden, h, out);
  for (int c = 0; c < 3; ++c) rgb[c] = exp(out[c]);
}

/* ------------------------------------------------------------------------- */
/* Ray casting t(p, w) (Eq. 3): watertight ray-triangle test of Woop, Benthin */
/* and Wald (JCGT 2013), here in double precision, no back-face culling.     */
/* Returns 1 on a hit with t > 0; bary = (U, V, W)/det (weights of v0,v1,v2). */
/* ------------------------------------------------------------------------- */
static void sub3(const double a[3], const double b[3], double r[3]) {
  r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double r[3]) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}

typedef struct { int kx, ky, kz; double Sx, Sy, Sz; } shear_t;

static shear_t make_shear(const double d[3]) {
  shear_t s;
  double ax = fabs(d[0]), ay = fabs(d[1]), az = fabs(d[2]);
  s.kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
  s.kx = (s.kz + 1) % 3;
  s.ky = (s.kx + 1) % 3;
  if (d[s.kz] < 0.0) { int t = s.kx; s.kx = s.ky; s.ky = t; }
  s.Sx = d[s.kx] / d[s.kz];
  s.Sy = d[s.ky] / d[s.kz];
  s.Sz = 1.0 / d[s.kz];
  return s;
}

/* Edge functions of the sheared triangle; returns det, fills U,V,W and t. */
static double tri_edges(const shear_t* s, const double o[3], const double v0[3],
                        const double v1[3], const double v2[3], double uvw[3], double* t) {
  double A[3], B[3], C[3];
  sub3(v0, o, A); sub3(v1, o, B); sub3(v2, o, C);
  double Ax = A[s->kx] - s->Sx * A[s->kz], Ay = A[s->ky] - s->Sy * A[s->kz];
  double Bx = B[s->kx] - s->Sx * B[s->kz], By = B[s->ky] - s->Sy * B[s->kz];
  double Cx = C[s->kx] - s->Sx * C[s->kz], Cy = C[s->ky] - s->Sy * C[s->kz];
  double U = Cx * By - Cy * Bx;
  double V = Ax * Cy - Ay * Cx;
  double W = Bx * Ay - By * Ax;
  double det = U + V + W;
  uvw[0] = U; uvw[1] = V; uvw[2] = W;
  if (det != 0.0) {
    double T = U * (s->Sz * A[s->kz]) + V * (s->Sz * B[s->kz]) + W * (s->Sz * C[s->kz]);
    *t = T / det;
  } else {
    *t = INFINITY;
  }
  return det;
}

int orc_intersect(const double o[3], const double d[3], const double v0[3], const double v1[3],
                  const double v2[3], double* t, double bary[3]) {
  shear_t s = make_shear(d);
  double uvw[3];
  double det = tri_edges(&s, o, v0, v1, v2, uvw, t);
  if ((uvw[0] < 0 || uvw[1] < 0 || uvw[2] < 0) && (uvw[0] > 0 || uvw[1] > 0 || uvw[2] > 0))
    return 0;
  if (det == 0.0) return 0;
  if (!(*t > 0.0)) return 0;
  for (int k = 0; k < 3; ++k) bary[k] = uvw[k] / det;
  return 1;
}

static void tri_verts(const orc_mesh* m, int id, double v[3][3]) {
  for (int a = 0; a < 3; ++a) {
    int vi = m->indices[3 * id + a];
    for (int k = 0; k < 3; ++k) v[a][k] = (double)m->vertices[3 * vi + k];
  }
}

/* Signed world-space distance from the ray's crossing of the triangle plane
 * to the nearest edge line (negative outside), times |cos| of the incidence
 * angle: how far the ray may move sideways before the decision flips. */
static double edge_margin(const double v[3][3], const double d[3], const double uvw[3], double det) {
  double e[3][3], n[3];
  sub3(v[2], v[1], e[0]);
  sub3(v[0], v[2], e[1]);
  sub3(v[1], v[0], e[2]);
  cross3(e[2], e[0], n);                  /* (v1-v0) x (v2-v1), |n| = 2 area */
  double a2 = sqrt(dot3(n, n));
  if (a2 == 0.0) return 0.0;
  double m = INFINITY;
  for (int k = 0; k < 3; ++k) {
    double h = a2 / sqrt(dot3(e[k], e[k]));     /* altitude onto the edge opposite vertex k */
    double dist = uvw[k] / det * h;
    if (dist < m) m = dist;
  }
  return m * fabs(dot3(d, n)) / a2;
}

/* Closest hit by brute force over all triangles: the lexicographic minimum of
 * (t, triangle id) with 0 < t <= t_max.  *tie is set when a single-precision
 * evaluation could decide differently: the best hit lies within tie_eps (world
 * units, scaled by the incidence cosine) of a triangle edge, another hit lies
 * within tie_eps (relative) in t, or a near-miss within tie_eps of an edge, or
 * a hit just outside the t range, would be at least as close. */
int orc_closest_hit(const orc_mesh* m, const double o[3], const double d[3], double t_max,
                    double tie_eps, double* t_hit, double bary_hit[3], int* tie) {
  int best = -1;
  double bt = INFINITY, second = INFINITY, bb[3] = {0, 0, 0};
  double bmargin = INFINITY;
  double near_t = INFINITY;              /* closest t among uncertain triangles */
  if (tie) *tie = 0;
  if (!m || m->nf == 0) return -1;
  shear_t s = make_shear(d);
  for (int i = 0; i < m->nf; ++i) {
    double v[3][3], uvw[3], t;
    tri_verts(m, i, v);
    double det = tri_edges(&s, o, v[0], v[1], v[2], uvw, &t);
    if (det == 0.0) continue;
    int inside = !((uvw[0] < 0 || uvw[1] < 0 || uvw[2] < 0) && (uvw[0] > 0 || uvw[1] > 0 || uvw[2] > 0));
    int in_range = t > 0.0 && t <= t_max;
    if (inside && in_range) {
      if (t < bt || (t == bt && i < best)) {
        second = bt;
        bt = t;
        best = i;
        for (int k = 0; k < 3; ++k) bb[k] = uvw[k] / det;
        bmargin = edge_margin(v, d, uvw, det);
      } else if (t < second) {
        second = t;
      }
    }
    if (tie) {
      double tol_t = tie_eps * fmax(1.0, fabs(t));
      if (t > -tol_t && t <= t_max + tol_t) {
        double mg = edge_margin(v, d, uvw, det);
        if (fabs(mg) < tie_eps) {
          if (t < near_t) near_t = t;
        } else if (inside && !in_range && t < near_t) {
          near_t = t;
        }
      }
    }
  }
  if (tie) {
    if (best >= 0) {
      double tol = tie_eps * fmax(1.0, bt);
      if (bmargin < tie_eps) *tie = 1;
      if (second - bt <= tol) *tie = 1;
      if (near_t <= bt + tol) *tie = 1;
      if (t_max - bt <= tol) *tie = 1;
    } else if (near_t < INFINITY) {
      *tie = 1;
    }
  }
  if (best >= 0) {
    *t_hit = bt;
    for (int k = 0; k < 3; ++k) bary_hit[k] = bb[k];
  }
  return best;
}

/* Record of a ray's decisions that single precision could take the other way
 * (ties).  flag: the ray met one.  Scalar decisions (occupancy of a sample,
 * visibility of a shadow ray, Fresnel choice, roulette, throughput cut-off,
 * emitter choice) are counted in the order the path meets them; bit k of
 * flip takes the other branch of the k-th, so that the outcomes a tie ray
 * can have in single precision are reachable one by one. */
typedef struct {
  int flag;
  int n;
  uint32_t flip;
} tie_t;

/* One flagged scalar decision: returns 1 when its other branch is taken. */
static int tie_decide(tie_t* t) {
  t->flag = 1;
  int k = t->n++;
  return k < 32 && ((t->flip >> k) & 1u);
}

/* Whether triangle h is an outcome single precision can reach for the
 * closest hit of (o, d) on (0, t_max] (h = -1: no hit).  Single precision may
 * miss a hit that lies within tie_eps of an edge or of either end of the t
 * range, may hit a near miss, and may order hits within tie_eps in t either
 * way; so the reachable outcomes are every hit or near miss up to the first
 * hit that is certain (inside by at least tie_eps, and within the range by
 * at least tie_eps relative), within tie_eps of it, and no hit when no
 * certain hit exists.  For a reachable h, *t_h and bary_h are its FP64
 * distance and barycentrics. */
static int hit_reachable(const orc_mesh* m, const double o[3], const double d[3], double t_max,
                         double tie_eps, int h, double* t_h, double bary_h[3]) {
  if (!m) return h < 0;
  shear_t s = make_shear(d);
  double t_cert = INFINITY, th = INFINITY;
  int h_ok = 0;
  for (int i = 0; i < m->nf; ++i) {
    double v[3][3], uvw[3], t;
    tri_verts(m, i, v);
    double det = tri_edges(&s, o, v[0], v[1], v[2], uvw, &t);
    if (det == 0.0) continue;
    int inside = !((uvw[0] < 0 || uvw[1] < 0 || uvw[2] < 0) && (uvw[0] > 0 || uvw[1] > 0 || uvw[2] > 0));
    double tol_t = tie_eps * fmax(1.0, fabs(t));
    double mg = edge_margin(v, d, uvw, det);
    if (inside && mg >= tie_eps && t > tol_t && t <= t_max - tol_t && t < t_cert) t_cert = t;
    if (i == h && t > -tol_t && t <= t_max + tol_t && (inside || fabs(mg) < tie_eps)) {
      h_ok = 1;
      th = t;
      for (int k = 0; k < 3; ++k) bary_h[k] = uvw[k] / det;
    }
  }
  if (h < 0) return t_cert == INFINITY;
  if (!h_ok || th > t_cert + tie_eps * fmax(1.0, t_cert)) return 0;
  *t_h = th;
  return 1;
}

/* Any hit with 0 < t < t_max (shadow rays, Sec. 3.1 "Shadow rays"). */
static int any_hit(const orc_mesh* m, const double o[3], const double d[3], double t_max,
                   double tie_eps, tie_t* tie) {
  if (!m) return 0;
  shear_t s = make_shear(d);
  int hit = 0, near = 0;
  for (int i = 0; i < m->nf; ++i) {
    double v[3][3], uvw[3], t;
    tri_verts(m, i, v);
    double det = tri_edges(&s, o, v[0], v[1], v[2], uvw, &t);
    if (det == 0.0) continue;
    int inside = !((uvw[0] < 0 || uvw[1] < 0 || uvw[2] < 0) && (uvw[0] > 0 || uvw[1] > 0 || uvw[2] > 0));
    double tol_t = tie_eps * fmax(1.0, fabs(t));
    if (inside && t > 0.0 && t < t_max) hit = 1;
    if (t > -tol_t && t < t_max + tol_t) {
      double mg = edge_margin(v, d, uvw, det);
      if (fabs(mg) < tie_eps) near = 1;
      else if (inside && (t < tol_t || t_max - t < tol_t)) near = 1;
    }
  }
  if (near && tie && tie_decide(tie)) hit = !hit;
  return hit;
}

/* ------------------------------------------------------------------------- */
/* Pinhole camera (Algorithm 1: initialise p0, w0 from the pixel and camera  */
/* centre).  Square pixels; vertical field of view fov; up = cam[6..8];      */
/* forward = normalize(look_at - pos); right = up x forward.  Pixel (i, j)   */
/* centre: u = (2(i+.5)/W - 1) tan(fov/2) W/H, v = (1 - 2(j+.5)/H) tan(fov/2). */
/* Ray id = j*W + i.                                                         */
/* ------------------------------------------------------------------------- */
void orc_rays_from_camera(const float* cam, double* o, double* d) {
  double pos[3] = {cam[0], cam[1], cam[2]}, at[3] = {cam[3], cam[4], cam[5]};
  double up0[3] = {cam[6], cam[7], cam[8]};
  double fov = (double)cam[9] * PI / 180.0;
  int W = (int)cam[10], H = (int)cam[11];
  double f[3], r[3], u[3];
  sub3(at, pos, f);
  double nf = sqrt(dot3(f, f));
  for (int k = 0; k < 3; ++k) f[k] /= nf;
  cross3(up0, f, r);
  double nr = sqrt(dot3(r, r));
  for (int k = 0; k < 3; ++k) r[k] /= nr;
  cross3(f, r, u);
  double th = tan(0.5 * fov);
  for (int j = 0; j < H; ++j)
    for (int i = 0; i < W; ++i) {
      double su = (2.0 * (i + 0.5) / W - 1.0) * th * ((double)W / H);
      double sv = (1.0 - 2.0 * (j + 0.5) / H) * th;
      double v[3];
      for (int k = 0; k < 3; ++k) v[k] = f[k] + su * r[k] + sv * u[k];
      double n = sqrt(dot3(v, v));
      int64_t id = (int64_t)j * W + i;
      for (int k = 0; k < 3; ++k) {
        d[3 * id + k] = v[k] / n;
        o[3 * id + k] = pos[k];
      }
    }
}

/* ------------------------------------------------------------------------- */
/* Placement: a world point p maps to the field's frame as R^T (p - c) and a */
/* direction d as R^T d.  The map is rigid, so a ray keeps its parameter t.  */
/* ------------------------------------------------------------------------- */
static void world_to_field(const orc_field* f, const double p[3], const double d[3], double pf[3],
                           double df[3]) {
  if (!f->has_pose) {
    for (int k = 0; k < 3; ++k) { pf[k] = p[k]; df[k] = d[k]; }
    return;
  }
  const double* P = f->pose;   /* R[i][k] = P[4 i + k], c[i] = P[4 i + 3] */
  const double q[3] = {p[0] - P[3], p[1] - P[7], p[2] - P[11]};
  for (int k = 0; k < 3; ++k) {
    pf[k] = P[k] * q[0] + P[4 + k] * q[1] + P[8 + k] * q[2];
    df[k] = P[k] * d[0] + P[4 + k] * d[1] + P[8 + k] * d[2];
  }
}

/* ------------------------------------------------------------------------- */
/* Marching one ray segment (Eq. 10-11, and Eq. 8-9 for the quadrature).     */
/* ------------------------------------------------------------------------- */
static int slab(const orc_field* f, const double o[3], const double d[3], double* t0,
                double* t1) {
  double lo = -INFINITY, hi = INFINITY;
  for (int k = 0; k < 3; ++k) {
    double inv = 1.0 / d[k];
    double a = (f->aabb_min[k] - o[k]) * inv, b = (f->aabb_max[k] - o[k]) * inv;
    if (d[k] == 0.0) {
      if (o[k] < f->aabb_min[k] || o[k] > f->aabb_max[k]) return 0;
      continue;
    }
    if (a > b) { double t = a; a = b; b = t; }
    lo = fmax(lo, a);
    hi = fmin(hi, b);
  }
  *t0 = lo; *t1 = hi;
  return hi > lo;
}

/* Occupancy lookup; a sample within tie_eps of a face between an occupied and
 * an empty cell is a tie, since single precision may place it on the other
 * side (a face between cells of equal state changes nothing). */
static int occ_cell(const orc_opts* opt, const int c[3]) {
  int R = opt->occ_res;
  for (int k = 0; k < 3; ++k)
    if (c[k] < 0 || c[k] >= R) return -1;
  return opt->occ[((int64_t)c[2] * R + c[1]) * R + c[0]] != 0;
}

static int occupied(const orc_opts* opt, const orc_field* f, const double x[3], tie_t* tie) {
  if (!opt->occ) return 1;
  int R = opt->occ_res;
  int c[3];
  double xr[3];
  for (int k = 0; k < 3; ++k) {
    double xh = (x[k] - f->aabb_min[k]) / (f->aabb_max[k] - f->aabb_min[k]);
    xr[k] = xh * R;
    int ci = (int)floor(xr[k]);
    c[k] = ci < 0 ? 0 : (ci >= R ? R - 1 : ci);
  }
  int here = occ_cell(opt, c), near = 0;
  for (int k = 0; k < 3; ++k) {
    double face = floor(xr[k] + 0.5);
    if (fabs(xr[k] - face) < opt->tie_eps * R) {
      int nb[3] = {c[0], c[1], c[2]};
      nb[k] = (face > xr[k] || face == (double)c[k] + 1.0) ? c[k] + 1 : c[k] - 1;
      if (nb[k] == c[k]) continue;
      int there = occ_cell(opt, nb);
      if (there >= 0 && there != here) near = 1;
    }
  }
  if (near && tie_decide(tie)) here = !here;
  return here;
}

/* What a sample's shadow mask needs: the meshes, the lights, the mask value
 * and the segment in world coordinates (the field may be placed elsewhere). */
typedef struct {
  const orc_mesh* m;
  const float* lights;       /* [n_lights][6]: position, intensity */
  int32_t n_lights;
  double mask;
  const double* o_world;
  const double* d_world;
} shadow_ctx;

/* Shadow mask m(p_t) of one sample: 1, times the mask value for every light
 * that a mesh hides from the sample's world position. */
static double sample_mask(const shadow_ctx* sh, const orc_opts* opt, double tm, tie_t* tie) {
  double m = 1.0, x[3];
  for (int k = 0; k < 3; ++k) x[k] = sh->o_world[k] + tm * sh->d_world[k];
  for (int li = 0; li < sh->n_lights; ++li) {
    const float* lt = sh->lights + 6 * li;
    double sd[3] = {lt[0] - x[0], lt[1] - x[1], lt[2] - x[2]};
    double dist = sqrt(dot3(sd, sd));
    for (int k = 0; k < 3; ++k) sd[k] /= dist;
    if (any_hit(sh->m, x, sd, dist, opt->tie_eps, tie)) m *= sh->mask;
  }
  return m;
}

/* Composite one interval [a, b] at its midpoint: alpha = 1 - exp(-sigma D),
 * L += T alpha m c with the sample's shadow mask m (1 without shadows),
 * T *= (1 - alpha).  Returns the number of field samples. */
static int composite_interval(const orc_field* f, const orc_opts* opt, const double o[3],
                              const double d[3], double a, double b, double T[3], double L[3],
                              tie_t* tie, const shadow_ctx* sh) {
  if (!(b > a)) return 0;
  double tm = 0.5 * (a + b), D = b - a, x[3], sigma, rgb[3];
  for (int k = 0; k < 3; ++k) x[k] = o[k] + tm * d[k];
  if (!occupied(opt, f, x, tie)) return 0;
  orc_field_eval(f, x, d, &sigma, rgb, NULL);
  double m = sh ? sample_mask(sh, opt, tm, tie) : 1.0;
  double alpha = -expm1(-sigma * D);
  for (int c = 0; c < 3; ++c) {
    L[c] += T[c] * alpha * m * rgb[c];
    T[c] *= (1.0 - alpha);
  }
  return 1;
}

/* Proposal weights w_j = T_j alpha_j on n uniform intervals of [lo, hi]. */
void orc_proposal_weights(const orc_field* p, const double o[3], const double d[3], double lo,
                          double hi, int32_t n, double* w) {
  double Tr = 1.0, step = (hi - lo) / n;
  for (int j = 0; j < n; ++j) {
    double a = lo + j * step, b = lo + (j + 1) * step, tm = 0.5 * (a + b), x[3], sigma;
    for (int k = 0; k < 3; ++k) x[k] = o[k] + tm * d[k];
    orc_field_eval(p, x, d, &sigma, NULL, NULL);
    double alpha = -expm1(-sigma * (b - a));
    w[j] = Tr * alpha;
    Tr *= (1.0 - alpha);
  }
}

/* Fine edges of the proposal sampler (the learned sampler is not in the
 * paper; it follows the proposal resampling of Mip-NeRF 360): the proposal
 * weights w_j on np uniform intervals of [lo, hi] are dilated to
 * max(w_{j-1}, w_j, w_{j+1}), their mean is added to every interval (a
 * half-and-half mixture with a uniform density) and so is 1e-3/np; the
 * resulting piecewise-constant density is inverted at u = k/nf for the
 * nf + 1 edges, edges[0] = lo and edges[nf] = hi. */
void orc_proposal_edges(const double* w, int32_t np, int32_t nf, double lo, double hi,
                        double* edges) {
  double wd[1024], cdf[1025], sw = 0.0, tot = 0.0;
  for (int j = 0; j < np; ++j) {
    double m = w[j];
    if (j > 0 && w[j - 1] > m) m = w[j - 1];
    if (j + 1 < np && w[j + 1] > m) m = w[j + 1];
    wd[j] = m;
    sw += m;
  }
  cdf[0] = 0.0;
  for (int j = 0; j < np; ++j) { tot += wd[j] + sw / np + 1e-3 / np; cdf[j + 1] = tot; }
  double step = (hi - lo) / np;
  int j = 0;
  for (int k = 0; k <= nf; ++k) {
    double u = (double)k / nf * tot;
    if (k == 0) { edges[k] = lo; continue; }
    if (k == nf) { edges[k] = hi; continue; }
    while (j < np - 1 && cdf[j + 1] < u) ++j;
    double fr = (u - cdf[j]) / (cdf[j + 1] - cdf[j]);
    edges[k] = lo + (j + fr) * step;
  }
}

/* Segment march over [lo, hi]: uniform grid of n_samples intervals of width
 * (t_far - t_near)/n_samples anchored at t_a, or, with a proposal, the
 * n_fine intervals between the edges of orc_proposal_edges. */
static int64_t march(const orc_field* f, const orc_opts* opt, const double o_world[3],
                     const double d_world[3], double t_a, double t_hit, double T[3], double L[3],
                     tie_t* tie, const shadow_ctx* sh_in) {
  if (!f) return 0;
  shadow_ctx shc;
  const shadow_ctx* sh = NULL;
  if (sh_in) {
    shc = *sh_in;
    shc.o_world = o_world;
    shc.d_world = d_world;
    sh = &shc;
  }
  /* the segment in the field's frame (the proposal field shares that frame) */
  double o[3], d[3];
  world_to_field(f, o_world, d_world, o, d);
  double span = opt->t_far - opt->t_near;
  double box0, box1;
  if (!slab(f, o, d, &box0, &box1)) return 0;
  double lo = fmax(t_a, box0), hi = fmin(fmin(t_a + span, t_hit), box1);
  if (!(hi > lo)) return 0;
  int64_t ns = 0;
  if (opt->proposal) {
    int np = opt->n_prop, nf = opt->n_fine;
    double w[1024], edges[1025];
    orc_proposal_weights(opt->proposal, o, d, lo, hi, np, w);
    orc_proposal_edges(w, np, nf, lo, hi, edges);
    for (int k = 0; k < nf; ++k) ns += composite_interval(f, opt, o, d, edges[k], edges[k + 1], T, L, tie, sh);
    return ns;
  }
  double delta = span / opt->n_samples;
  for (int k = 0; k < opt->n_samples; ++k) {
    double a = t_a + k * delta, b = t_a + (k + 1) * delta;
    if (b <= lo) continue;
    if (a >= hi) break;
    ns += composite_interval(f, opt, o, d, fmax(a, lo), fmin(b, hi), T, L, tie, sh);
  }
  return ns;
}

/* Several fields in one scene (each a NeRF object with its own placement):
 * the medium's density is the sum of the fields' densities, each zero outside
 * its own box, and its colour their density-weighted mean, the usual rule for
 * overlapping emission-absorption media.  Every grid interval of the uniform
 * march is cut at each box face the ray crosses inside it, so every piece lies
 * wholly inside or outside each box, and each piece is composited at its
 * midpoint as in the single-field march (with one field the two agree).
 * A piece inside no box, or whose fields are all empty there by their
 * occupancy grids, leaves L and T unchanged. */
static int64_t march_fields(const orc_opts* opt, const double o_world[3], const double d_world[3],
                            double t_a, double t_hit, double T[3], double L[3], tie_t* tie,
                            const shadow_ctx* sh_in) {
  enum { MAXF = 16 };
  int nf = opt->n_fields;
  if (nf > MAXF) nf = MAXF;
  double span = opt->t_far - opt->t_near;
  double t_b = fmin(t_a + span, t_hit);
  double of[MAXF][3], df[MAXF][3], in[MAXF], out[MAXF];
  int valid[MAXF];
  orc_opts fo[MAXF];
  for (int k = 0; k < nf; ++k) {
    world_to_field(opt->fields[k], o_world, d_world, of[k], df[k]);
    double b0, b1;
    valid[k] = slab(opt->fields[k], of[k], df[k], &b0, &b1);
    in[k] = fmax(t_a, b0);
    out[k] = fmin(t_b, b1);
    if (!(out[k] > in[k])) valid[k] = 0;
    fo[k] = *opt;
    fo[k].occ = opt->field_occ ? opt->field_occ[k] : NULL;
    fo[k].occ_res = opt->field_occ_res ? opt->field_occ_res[k] : 0;
  }
  shadow_ctx shc;
  if (sh_in) {
    shc = *sh_in;
    shc.o_world = o_world;
    shc.d_world = d_world;
  }
  int64_t ns = 0;
  double delta = span / opt->n_samples;
  for (int j = 0; j < opt->n_samples; ++j) {
    double a = t_a + j * delta, b = fmin(t_a + (j + 1) * delta, t_b);
    if (a >= t_b) break;
    double cut[2 * MAXF + 2];
    int nc = 0;
    cut[nc++] = a;
    for (int k = 0; k < nf; ++k) {
      if (!valid[k]) continue;
      if (in[k] > a && in[k] < b) cut[nc++] = in[k];
      if (out[k] > a && out[k] < b) cut[nc++] = out[k];
    }
    cut[nc++] = b;
    for (int x = 1; x < nc; ++x)        /* insertion sort of the cut points */
      for (int y = x; y > 0 && cut[y] < cut[y - 1]; --y) { double t = cut[y]; cut[y] = cut[y - 1]; cut[y - 1] = t; }
    for (int c = 0; c + 1 < nc; ++c) {
      double lo = cut[c], hi = cut[c + 1];
      if (!(hi > lo)) continue;
      double tm = 0.5 * (lo + hi), D = hi - lo, sig = 0.0, sc[3] = {0, 0, 0};
      int any = 0;
      for (int k = 0; k < nf; ++k) {
        if (!valid[k] || lo < in[k] || hi > out[k]) continue;
        double x[3], sk, ck[3];
        for (int i = 0; i < 3; ++i) x[i] = of[k][i] + tm * df[k][i];
        if (!occupied(&fo[k], opt->fields[k], x, tie)) continue;
        orc_field_eval(opt->fields[k], x, df[k], &sk, ck, NULL);
        sig += sk;
        for (int i = 0; i < 3; ++i) sc[i] += sk * ck[i];
        ++any;
      }
      if (!any) continue;
      ns += any;
      double m = sh_in ? sample_mask(&shc, opt, tm, tie) : 1.0;
      double alpha = -expm1(-sig * D);
      for (int i = 0; i < 3; ++i) {
        double ci = sig > 0.0 ? sc[i] / sig : 0.0;
        L[i] += T[i] * alpha * m * ci;
        T[i] *= (1.0 - alpha);
      }
    }
  }
  return ns;
}

/* Several fields, each sampled by its own proposal.  Reading: with boxes
 * that do not overlap, every point of the segment belongs to at most one
 * field, so the summed medium is the fields one after another; each is
 * marched on its own clipped range with its own proposal (the single-field
 * proposal march) in the order the ray enters the boxes. */
static int64_t march_fields_proposal(const orc_opts* opt, const double o_world[3], const double d_world[3],
                                     double t_a, double t_hit, double T[3], double L[3], tie_t* tie,
                                     const shadow_ctx* sh_in) {
  enum { MAXF = 16 };
  int nf = opt->n_fields < MAXF ? opt->n_fields : MAXF;
  double entry[MAXF];
  int order[MAXF];
  for (int k = 0; k < nf; ++k) {
    double of[3], df[3], b0, b1;
    world_to_field(opt->fields[k], o_world, d_world, of, df);
    entry[k] = slab(opt->fields[k], of, df, &b0, &b1) ? b0 : INFINITY;
    int j = k;
    while (j > 0 && entry[order[j - 1]] > entry[k]) { order[j] = order[j - 1]; --j; }
    order[j] = k;
  }
  int64_t ns = 0;
  for (int i = 0; i < nf; ++i) {
    const int k = order[i];
    orc_opts fo = *opt;
    fo.proposal = opt->field_proposals[k];
    fo.occ = opt->field_occ ? opt->field_occ[k] : NULL;
    fo.occ_res = opt->field_occ_res ? opt->field_occ_res[k] : 0;
    ns += march(opt->fields[k], &fo, o_world, d_world, t_a, t_hit, T, L, tie, sh_in);
  }
  return ns;
}

/* ------------------------------------------------------------------------- */
/* Surface interaction (Eq. 12-13): perfect mirror, smooth dielectric with   */
/* exact unpolarised Fresnel (reflect with probability R, else refract),     */
/* Lambertian with cosine-weighted sampling (Malley) and, at each diffuse    */
/* hit, one shadow ray to every point light (Sec. 3.1 "Shadow rays").        */
/* ------------------------------------------------------------------------- */
static double fresnel(double cos_i, double eta_i, double eta_t, double* cos_t) {
  double eta = eta_i / eta_t;
  double sin2t = eta * eta * (1.0 - cos_i * cos_i);
  if (sin2t >= 1.0) { *cos_t = 0.0; return 1.0; }
  double ct = sqrt(1.0 - sin2t);
  *cos_t = ct;
  double rs = (eta_i * cos_i - eta_t * ct) / (eta_i * cos_i + eta_t * ct);
  double rp = (eta_i * ct - eta_t * cos_i) / (eta_i * ct + eta_t * cos_i);
  return 0.5 * (rs * rs + rp * rp);
}

/* Orthonormal basis around unit n (Duff et al., JCGT 2017). */
static void onb(const double n[3], double b1[3], double b2[3]) {
  double sgn = copysign(1.0, n[2]);
  double a = -1.0 / (sgn + n[2]);
  double b = n[0] * n[1] * a;
  b1[0] = 1.0 + sgn * n[0] * n[0] * a; b1[1] = sgn * b; b1[2] = -sgn * n[0];
  b2[0] = b; b2[1] = sgn + n[1] * n[1] * a; b2[2] = -n[1];
}

/* BSDF sampling at a surface hit (Eq. 13).  mat = {kind, ior, albedo rgb};
 * d = unit incoming direction; n = unit geometric normal (either side);
 * u = four uniforms.  Writes the new direction, the side to offset the
 * spawn point towards, and the throughput factor f|cos|/P:
 *   mirror  d' = d - 2(d.n)n, factor 1;
 *   glass   reflect if u0 < R (exact unpolarised Fresnel, R = 1 under total
 *           internal reflection), else refract by Snell's law; factor 1, so
 *           throughput never grows (no radiance scaling by eta^2);
 *   diffuse cosine-weighted direction about the normal facing the incoming
 *           ray, factor = albedo (f = albedo/pi, P = cos/pi). */
void orc_scatter(const float* mat, const double d[3], const double n[3], const double u[4],
                 double nd[3], double side[3], double wgt[3], double* R_out) {
  int kind = (int)mat[0];
  double dn = dot3(d, n), nf[3];
  for (int k = 0; k < 3; ++k) nf[k] = dn < 0.0 ? n[k] : -n[k];
  for (int c = 0; c < 3; ++c) wgt[c] = 1.0;
  if (kind == 0) {
    for (int k = 0; k < 3; ++k) { nd[k] = d[k] - 2.0 * dn * n[k]; side[k] = nf[k]; }
  } else if (kind == 1) {
    double ior = mat[1];
    int entering = dn < 0.0;
    double eta_i = entering ? 1.0 : ior, eta_t = entering ? ior : 1.0, ct;
    double ci = fabs(dn);
    double R = fresnel(ci, eta_i, eta_t, &ct);
    if (R_out) *R_out = R;
    if (u[0] < R) {
      for (int k = 0; k < 3; ++k) { nd[k] = d[k] - 2.0 * dn * n[k]; side[k] = nf[k]; }
    } else {
      double eta = eta_i / eta_t;
      for (int k = 0; k < 3; ++k) {
        nd[k] = eta * d[k] + (eta * ci - ct) * nf[k];
        side[k] = -nf[k];
      }
      double nn = sqrt(dot3(nd, nd));
      for (int k = 0; k < 3; ++k) nd[k] /= nn;
    }
  } else {
    double b1[3], b2[3];
    double rr = sqrt(u[0]), phi = 2.0 * PI * u[1];
    double lx = rr * cos(phi), ly = rr * sin(phi), lz = sqrt(fmax(0.0, 1.0 - u[0]));
    onb(nf, b1, b2);
    for (int k = 0; k < 3; ++k) { nd[k] = lx * b1[k] + ly * b2[k] + lz * nf[k]; side[k] = nf[k]; }
    for (int c = 0; c < 3; ++c) wgt[c] = mat[2 + c];
  }
}

double orc_fresnel(double cos_i, double eta_i, double eta_t) {
  double ct;
  return fresnel(cos_i, eta_i, eta_t, &ct);
}

static int near_rel(double a, double b, double eps) {
  return fabs(a - b) <= eps * fmax(fabs(b), 1e-30);
}

/* Light sampling toward emitting triangles (Eq. 12's L_e read as area
 * lights; the paper estimates light sources but sets out no sampling rule).
 * Reading: triangle k of the emitters (faces whose material emits, in face
 * order) is chosen with probability p_k = w_k / W, w_k = sum of its emitted
 * radiance over the three channels (not its power, so the choice does not
 * change when a mesh deforms), by the first k with u0 W < w_0 + ... + w_k; on
 * it the point x = (1 - s) v0 + s (1 - u2) v1 + s u2 v2, s = sqrt(u1), is
 * uniform by area (pdf 1 / A_k).  The estimate of the light reflected by a
 * Lambertian point p with normal nf is
 *     (albedo / pi) L_e cos_p cos_x / |x - p|^2 * A_k / p_k,
 * cos_p = nf . l, cos_x = |n_k . l| (emitters are two-sided, as the L_e term
 * is added on either side), zero when either cosine is not positive or a
 * mesh lies between: a ray from p + 1e-4 nf toward x finds a triangle before
 * (1 - 1e-3) of the way.  The light the sample carries crosses the medium
 * from p + 1e-4 nf to x, so the estimate is multiplied by the transmittance
 * of that segment (shadow_transmittance); a path that reaches the emitter
 * by its own bounce is attenuated by the same medium (Eq. 10 then Eq. 12),
 * so both estimate the same light.  Flagged decisions of the choice, the
 * shadow ray and the occupancy of the segment's samples go to *tie. */
static double shadow_transmittance(const orc_opts* opt, const orc_field* f, const double so[3],
                                   const double sd[3], double len, tie_t* tie);

static void emitter_sample(const orc_mesh* m, const orc_opts* opt, const orc_field* f, const double p[3],
                           const double nf[3], const float* mat, const double u[4], double tie_eps,
                           double tie_rel, double L_add[3], tie_t* tie) {
  for (int c = 0; c < 3; ++c) L_add[c] = 0.0;
  double W = 0.0;
  for (int i = 0; i < m->nf; ++i) {
    const float* em = m->materials + 8 * m->mat_ids[i] + 5;
    W += (double)em[0] + (double)em[1] + (double)em[2];
  }
  if (!(W > 0.0)) return;
  double target = u[0] * W, cum = 0.0;
  int k = -1, prev = -1, alt = -1, want_next = 0;
  double wk = 0.0, wprev = 0.0, walt = 0.0;
  for (int i = 0; i < m->nf; ++i) {
    const float* em = m->materials + 8 * m->mat_ids[i] + 5;
    double w = (double)em[0] + (double)em[1] + (double)em[2];
    if (!(w > 0.0)) continue;
    double lo = cum;
    cum += w;
    if (k < 0 && target < cum) {
      k = i;
      wk = w;
      /* near a boundary of its share: the neighbour across it is the other outcome */
      if (lo > 0.0 && near_rel(target, lo, tie_rel)) { alt = prev; walt = wprev; }
      else if (cum < W && near_rel(target, cum, tie_rel)) want_next = 1;
    } else if (want_next && alt < 0) {
      alt = i;
      walt = w;
    }
    prev = i;
    wprev = w;
  }
  if (k < 0) return;                     /* u0 < 1 always finds one; kept for safety */
  if (alt >= 0 && tie_decide(tie)) { k = alt; wk = walt; }
  double v[3][3], e1[3], e2[3], nk[3], x[3], wi[3], l[3];
  tri_verts(m, k, v);
  double s = sqrt(u[1]);
  for (int j = 0; j < 3; ++j) x[j] = (1.0 - s) * v[0][j] + s * (1.0 - u[2]) * v[1][j] + s * u[2] * v[2][j];
  sub3(v[1], v[0], e1);
  sub3(v[2], v[0], e2);
  cross3(e1, e2, nk);
  double a2 = sqrt(dot3(nk, nk));       /* twice the area */
  sub3(x, p, wi);
  double d2 = dot3(wi, wi), dist = sqrt(d2);
  for (int j = 0; j < 3; ++j) l[j] = wi[j] / dist;
  double cos_p = dot3(nf, l), cos_x = fabs(dot3(nk, l)) / a2;
  if (!(cos_p > 0.0) || !(cos_x > 0.0)) return;
  double so[3], sd[3];
  for (int j = 0; j < 3; ++j) so[j] = p[j] + 1e-4 * nf[j];
  sub3(x, so, sd);
  double sdist = sqrt(dot3(sd, sd));
  for (int j = 0; j < 3; ++j) sd[j] /= sdist;
  if (any_hit(m, so, sd, (1.0 - 1e-3) * sdist, tie_eps, tie)) return;
  const float* em = m->materials + 8 * m->mat_ids[k] + 5;
  double g = cos_p * cos_x / d2 * (0.5 * a2) * (W / wk) / PI;
  g *= shadow_transmittance(opt, f, so, sd, sdist, tie);
  for (int c = 0; c < 3; ++c) L_add[c] = (double)mat[2 + c] * (double)em[c] * g;
}

/* Optical depth of one field along [0, len] of the ray so + t sd (world):
 * its density integrated by the midpoint rule over the march's grid
 * (spacing (t_far - t_near)/n_samples from t = 0, or /light_depth_samples
 * when that is set), each interval clipped to
 * the segment and to the field's box; samples in empty occupancy cells count
 * zero. */
static double field_depth(const orc_field* f, const orc_opts* opt, const double so[3], const double sd[3],
                          double len, tie_t* tie) {
  double o[3], d[3], b0, b1;
  world_to_field(f, so, sd, o, d);
  if (!slab(f, o, d, &b0, &b1)) return 0.0;
  double lo = fmax(0.0, b0), hi = fmin(len, b1);
  if (!(hi > lo)) return 0.0;
  int ns = opt->light_depth_samples > 0 ? opt->light_depth_samples : opt->n_samples;
  double delta = (opt->t_far - opt->t_near) / ns, tau = 0.0;
  for (int k = 0;; ++k) {
    double a = k * delta, b = (k + 1) * delta;
    if (b <= lo) continue;
    if (a >= hi) break;
    a = fmax(a, lo);
    b = fmin(b, hi);
    double tm = 0.5 * (a + b), x[3], sigma;
    for (int j = 0; j < 3; ++j) x[j] = o[j] + tm * d[j];
    if (!occupied(opt, f, x, tie)) continue;
    orc_field_eval(f, x, d, &sigma, NULL, NULL);
    tau += sigma * (b - a);
  }
  return tau;
}

/* Transmittance exp(-optical depth) of the medium along a light sample's
 * shadow segment: the field's, or with several fields the sum of each
 * field's own depth (the medium is their summed density). */
static double shadow_transmittance(const orc_opts* opt, const orc_field* f, const double so[3],
                                   const double sd[3], double len, tie_t* tie) {
  double tau = 0.0;
  if (opt->n_fields > 0) {
    for (int k = 0; k < opt->n_fields; ++k) {
      orc_opts fo = *opt;
      fo.occ = opt->field_occ ? opt->field_occ[k] : NULL;
      fo.occ_res = opt->field_occ_res ? opt->field_occ_res[k] : 0;
      tau += field_depth(opt->fields[k], &fo, so, sd, len, tie);
    }
  } else if (f) {
    tau = field_depth(f, opt, so, sd, len, tie);
  }
  return exp(-tau);
}

typedef struct {
  const orc_field* f;
  const orc_mesh* m;
  const float* origins;
  const float* dirs;
  const int64_t* ray_ids;
  const int32_t* max_bounces;
  const float* lights;
  int32_t n_lights;
  const orc_opts* opt;
  orc_out* out;
  int64_t begin, end;
} job_t;

static void render_ray(const job_t* J, int64_t r) {
  const orc_opts* opt = J->opt;
  const orc_mesh* m = J->m;
  int mb = J->max_bounces ? J->max_bounces[r] : opt->max_bounces;
  int64_t rid = J->ray_ids ? J->ray_ids[r] : r;
  double o[3], d[3], T[3] = {1, 1, 1}, L[3] = {0, 0, 0};
  for (int k = 0; k < 3; ++k) { o[k] = J->origins[3 * r + k]; d[k] = J->dirs[3 * r + k]; }
  int nscat = 0, segs = 0, after_diffuse = 0, invalid = 0;
  tie_t tie = {0, 0, opt->flip ? opt->flip[r] : 0u};
  int64_t nsamp = 0;
  int stride = opt->max_bounces + 1;
  if (J->out->hit_ids)
    for (int s = 0; s < stride; ++s) J->out->hit_ids[r * stride + s] = -1;
  double span = opt->t_far - opt->t_near;
  for (int s = 0; s <= mb; ++s) {
    double t_a = (s == 0) ? opt->t_near : 0.0;
    double t_max = (s == 0) ? opt->t_far : span;
    double t_hit = INFINITY, bary[3];
    int t_tie = 0;
    int hit = m ? orc_closest_hit(m, o, d, t_max, opt->tie_eps, &t_hit, bary, &t_tie) : -1;
    tie.flag |= t_tie;
    if (opt->force_hits && opt->force_hits[r * stride + s] != hit) {
      /* an outcome single precision reached instead: taken if reachable */
      int h = opt->force_hits[r * stride + s];
      double th = 0.0, bh[3];
      if (h >= -1 && h < (m ? m->nf : 0) && hit_reachable(m, o, d, t_max, opt->tie_eps, h, &th, bh)) {
        hit = h;
        if (h >= 0) {
          t_hit = th;
          for (int k = 0; k < 3; ++k) bary[k] = bh[k];
        }
      } else {
        invalid = 1;
      }
    }
    if (J->out->hit_ids) J->out->hit_ids[r * stride + s] = hit;
    shadow_ctx sh = {m, J->lights, J->n_lights, opt->shadow_mask, NULL, NULL};
    if (opt->n_fields > 0 && opt->field_proposals)
      nsamp += march_fields_proposal(opt, o, d, t_a, hit >= 0 ? t_hit : INFINITY, T, L, &tie,
                                     opt->sample_shadows && m && J->n_lights > 0 ? &sh : NULL);
    else if (opt->n_fields > 0)
      nsamp += march_fields(opt, o, d, t_a, hit >= 0 ? t_hit : INFINITY, T, L, &tie,
                            opt->sample_shadows && m && J->n_lights > 0 ? &sh : NULL);
    else
      nsamp += march(J->f, opt, o, d, t_a, hit >= 0 ? t_hit : INFINITY, T, L, &tie,
                     opt->sample_shadows && m && J->n_lights > 0 ? &sh : NULL);
    ++segs;
    if (hit < 0) break;                  /* escaped the scene: background is 0 */
    if (!(opt->sample_emitters && after_diffuse)) {   /* Eq. 12: emitted radiance, attenuated by the segment */
      const float* em = m->materials + 8 * m->mat_ids[hit] + 5;
      for (int c = 0; c < 3; ++c) L[c] += T[c] * (double)em[c];
    }
    if (s == mb) break;                  /* bounce limit: stop at the surface   */
    double v[3][3], e1[3], e2[3], n[3], p[3], nd[3], side[3];
    tri_verts(m, hit, v);
    sub3(v[1], v[0], e1);
    sub3(v[2], v[0], e2);
    cross3(e1, e2, n);
    double nl = sqrt(dot3(n, n));
    for (int k = 0; k < 3; ++k) n[k] /= nl;
    for (int k = 0; k < 3; ++k) p[k] = o[k] + t_hit * d[k];
    double dn = dot3(d, n);
    double nf[3];                        /* normal on the side the ray came from */
    for (int k = 0; k < 3; ++k) nf[k] = dn < 0.0 ? n[k] : -n[k];
    const float* mat = m->materials + 8 * m->mat_ids[hit];
    int kind = (int)mat[0];
    if (kind == 2) {                     /* Lambertian: shadow ray to every light */
      for (int li = 0; li < J->n_lights; ++li) {
        const float* lt = J->lights + 6 * li;
        double lp[3] = {lt[0], lt[1], lt[2]}, wi[3], so[3], sd[3];
        sub3(lp, p, wi);
        double d2 = dot3(wi, wi), dist = sqrt(d2);
        double cosl = dot3(nf, wi) / dist;
        if (cosl <= 0.0) continue;
        for (int k = 0; k < 3; ++k) so[k] = p[k] + 1e-4 * nf[k];
        sub3(lp, so, sd);
        double sdist = sqrt(dot3(sd, sd));
        for (int k = 0; k < 3; ++k) sd[k] /= sdist;
        int blocked = any_hit(m, so, sd, sdist, opt->tie_eps, &tie);
        if (blocked) continue;
        for (int c = 0; c < 3; ++c) L[c] += T[c] * ((double)mat[2 + c] / PI) * lt[3 + c] * cosl / d2;
      }
      if (opt->sample_emitters) {        /* one light sample on the emitting triangles */
        double ue[4], Le[3];
        draw(opt->seed, rid, s, RNG_EMITTER, ue);
        emitter_sample(m, opt, J->f, p, nf, mat, ue, opt->tie_eps, opt->tie_rel, Le, &tie);
        for (int c = 0; c < 3; ++c) L[c] += T[c] * Le[c];
      }
    }
    after_diffuse = kind == 2;
    double u[4];
    draw(opt->seed, rid, s, kind == 1 ? RNG_GLASS : RNG_DIFFUSE, u);
    double wgt[3], R = -1.0;
    orc_scatter(mat, d, n, u, nd, side, wgt, &R);
    if (kind == 1 && R < 1.0 && near_rel(u[0], R, opt->tie_rel) && tie_decide(&tie)) {
      u[0] = u[0] < R ? 1.0 : 0.0;       /* the other branch of the Fresnel choice */
      orc_scatter(mat, d, n, u, nd, side, wgt, &R);
    }
    for (int c = 0; c < 3; ++c) T[c] *= wgt[c];
    ++nscat;
    if (opt->rr_after >= 0 && nscat >= opt->rr_after) {   /* Russian roulette */
      double q = fmin(1.0, fmax(T[0], fmax(T[1], T[2])));
      double u[4];
      draw(opt->seed, rid, s, RNG_RR, u);
      int survive = u[0] < q;
      if (q < 1.0 && near_rel(u[0], q, opt->tie_rel) && tie_decide(&tie)) survive = !survive;
      if (!survive) { T[0] = T[1] = T[2] = 0.0; break; }
      for (int c = 0; c < 3; ++c) T[c] /= q;
    }
    double tmax = fmax(T[0], fmax(T[1], T[2]));
    int cut = tmax < opt->t_min_throughput;
    if (near_rel(tmax, opt->t_min_throughput, opt->tie_rel) && tie_decide(&tie)) cut = !cut;
    if (cut) break;
    for (int k = 0; k < 3; ++k) { o[k] = p[k] + 1e-4 * side[k]; d[k] = nd[k]; }
  }
  for (int c = 0; c < 3; ++c) {
    J->out->radiance[3 * r + c] = L[c];
    J->out->throughput[3 * r + c] = T[c];
  }
  J->out->bounces[r] = nscat;
  if (J->out->tie) J->out->tie[r] = (uint8_t)tie.flag;
  if (J->out->invalid) J->out->invalid[r] = (uint8_t)invalid;
  if (J->out->n_flagged) J->out->n_flagged[r] = tie.n;
  if (J->out->samples) J->out->samples[r] = nsamp;
  if (J->out->segments) J->out->segments[r] = segs;
}

static void* render_worker(void* arg) {
  job_t* J = (job_t*)arg;
  for (int64_t r = J->begin; r < J->end; ++r) render_ray(J, r);
  return NULL;
}

int orc_render(const orc_field* f, const orc_mesh* m, int64_t n, const float* origins,
               const float* dirs, const int64_t* ray_ids, const int32_t* max_bounces,
               const float* lights, int32_t n_lights, const orc_opts* opt, orc_out* out,
               int32_t n_threads) {
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  pthread_t th[256];
  job_t jobs[256];
  int64_t chunk = (n + n_threads - 1) / n_threads;
  for (int i = 0; i < n_threads; ++i) {
    job_t J = {f, m, origins, dirs, ray_ids, max_bounces, lights, n_lights, opt, out,
               i * chunk, (i + 1) * chunk < n ? (i + 1) * chunk : n};
    if (J.begin > n) J.begin = n;
    jobs[i] = J;
    pthread_create(&th[i], NULL, render_worker, &jobs[i]);
  }
  for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Batched field evaluation, occupancy grid.                                 */
/* ------------------------------------------------------------------------- */
typedef struct {
  const orc_field* f;
  const float* x;
  const float* d;
  double *sigma, *rgb, *feat, *raw;
  int64_t begin, end;
} fjob_t;

static void* field_worker(void* arg) {
  fjob_t* J = (fjob_t*)arg;
  const orc_field* f = J->f;
  for (int64_t i = J->begin; i < J->end; ++i) {
    double pw[3], dw[3] = {0, 0, 1}, p[3], d[3], xhat[3], rgb[3], raw[MAXW];
    for (int k = 0; k < 3; ++k) pw[k] = J->x[3 * i + k];
    if (J->d)
      for (int k = 0; k < 3; ++k) dw[k] = J->d[3 * i + k];
    world_to_field(f, pw, dw, p, d);
    orc_field_eval(f, p, d, &J->sigma[i], J->rgb ? rgb : NULL, raw);
    if (J->rgb)
      for (int c = 0; c < 3; ++c) J->rgb[3 * i + c] = rgb[c];
    if (J->raw)
      for (int c = 0; c < f->d_out; ++c) J->raw[(int64_t)i * f->d_out + c] = raw[c];
    if (J->feat) {
      for (int k = 0; k < 3; ++k) xhat[k] = (p[k] - f->aabb_min[k]) / (f->aabb_max[k] - f->aabb_min[k]);
      orc_hash_encode(f, xhat, J->feat + (int64_t)i * f->n_levels * f->feats);
    }
  }
  return NULL;
}

void orc_field_batch(const orc_field* f, int64_t n, const float* x, const float* d,
                     double* sigma, double* rgb, double* feat, double* raw, int32_t n_threads) {
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  pthread_t th[256];
  fjob_t jobs[256];
  int64_t chunk = (n + n_threads - 1) / n_threads;
  for (int i = 0; i < n_threads; ++i) {
    int64_t b = i * chunk, e = (i + 1) * chunk;
    if (b > n) b = n;
    if (e > n) e = n;
    fjob_t J = {f, x, d, sigma, rgb, feat, raw, b, e};
    jobs[i] = J;
    pthread_create(&th[i], NULL, field_worker, &jobs[i]);
  }
  for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
}

/* Occupancy: cell (x fastest) is occupied when sigma >= thresh at any of the
 * centres of its 2x2x2 sub-cells.  margin[cell] = max sigma - thresh. */
typedef struct {
  const orc_field* f;
  int32_t res;
  double thresh;
  uint8_t* bits;
  double* margin;
  int64_t begin, end;
} ojob_t;

static void* occ_worker(void* arg) {
  ojob_t* J = (ojob_t*)arg;
  const orc_field* f = J->f;
  int R = J->res;
  for (int64_t c = J->begin; c < J->end; ++c) {
    int cx = (int)(c % R), cy = (int)((c / R) % R), cz = (int)(c / ((int64_t)R * R));
    double best = -INFINITY;
    for (int s = 0; s < 8; ++s) {
      double xh[3] = {(cx + 0.25 + 0.5 * (s & 1)) / R, (cy + 0.25 + 0.5 * ((s >> 1) & 1)) / R,
                      (cz + 0.25 + 0.5 * ((s >> 2) & 1)) / R};
      double p[3], sigma;
      for (int k = 0; k < 3; ++k) p[k] = f->aabb_min[k] + xh[k] * (f->aabb_max[k] - f->aabb_min[k]);
      orc_field_eval(f, p, p, &sigma, NULL, NULL);
      if (sigma > best) best = sigma;
    }
    J->bits[c] = best >= J->thresh;
    if (J->margin) J->margin[c] = best - J->thresh;
  }
  return NULL;
}

void orc_build_occupancy(const orc_field* f, int32_t res, double thresh, uint8_t* bits,
                         double* margin, int32_t n_threads) {
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  int64_t n = (int64_t)res * res * res;
  pthread_t th[256];
  ojob_t jobs[256];
  int64_t chunk = (n + n_threads - 1) / n_threads;
  for (int i = 0; i < n_threads; ++i) {
    int64_t b = i * chunk, e = (i + 1) * chunk;
    if (b > n) b = n;
    if (e > n) e = n;
    ojob_t J = {f, res, thresh, bits, margin, b, e};
    jobs[i] = J;
    pthread_create(&th[i], NULL, occ_worker, &jobs[i]);
  }
  for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
}

/* ------------------------------------------------------------------------- */
/* Proposal loss and its exact gradient.                                     */
/* Per segment: proposal weights w_j on n_bins uniform intervals of [lo, hi] */
/* versus target histogram h_j; loss = sum_j max(0, h_j - w_j)^2/(h_j+1e-7), */
/* averaged over segments (the proposal loss of Barron et al., Mip-NeRF 360, */
/* CVPR 2022, with bins that coincide with the proposal intervals).          */
/* Backward by the chain rule through w_j = T_j alpha_j,                     */
/* alpha = 1 - exp(-sigma D), sigma = softplus(z + offset), z = W2 relu(W1 f) */
/* and the trilinear hash lookups.                                           */
/* ------------------------------------------------------------------------- */
typedef struct {
  const orc_field* p;
  const float *o, *d, *lohi, *target;
  int32_t n_bins;
  int64_t begin, end;
  double loss;
  double* g_table;
  double* g_mlp;
} pjob_t;

static void prop_segment(pjob_t* J, int64_t s) {
  const orc_field* p = J->p;
  int nb = J->n_bins;
  int nin = p->n_levels * p->feats, H = p->d_hidden;
  int64_t TT = (int64_t)1 << p->log2_table;
  double o[3], d[3];
  for (int k = 0; k < 3; ++k) { o[k] = J->o[3 * s + k]; d[k] = J->d[3 * s + k]; }
  double lo = J->lohi[2 * s], hi = J->lohi[2 * s + 1], D = (hi - lo) / nb;
  double sigma[1024], w[1024], Tr[1024], g[1024], feat[1024][16], hpre[1024][32], z[1024];
  const float* W1 = p->mlp;
  const float* W2 = p->mlp + (int64_t)H * p->d_in;
  double T = 1.0;
  for (int j = 0; j < nb; ++j) {
    double tm = lo + (j + 0.5) * D, x[3], xh[3];
    for (int k = 0; k < 3; ++k) {
      x[k] = o[k] + tm * d[k];
      xh[k] = (x[k] - p->aabb_min[k]) / (p->aabb_max[k] - p->aabb_min[k]);
    }
    orc_hash_encode(p, xh, feat[j]);
    for (int i = nin; i < p->d_in; ++i) feat[j][i] = 0.0;
    matvec(W1, H, p->d_in, feat[j], hpre[j]);
    double zz = 0.0;
    for (int i = 0; i < H; ++i) zz += (double)W2[i] * (hpre[j][i] > 0.0 ? hpre[j][i] : 0.0);
    z[j] = zz;
    sigma[j] = softplus(zz + p->density_offset);
    double alpha = -expm1(-sigma[j] * D);
    Tr[j] = T;
    w[j] = T * alpha;
    T *= 1.0 - alpha;
  }
  double loss = 0.0;
  for (int j = 0; j < nb; ++j) {
    double h = J->target[s * nb + j];
    double r = h - w[j];
    if (r > 0.0) {
      loss += r * r / (h + 1e-7);
      g[j] = -2.0 * r / (h + 1e-7);
    } else {
      g[j] = 0.0;
    }
  }
  J->loss += loss;
  if (!J->g_table && !J->g_mlp) return;
  /* dL/dsigma_k = g_k T_k D exp(-sigma_k D) - D sum_{j>k} g_j w_j */
  double suffix = 0.0;
  for (int k = nb - 1; k >= 0; --k) {
    double dsig = g[k] * Tr[k] * D * exp(-sigma[k] * D) - D * suffix;
    suffix += g[k] * w[k];
    double zz = z[k] + p->density_offset;
    double dz = dsig / (1.0 + exp(-zz));                 /* softplus' = logistic */
    double dh[32];
    for (int i = 0; i < H; ++i) {
      double a = hpre[k][i] > 0.0 ? hpre[k][i] : 0.0;
      if (J->g_mlp) J->g_mlp[(int64_t)H * p->d_in + i] += dz * a;
      dh[i] = hpre[k][i] > 0.0 ? dz * (double)W2[i] : 0.0;
    }
    double df[16] = {0};
    for (int i = 0; i < H; ++i)
      for (int c = 0; c < p->d_in; ++c) {
        if (J->g_mlp) J->g_mlp[(int64_t)i * p->d_in + c] += dh[i] * feat[k][c];
        if (c < nin) df[c] += dh[i] * (double)W1[(int64_t)i * p->d_in + c];
      }
    if (!J->g_table) continue;
    double tm = lo + (k + 0.5) * D, xh[3];
    for (int q = 0; q < 3; ++q) {
      double x = o[q] + tm * d[q];
      xh[q] = fmin(fmax((x - p->aabb_min[q]) / (p->aabb_max[q] - p->aabb_min[q]), 0.0), 1.0);
    }
    for (int l = 0; l < p->n_levels; ++l) {
      int32_t N = p->res[l];
      int64_t v0[3];
      double wt3[3];
      for (int q = 0; q < 3; ++q) {
        double xl = xh[q] * N, fl = floor(xl);
        if (fl > N - 1) fl = N - 1;
        v0[q] = (int64_t)fl;
        wt3[q] = xl - fl;
      }
      for (int corner = 0; corner < 8; ++corner) {
        int64_t v[3];
        double wt = 1.0;
        for (int q = 0; q < 3; ++q) {
          int bit = (corner >> q) & 1;
          v[q] = v0[q] + bit;
          wt *= bit ? wt3[q] : 1.0 - wt3[q];
        }
        uint32_t idx;
        orc_hash_index(N, p->log2_table, v, &idx);
        for (int c = 0; c < p->feats; ++c)
          J->g_table[((int64_t)l * TT + idx) * p->feats + c] += wt * df[l * p->feats + c];
      }
    }
  }
}

static void* prop_worker(void* arg) {
  pjob_t* J = (pjob_t*)arg;
  for (int64_t s = J->begin; s < J->end; ++s) prop_segment(J, s);
  return NULL;
}

double orc_proposal_loss(const orc_field* p, int64_t n_seg, const float* o, const float* d,
                         const float* lohi, const float* target, int32_t n_bins,
                         double* g_table, double* g_mlp, int32_t n_threads) {
  /* gradients of different threads go to private buffers, summed in order */
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 64) n_threads = 64;
  int64_t TT = (int64_t)1 << p->log2_table;
  int64_t nt = (int64_t)p->n_levels * TT * p->feats;
  int64_t nm = (int64_t)p->d_hidden * p->d_in + p->d_hidden;
  pthread_t th[64];
  pjob_t jobs[64];
  int64_t chunk = (n_seg + n_threads - 1) / n_threads;
  for (int i = 0; i < n_threads; ++i) {
    int64_t b = i * chunk, e = (i + 1) * chunk;
    if (b > n_seg) b = n_seg;
    if (e > n_seg) e = n_seg;
    pjob_t J = {p, o, d, lohi, target, n_bins, b, e, 0.0,
                g_table ? (double*)calloc(nt, sizeof(double)) : NULL,
                g_mlp ? (double*)calloc(nm, sizeof(double)) : NULL};
    jobs[i] = J;
    pthread_create(&th[i], NULL, prop_worker, &jobs[i]);
  }
  double loss = 0.0;
  for (int i = 0; i < n_threads; ++i) {
    pthread_join(th[i], NULL);
    loss += jobs[i].loss;
  }
  double inv = n_seg > 0 ? 1.0 / n_seg : 0.0;
  if (g_table) {
    for (int64_t k = 0; k < nt; ++k) {
      double s = 0.0;
      for (int i = 0; i < n_threads; ++i) s += jobs[i].g_table[k];
      g_table[k] = s * inv;
    }
  }
  if (g_mlp) {
    for (int64_t k = 0; k < nm; ++k) {
      double s = 0.0;
      for (int i = 0; i < n_threads; ++i) s += jobs[i].g_mlp[k];
      g_mlp[k] = s * inv;
    }
  }
  for (int i = 0; i < n_threads; ++i) { free(jobs[i].g_table); free(jobs[i].g_mlp); }
  return loss * inv;
}

/* ------------------------------------------------------------------------- */
/* Rounding-error tolerance of the proposal gradient (for tests; it enters   */
/* no value above).  The gradient of orc_proposal_loss, evaluated in a       */
/* binary format of unit roundoff u with the contributions of each element   */
/* summed in any order, is compared with this FP64 result element by element. */
/* Following the probabilistic rounding error analysis of Higham and Mary    */
/* (SIAM J. Sci. Comput. 41, 2019), rounding errors are taken as independent */
/* and of mean zero, so errors of independent terms add in quadrature:        */
/*   tol_e = u min(n_e, lambda sqrt(n_e)) S_e                                */
/*         + u min(sum_s b_s, lambda sqrt(sum_s b_s^2)) + Z_e,  b = K m + p,  */
/* where each min takes the smaller of a worst-case bound and a bound that   */
/* fails with probability at most about 2 n_e exp(-lambda^2 / 2).  Per      */
/* element e, over its n_e contributions c_s:                                */
/*   S_e  sum |c_s|: the final sum (Higham and Mary's bound for summation);  */
/*   m_s  a running error bound of one contribution: every node of the chain  */
/*        carries sum |partial| x m(operand) plus |node| (its own rounding),  */
/*        so differences add up; K bounds the roundings folded into one node */
/*        (dot products, the 64-lane scans, a few ulps of exp and log);     */
/*   p_s  the same chain seeded only with the error of the trilinear weights: */
/*        the lattice coordinate x N of the rounded sample position o + t d   */
/*        carries N times its error, and each corner weight changes by the    */
/*        coordinate errors times the other two weight factors;              */
/*   Z_e  for each ReLU whose sign lies within its own bound, the whole      */
/*        contribution that hinges on that sign.                             */
/* Scaled by 1 / n_seg like the gradient.                                    */
/* ------------------------------------------------------------------------- */

/* lattice-coordinate error (units of u) of one sample and level, per axis,  */
/* for a position computed as o + (lo + (j + 1/2) D) d and moved to the box */
static void prop_lattice(const orc_field* p, const double o[3], const double d[3], double lo, double D, int j,
                         int32_t R, int64_t v0[3], double fr[3], double dxl[3]) {
  double tm = lo + (j + 0.5) * D;
  double dtm = 3.0 * (j + 0.5) * D + fabs(tm);
  for (int k = 0; k < 3; ++k) {
    double ext = p->aabb_max[k] - p->aabb_min[k], x = o[k] + tm * d[k];
    double xh = fmin(fmax((x - p->aabb_min[k]) / ext, 0.0), 1.0);
    double dx = fabs(d[k]) * dtm + fabs(tm * d[k]) + fabs(x);
    double xl = xh * R, fl = floor(xl);
    if (fl > R - 1) fl = R - 1;
    v0[k] = (int64_t)fl;
    fr[k] = xl - fl;
    dxl[k] = R * (dx + 2.0 * fabs(x - p->aabb_min[k])) / ext + xl;
  }
}

/* corner weight, its rounding magnitude and its position-error magnitude */
static double prop_corner(int corner, const double fr[3], const double dxl[3], double* mw, double* pw) {
  double f3[3], ww = 1.0, pp = 0.0;
  for (int k = 0; k < 3; ++k) {
    f3[k] = ((corner >> k) & 1) ? fr[k] : 1.0 - fr[k];
    ww *= f3[k];
  }
  for (int k = 0; k < 3; ++k) pp += dxl[k] * f3[(k + 1) % 3] * f3[(k + 2) % 3];
  *mw = 4.0 * ww;   /* 1 - fr, two products, own rounding */
  *pw = pp;
  return ww;
}

void orc_proposal_grad_bound(const orc_field* p, int64_t n_seg, const float* o_in, const float* d_in,
                             const float* lohi, const float* target, int32_t nb, double u, double K,
                             double lambda, double* b_table, double* b_mlp) {
  int nin = p->n_levels * p->feats, H = p->d_hidden, DI = p->d_in;
  int64_t TT = (int64_t)1 << p->log2_table;
  int64_t nt = (int64_t)p->n_levels * TT * p->feats, ne = nt + (int64_t)H * DI + H;
  /* per element: S, sum b, sum b^2, Z, n */
  double* S = (double*)calloc(ne, sizeof(double));
  double* B = (double*)calloc(ne, sizeof(double));
  double* Q = (double*)calloc(ne, sizeof(double));
  double* Z = (double*)calloc(ne, sizeof(double));
  double* N = (double*)calloc(ne, sizeof(double));
  /* per bin: features and hidden units with their two magnitudes */
  double (*f)[16] = calloc(nb, sizeof *f), (*mf)[16] = calloc(nb, sizeof *mf), (*pf)[16] = calloc(nb, sizeof *pf);
  double (*h)[32] = calloc(nb, sizeof *h), (*mh)[32] = calloc(nb, sizeof *mh), (*ph)[32] = calloc(nb, sizeof *ph);
  /* per bin scalars: value, rounding magnitude, position magnitude */
  double* sc = (double*)calloc((size_t)15 * (nb + 1), sizeof(double));
  double *z = sc, *mz = z + nb + 1, *pz = mz + nb + 1, *w = pz + nb + 1, *mw = w + nb + 1, *pw = mw + nb + 1;
  double *g = pw + nb + 1, *mg = g + nb + 1, *pg = mg + nb + 1, *T = pg + nb + 1, *mT = T + nb + 1;
  double *pT = mT + nb + 1, *E = pT + nb + 1, *mE = E + nb + 1, *pE = mE + nb + 1;
  const float* W1 = p->mlp;
  const float* W2 = p->mlp + (int64_t)H * DI;
#define ADD(e, c, m, pp)                \
  do {                                  \
    double b_ = K * (m) + (pp);         \
    S[e] += fabs(c);                    \
    B[e] += b_;                         \
    Q[e] += b_ * b_;                    \
    N[e] += 1.0;                        \
  } while (0)
  for (int64_t s = 0; s < n_seg; ++s) {
    double o[3], d[3];
    for (int k = 0; k < 3; ++k) { o[k] = o_in[3 * s + k]; d[k] = d_in[3 * s + k]; }
    double lo = lohi[2 * s], hi = lohi[2 * s + 1];
    if (!(hi > lo)) continue;
    double D = (hi - lo) / nb;
    T[0] = 1.0;
    mT[0] = pT[0] = 0.0;
    for (int j = 0; j < nb; ++j) {
      for (int c = 0; c < 16; ++c) f[j][c] = mf[j][c] = pf[j][c] = 0.0;
      for (int l = 0; l < p->n_levels; ++l) {
        int64_t v0[3];
        double fr[3], dxl[3];
        prop_lattice(p, o, d, lo, D, j, p->res[l], v0, fr, dxl);
        for (int corner = 0; corner < 8; ++corner) {
          int64_t v[3];
          for (int k = 0; k < 3; ++k) v[k] = v0[k] + ((corner >> k) & 1);
          double mwt, pwt, ww = prop_corner(corner, fr, dxl, &mwt, &pwt);
          uint32_t idx;
          orc_hash_index(p->res[l], p->log2_table, v, &idx);
          const float* e = p->table + ((int64_t)l * TT + idx) * p->feats;
          for (int c = 0; c < p->feats; ++c) {
            double ae = fabs((double)e[c]);
            f[j][l * p->feats + c] += ww * e[c];
            mf[j][l * p->feats + c] += mwt * ae + 2.0 * ww * ae;
            pf[j][l * p->feats + c] += pwt * ae;
          }
        }
      }
      double zz = 0.0, mzz = 0.0, pzz = 0.0;
      for (int i = 0; i < H; ++i) {
        double hv = 0.0, m = 0.0, pp = 0.0;
        for (int c = 0; c < nin; ++c) {
          double a = W1[(int64_t)i * DI + c];
          hv += a * f[j][c];
          m += fabs(a) * mf[j][c] + fabs(a * f[j][c]);
          pp += fabs(a) * pf[j][c];
        }
        h[j][i] = hv;
        mh[j][i] = m;
        ph[j][i] = pp;
        if (hv > 0.0) {
          zz += W2[i] * hv;
          mzz += fabs(W2[i]) * m + fabs(W2[i] * hv);
          pzz += fabs(W2[i]) * pp;
        }
      }
      z[j] = zz;
      mz[j] = mzz;
      pz[j] = pzz;
      double zo = zz + p->density_offset, L = 1.0 / (1.0 + exp(-zo));
      double sg = softplus(zo), msg = L * (mzz + fabs(zo)) + 4.0 * sg, psg = L * pzz;
      double y = sg * D, al = -expm1(-y), Ej = exp(-y);
      double mal = Ej * (D * msg + 2.0 * y) + 2.0 * al, pal = Ej * D * psg;
      E[j] = Ej;
      mE[j] = Ej * (D * msg + 2.0 * y + 2.0);
      pE[j] = pal;
      double om = 1.0 - al, mom = mal + om;
      w[j] = T[j] * al;
      mw[j] = mT[j] * al + T[j] * mal + w[j];
      pw[j] = pT[j] * al + T[j] * pal;
      T[j + 1] = T[j] * om;
      mT[j + 1] = mT[j] * om + T[j] * mom + T[j + 1];
      pT[j + 1] = pT[j] * om + T[j] * pal;
      double ht = target[s * nb + j], hd = ht + 1e-7, r = ht - w[j], mr = mw[j] + fabs(r), pr = pw[j];
      g[j] = r > 0.0 ? -2.0 * r / hd : 0.0;
      if (r > 0.0 || fabs(r) <= u * (K * mr + pr)) {   /* the sign of r may be rounded either way */
        mg[j] = 2.0 * mr / hd + 2.0 * fabs(g[j]);
        pg[j] = 2.0 * pr / hd;
      } else {
        mg[j] = pg[j] = 0.0;
      }
    }
    /* the suffix sums come from a scan over all bins: their rounding scales
       with the sum over all of them */
    double sall = 0.0;
    for (int j = 0; j < nb; ++j) sall += fabs(g[j] * w[j]);
    double suf = 0.0, msuf = 0.0, psuf = 0.0;
    for (int k = nb - 1; k >= 0; --k) {
      double a1 = g[k] * T[k] * D * E[k];
      double ma1 = (mg[k] * T[k] + fabs(g[k]) * mT[k]) * D * E[k] + fabs(g[k]) * T[k] * D * mE[k] + 4.0 * fabs(a1);
      double pa1 = (pg[k] * T[k] + fabs(g[k]) * pT[k]) * D * E[k] + fabs(g[k]) * T[k] * D * pE[k];
      double a2 = D * suf, ma2 = D * (msuf + sall) + 3.0 * fabs(a2), pa2 = D * psuf;
      double dsig = a1 - a2, mds = ma1 + ma2 + fabs(dsig), pds = pa1 + pa2;
      suf += g[k] * w[k];
      msuf += mg[k] * w[k] + fabs(g[k]) * mw[k] + fabs(g[k] * w[k]);
      psuf += pg[k] * w[k] + fabs(g[k]) * pw[k];
      double zo = z[k] + p->density_offset, L = 1.0 / (1.0 + exp(-zo)), dL = L * (1.0 - L);
      double dz = dsig * L;
      double mdz = mds * L + fabs(dsig) * dL * (mz[k] + fabs(zo)) + 4.0 * fabs(dz);
      double pdz = pds * L + fabs(dsig) * dL * pz[k];
      double dh[32], mdh[32], pdh[32];
      int tie[32];
      for (int i = 0; i < H; ++i) {
        int on = h[k][i] > 0.0;
        tie[i] = fabs(h[k][i]) <= u * (K * mh[k][i] + ph[k][i]);
        dh[i] = on ? dz * W2[i] : 0.0;
        mdh[i] = on ? mdz * fabs(W2[i]) + fabs(dh[i]) : 0.0;
        pdh[i] = on ? pdz * fabs(W2[i]) : 0.0;
      }
      double df[16] = {0}, mdf[16] = {0}, pdf[16] = {0}, zdf[16] = {0};
      for (int i = 0; i < H; ++i)
        for (int c = 0; c < nin; ++c) {
          double a = W1[(int64_t)i * DI + c];
          df[c] += dh[i] * a;
          mdf[c] += mdh[i] * fabs(a) + fabs(dh[i] * a);
          pdf[c] += pdh[i] * fabs(a);
          if (tie[i]) zdf[c] += fabs(dz * W2[i] * a);
        }
      /* MLP elements: dz [h > 0] W2 f for W1, dz relu(h) for W2; the sums
         over |W1 f| (inside mh) also cover the form sum_c W1 (dz f) */
      for (int i = 0; i < H; ++i) {
        int on = h[k][i] > 0.0;
        for (int c = 0; c < nin; ++c) {
          int64_t e = nt + (int64_t)i * DI + c;
          if (on) ADD(e, dh[i] * f[k][c], mdh[i] * fabs(f[k][c]) + fabs(dh[i]) * mf[k][c] + fabs(dh[i] * f[k][c]),
                      pdh[i] * fabs(f[k][c]) + fabs(dh[i]) * pf[k][c]);
          if (tie[i]) Z[e] += fabs(dz * W2[i] * f[k][c]);
        }
        int64_t e2 = nt + (int64_t)H * DI + i;
        if (on) ADD(e2, dz * h[k][i], mdz * mh[k][i] + 2.0 * fabs(dz) * mh[k][i], pdz * mh[k][i] + fabs(dz) * ph[k][i]);
        if (tie[i]) Z[e2] += fabs(dz) * u * (K * mh[k][i] + ph[k][i]);
      }
      /* table elements: corner weight x df */
      for (int l = 0; l < p->n_levels; ++l) {
        int64_t v0[3];
        double fr[3], dxl[3];
        prop_lattice(p, o, d, lo, D, k, p->res[l], v0, fr, dxl);
        for (int corner = 0; corner < 8; ++corner) {
          int64_t v[3];
          for (int q = 0; q < 3; ++q) v[q] = v0[q] + ((corner >> q) & 1);
          double mwt, pwt, ww = prop_corner(corner, fr, dxl, &mwt, &pwt);
          uint32_t idx;
          orc_hash_index(p->res[l], p->log2_table, v, &idx);
          for (int c = 0; c < p->feats; ++c) {
            int64_t e = ((int64_t)l * TT + idx) * p->feats + c;
            int cc = l * p->feats + c;
            ADD(e, ww * df[cc], mwt * fabs(df[cc]) + ww * mdf[cc] + fabs(ww * df[cc]), pwt * fabs(df[cc]) + ww * pdf[cc]);
            Z[e] += ww * zdf[cc];
          }
        }
        /* a lattice coordinate within its error of a cell face: the sample
           may land in the neighbouring cell, whose far corners then take a
           weight of at most that error */
        for (int q = 0; q < 3; ++q) {
          double ed = u * dxl[q];
          int64_t far = -1;
          if (fr[q] <= ed && v0[q] > 0) far = v0[q] - 1;
          if (1.0 - fr[q] <= ed && v0[q] + 2 <= p->res[l]) far = v0[q] + 2;
          if (far < 0) continue;
          for (int corner = 0; corner < 4; ++corner) {
            int64_t v[3];
            int b = 0;
            for (int a = 0; a < 3; ++a) v[a] = a == q ? far : v0[a] + ((corner >> b++) & 1);
            uint32_t idx;
            orc_hash_index(p->res[l], p->log2_table, v, &idx);
            for (int c = 0; c < p->feats; ++c)
              Z[((int64_t)l * TT + idx) * p->feats + c] += ed * (fabs(df[l * p->feats + c]) + zdf[l * p->feats + c]);
          }
        }
      }
    }
  }
#undef ADD
  double inv = n_seg > 0 ? 1.0 / n_seg : 0.0;
  for (int64_t e = 0; e < ne; ++e) {
    double b = u * fmin(N[e], lambda * sqrt(N[e])) * S[e] + u * fmin(B[e], lambda * sqrt(Q[e])) + Z[e];
    b *= inv;
    if (e < nt) b_table[e] = b; else b_mlp[e - nt] = b;
  }
  free(S); free(B); free(Q); free(Z); free(N);
  free(f); free(mf); free(pf); free(h); free(mh); free(ph); free(sc);
}

/* ------------------------------------------------------------------------- */
/* Proposal training targets: the plain marcher's weights w_i = T_i alpha_i  */
/* on the uniform grid of the first (camera) segment, without surfaces, split */
/* over n_bins equal bins of the clipped range [lo, hi] in proportion to the */
/* overlap of each interval with each bin.  lohi = (0, 0) and zero targets   */
/* for rays that miss the field box.                                         */
/* ------------------------------------------------------------------------- */
void orc_proposal_targets(const orc_field* f, int64_t n, const float* origins, const float* dirs,
                          double t_near, double t_far, int32_t n_samples, int32_t n_bins,
                          double* lohi, double* target) {
  double span = t_far - t_near, delta = span / n_samples;
  for (int64_t r = 0; r < n; ++r) {
    double o[3], d[3], b0, b1;
    for (int k = 0; k < 3; ++k) { o[k] = origins[3 * r + k]; d[k] = dirs[3 * r + k]; }
    for (int j = 0; j < n_bins; ++j) target[r * n_bins + j] = 0.0;
    lohi[2 * r] = lohi[2 * r + 1] = 0.0;
    if (!slab(f, o, d, &b0, &b1)) continue;
    double lo = fmax(t_near, b0), hi = fmin(t_far, b1);
    if (!(hi > lo)) continue;
    lohi[2 * r] = lo;
    lohi[2 * r + 1] = hi;
    double bw = (hi - lo) / n_bins, T = 1.0;
    for (int k = 0; k < n_samples; ++k) {
      double a = fmax(t_near + k * delta, lo), b = fmin(t_near + (k + 1) * delta, hi);
      if (!(b > a)) continue;
      double tm = 0.5 * (a + b), x[3], sigma;
      for (int q = 0; q < 3; ++q) x[q] = o[q] + tm * d[q];
      orc_field_eval(f, x, d, &sigma, NULL, NULL);
      double alpha = -expm1(-sigma * (b - a));
      double w = T * alpha;
      T *= 1.0 - alpha;
      for (int j = 0; j < n_bins; ++j) {
        double c0 = lo + j * bw, c1 = lo + (j + 1) * bw;
        double ov = fmin(b, c1) - fmax(a, c0);
        if (ov > 0.0) target[r * n_bins + j] += w * ov / (b - a);
      }
    }
  }
}
