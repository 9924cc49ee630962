/*
 * perch_oracle.c -- scalar CPU oracle for PERCH successor evaluation.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code,
 * header, table or constant generator with the GPU library.
 *
 * What it follows (arXiv:1510.05613):
 *   Sec. III-A  notation: object state O = (ID, x, y, theta); observed cloud I;
 *               rendered cloud R_j; dR_j = R_j - R_{j-1}; volume V(O).
 *   Sec. III-B  explanation cost J = J_o + J_r and the indicator Eq.(1):
 *               a point is unexplained by C iff min_{p' in C} |p' - p| > delta.
 *   Sec. IV-A   the incremental render with R_{i-1} subset of R_i, the per-object
 *               decomposition Eq.(2) with dJ_r^i, dJ_o^i and residual(i), the
 *               successor set Eq.(3) and edge cost Eq.(4).
 *   Sec. IV-B   exhaustive tree search (Theorems 1-2 with w = 1), used here as
 *               exhaustive enumeration and uniform-cost search.
 *   Sec. IV-E    local ICP alignment of each new object's non-occluded part
 *               (compensating for a coarse pose discretization).
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - a rendered point cloud holds one point per covered pixel centre, at the
 *     camera-Z depth of the frontmost front-facing triangle, back-projected
 *     through that pixel centre;
 *   - rasterisation: float32 vertex stage with a fixed operation order, vertices
 *     snapped to 1/256 pixel, integer edge functions, top-left fill rule,
 *     front faces only (closed outward-CCW meshes);
 *   - "does not occlude" is strict: any pixel with D_new < D_parent < inf makes
 *     the successor invalid, equal depths keep the parent pixel;
 *   - explained iff distance <= delta (closed ball); min over an empty set is +inf;
 *   - V(O) is the convex solid {n.p <= d} of the mesh's planes.
 *
 * Floating point is FP64 except the vertex stage (IEEE float32, no contraction;
 * build with -ffp-contract=off).
 */
#include "perch_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define FLAG_EPS 1e-6 /* near-tie band (metres) for the flags */
/* ICP association near-ties, in metres (radius tests) and pixels (rounding of a
 * projection to the nearest pixel): the association is FP64 on both sides, which
 * differ only by FP64 rounding, far inside these bands */
#define ICP_FLAG_EPS 1e-9
#define ICP_FLAG_PX 1e-9
#define ORC_MAX_K 16   /* most objects in a scene */

struct orc_scene {
  orc_sensor s;
  int W, H;
  double fx, fy, cx, cy, delta, delta2;
  double Rinv[9], t[3]; /* p_world = Rinv (p_cam - t), exact FP64 inverse of the f32 R */
  int nI;               /* observed points */
  int32_t* I_pix;       /* pixel index v*W+u of each observed point */
  double* I_cam;        /* camera frame, 3 per point */
  double* I_w;          /* world frame, 3 per point */
  int32_t* pix2pt;      /* H*W -> point index or -1 */
  int n_mesh;
  int32_t *v_off, *t_off, *f_off;
  float* verts;
  int32_t* tris;
  float* planes;
  int max_v;
  int P;
  float* poses;
  int K;
  int32_t* obj_mesh;
  int radius_mode;
  int nthreads;
  uint8_t* sym; /* per mesh: rotationally symmetric, searched over (x, y) only */
};

/* ------------------------------------------------------------------------- */
/* small helpers                                                             */
/* ------------------------------------------------------------------------- */

static int64_t floor_div256(int64_t a) { return a >= 0 ? a / 256 : -((-a + 255) / 256); }
static int64_t ceil_div256(int64_t a) { return -floor_div256(-a); }

static int inv3(const double* m, double* r) {
  double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5], g = m[6], h = m[7],
         i = m[8];
  double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
  double det = a * A + b * B + c * C;
  if (det == 0.0) return -1;
  r[0] = A / det;
  r[1] = -(b * i - c * h) / det;
  r[2] = (b * f - c * e) / det;
  r[3] = B / det;
  r[4] = (a * i - c * g) / det;
  r[5] = -(a * f - c * d) / det;
  r[6] = C / det;
  r[7] = -(a * h - b * g) / det;
  r[8] = (a * e - b * d) / det;
  return 0;
}

/* back-projection of pixel (u, v) at depth z through its centre (FP64) */
static void backproject(const orc_scene* sc, int u, int v, double z, double* q) {
  q[0] = ((double)u - sc->cx) * z / sc->fx;
  q[1] = ((double)v - sc->cy) * z / sc->fy;
  q[2] = z;
}

/* ------------------------------------------------------------------------- */
/* vertex stage: float32 spec (model -> world -> camera -> snapped screen)   */
/* ------------------------------------------------------------------------- */

/* World placement of model point m by pose (x, y, c, s):
 *   w = (c m_x - s m_y + x, s m_x + c m_y + y, m_z).
 * Camera: cam_k = ((M_k0 w_x + M_k1 w_y) + M_k2 w_z) + M_k3.
 * Projection: inv = 1 / cam_z, u = fx (cam_x inv) + cx, v = fy (cam_y inv) + cy.
 * Snap: U = rint(256 u), V = rint(256 v) (round half to even). */
static int vertex_stage_f32(const orc_scene* sc, int mesh, int pose, float* cam,
                            int64_t* U, int64_t* V) {
  const float* pz = sc->poses + 4 * (size_t)pose;
  const float x = pz[0], y = pz[1], c = pz[2], s = pz[3];
  const float* M = sc->s.cam_from_world;
  const float fx = sc->s.fx, fy = sc->s.fy, cx = sc->s.cx, cy = sc->s.cy;
  int bad = 0;
  for (int k = sc->v_off[mesh]; k < sc->v_off[mesh + 1]; ++k) {
    const float* m = sc->verts + 3 * (size_t)k;
    float wx = (c * m[0] - s * m[1]) + x;
    float wy = (s * m[0] + c * m[1]) + y;
    float wz = m[2];
    float* o = cam + 3 * (size_t)(k - sc->v_off[mesh]);
    for (int r = 0; r < 3; ++r)
      o[r] = ((M[4 * r] * wx + M[4 * r + 1] * wy) + M[4 * r + 2] * wz) + M[4 * r + 3];
    float inv = 1.0f / o[2];
    float u = fx * (o[0] * inv) + cx;
    float v = fy * (o[1] * inv) + cy;
    float su = rintf(256.0f * u), sv = rintf(256.0f * v);
    if (!(o[2] > 0.01f) || !(fabsf(su) <= 16777216.0f) || !(fabsf(sv) <= 16777216.0f)) bad = 1;
    U[k - sc->v_off[mesh]] = (int64_t)su;
    V[k - sc->v_off[mesh]] = (int64_t)sv;
  }
  return bad ? -2 : 0;
}

/* ------------------------------------------------------------------------- */
/* rasteriser: integer coverage, top-left rule, FP64 plane depth             */
/* ------------------------------------------------------------------------- */

/* Edge a->b of a positively oriented triangle covers p iff its edge function is
 * positive, or zero on a top or left edge.  With y pointing down the inward
 * normal is (-dy, dx): a left edge has dy < 0, a top edge has dy == 0, dx > 0. */
static int edge_covers(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t px, int64_t py) {
  int64_t dx = bx - ax, dy = by - ay;
  int64_t e = dx * (py - ay) - dy * (px - ax);
  if (e > 0) return 1;
  if (e < 0) return 0;
  return (dy < 0) || (dy == 0 && dx > 0);
}

/* Renders one object, taking D[u] = min(D[u], z).  cam/U/V are scratch (>= V). */
static int render_into(const orc_scene* sc, int mesh, int pose, int cull, double* D,
                       float* cam, int64_t* U, int64_t* V) {
  int rc = vertex_stage_f32(sc, mesh, pose, cam, U, V);
  if (rc) return rc;
  const int W = sc->W, H = sc->H;
  for (int t = sc->t_off[mesh]; t < sc->t_off[mesh + 1]; ++t) {
    const int32_t* tri = sc->tris + 3 * (size_t)t;
    int i0 = tri[0], i1 = tri[1], i2 = tri[2];
    int64_t x0 = U[i0], y0 = V[i0], x1 = U[i1], y1 = V[i1], x2 = U[i2], y2 = V[i2];
    int64_t area = (x1 - x0) * (y2 - y0) - (y1 - y0) * (x2 - x0);
    if (area == 0) continue;
    /* outward-CCW faces seen from the front project with negative area here */
    if (cull && area > 0) continue;
    if (area < 0) { /* orient positively */
      int64_t tx = x1, ty = y1;
      x1 = x2; y1 = y2; x2 = tx; y2 = ty;
    }
    int64_t xmin = x0 < x1 ? (x0 < x2 ? x0 : x2) : (x1 < x2 ? x1 : x2);
    int64_t xmax = x0 > x1 ? (x0 > x2 ? x0 : x2) : (x1 > x2 ? x1 : x2);
    int64_t ymin = y0 < y1 ? (y0 < y2 ? y0 : y2) : (y1 < y2 ? y1 : y2);
    int64_t ymax = y0 > y1 ? (y0 > y2 ? y0 : y2) : (y1 > y2 ? y1 : y2);
    int64_t ia = ceil_div256(xmin), ib = floor_div256(xmax);
    int64_t ja = ceil_div256(ymin), jb = floor_div256(ymax);
    if (ia < 0) ia = 0;
    if (ja < 0) ja = 0;
    if (ib > W - 1) ib = W - 1;
    if (jb > H - 1) jb = H - 1;
    if (ia > ib || ja > jb) continue;
    /* plane of the triangle from its float32 camera-space vertices, in FP64 */
    const float* A = cam + 3 * (size_t)i0;
    const float* B = cam + 3 * (size_t)i1;
    const float* C = cam + 3 * (size_t)i2;
    double e1[3] = {(double)B[0] - A[0], (double)B[1] - A[1], (double)B[2] - A[2]};
    double e2[3] = {(double)C[0] - A[0], (double)C[1] - A[1], (double)C[2] - A[2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                   e1[0] * e2[1] - e1[1] * e2[0]};
    double na = n[0] * A[0] + n[1] * A[1] + n[2] * A[2];
    for (int64_t j = ja; j <= jb; ++j) {
      for (int64_t i = ia; i <= ib; ++i) {
        int64_t px = 256 * i, py = 256 * j;
        if (!edge_covers(x0, y0, x1, y1, px, py)) continue;
        if (!edge_covers(x1, y1, x2, y2, px, py)) continue;
        if (!edge_covers(x2, y2, x0, y0, px, py)) continue;
        double r0 = ((double)i - sc->cx) / sc->fx, r1 = ((double)j - sc->cy) / sc->fy;
        double z = na / (n[0] * r0 + n[1] * r1 + n[2]);
        double* d = D + j * W + i;
        if (z < *d) *d = z;
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* volumes and radius queries                                                */
/* ------------------------------------------------------------------------- */

/* max_f (n_f . p_obj - d_f) for world point pw and object (mesh, pose); the
 * point is in V(O) iff the result is <= 0.  p_obj inverts the pose exactly. */
static double vol_margin(const orc_scene* sc, int mesh, int pose, const double* pw) {
  const float* pz = sc->poses + 4 * (size_t)pose;
  double c = pz[2], s = pz[3], n2 = c * c + s * s;
  double dx = pw[0] - (double)pz[0], dy = pw[1] - (double)pz[1];
  double ox = (c * dx + s * dy) / n2, oy = (-s * dx + c * dy) / n2, oz = pw[2];
  double best = -INFINITY;
  for (int f = sc->f_off[mesh]; f < sc->f_off[mesh + 1]; ++f) {
    const float* pl = sc->planes + 4 * (size_t)f;
    double m = (double)pl[0] * ox + (double)pl[1] * oy + (double)pl[2] * oz - (double)pl[3];
    if (m > best) best = m;
  }
  return best;
}

static double d2(const double* a, const double* b) {
  double x = a[0] - b[0], y = a[1] - b[1], z = a[2] - b[2];
  return x * x + y * y + z * z;
}

/* Pixel window that provably holds every point within delta of a point p seen
 * at (X, Y, Z): a point q with |q - p| <= r satisfies
 *   |u_q - u_p| <= fx r sqrt(1 + (X/Z)^2) / (Z - r)   (and likewise for v),
 * by Cauchy-Schwarz on (dX - (X/Z) dZ) and Z_q >= Z - r.  r = delta + 2e-6 so the
 * flag band is covered; +1 pixel absorbs rounding in the bound itself. */
static void window_radius(const orc_scene* sc, const double* p, int* ru, int* rv) {
  double r = sc->delta + 2e-6;
  double den = p[2] - r;
  if (den <= 0) { *ru = sc->W; *rv = sc->H; return; }
  double a = p[0] / p[2], b = p[1] / p[2];
  double bu = sc->fx * r * sqrt(1.0 + a * a) / den;
  double bv = sc->fy * r * sqrt(1.0 + b * b) / den;
  *ru = bu > sc->W ? sc->W : (int)floor(bu) + 1;
  *rv = bv > sc->H ? sc->H : (int)floor(bv) + 1;
}

/* min squared distance from q (camera frame, seen at pixel (uq, vq)) to I */
static double min_d2_to_I(const orc_scene* sc, const double* q, int uq, int vq) {
  double best = INFINITY;
  if (sc->radius_mode == 1) {
    for (int k = 0; k < sc->nI; ++k) {
      double e = d2(q, sc->I_cam + 3 * (size_t)k);
      if (e < best) best = e;
    }
    return best;
  }
  int ru, rv;
  window_radius(sc, q, &ru, &rv);
  int va = vq - rv < 0 ? 0 : vq - rv, vb = vq + rv > sc->H - 1 ? sc->H - 1 : vq + rv;
  int ua = uq - ru < 0 ? 0 : uq - ru, ub = uq + ru > sc->W - 1 ? sc->W - 1 : uq + ru;
  for (int v = va; v <= vb; ++v)
    for (int u = ua; u <= ub; ++u) {
      int k = sc->pix2pt[v * sc->W + u];
      if (k < 0) continue;
      double e = d2(q, sc->I_cam + 3 * (size_t)k);
      if (e < best) best = e;
    }
  return best;
}

/* min squared distance from p (camera frame, pixel (up, vp)) to the rendered
 * points of depth map Dsel (+inf = no point) */
static double min_d2_to_depth(const orc_scene* sc, const double* p, int up, int vp,
                              const double* Dsel) {
  double best = INFINITY, q[3];
  int ua, ub, va, vb;
  if (sc->radius_mode == 1) {
    ua = 0; ub = sc->W - 1; va = 0; vb = sc->H - 1;
  } else {
    int ru, rv;
    window_radius(sc, p, &ru, &rv);
    va = vp - rv < 0 ? 0 : vp - rv; vb = vp + rv > sc->H - 1 ? sc->H - 1 : vp + rv;
    ua = up - ru < 0 ? 0 : up - ru; ub = up + ru > sc->W - 1 ? sc->W - 1 : up + ru;
  }
  for (int v = va; v <= vb; ++v)
    for (int u = ua; u <= ub; ++u) {
      double z = Dsel[v * sc->W + u];
      if (!(z < INFINITY)) continue;
      backproject(sc, u, v, z, q);
      double e = d2(p, q);
      if (e < best) best = e;
    }
  return best;
}

static int near_delta(const orc_scene* sc, double m2) {
  return fabs(sqrt(m2) - sc->delta) <= FLAG_EPS;
}

/* ------------------------------------------------------------------------- */
/* scene                                                                     */
/* ------------------------------------------------------------------------- */

orc_scene* orc_create(const orc_sensor* sensor, const float* depth_obs, int32_t n_mesh,
                      const int32_t* v_off, const int32_t* t_off, const int32_t* f_off,
                      const float* verts, const int32_t* tris, const float* planes,
                      int32_t n_poses, const float* poses, int32_t K,
                      const int32_t* obj_mesh) {
  if (!sensor || sensor->width <= 0 || sensor->height <= 0 || n_mesh <= 0 || n_poses <= 0 ||
      K < 0 || K > ORC_MAX_K)
    return NULL;
  orc_scene* sc = (orc_scene*)calloc(1, sizeof(orc_scene));
  sc->s = *sensor;
  sc->W = sensor->width;
  sc->H = sensor->height;
  sc->fx = sensor->fx; sc->fy = sensor->fy; sc->cx = sensor->cx; sc->cy = sensor->cy;
  sc->delta = sensor->delta;
  sc->delta2 = sc->delta * sc->delta;
  double R[9];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) R[3 * r + c] = sensor->cam_from_world[4 * r + c];
    sc->t[r] = sensor->cam_from_world[4 * r + 3];
  }
  if (inv3(R, sc->Rinv)) { free(sc); return NULL; }
  sc->n_mesh = n_mesh;
  sc->v_off = (int32_t*)malloc(sizeof(int32_t) * (n_mesh + 1));
  sc->t_off = (int32_t*)malloc(sizeof(int32_t) * (n_mesh + 1));
  sc->f_off = (int32_t*)malloc(sizeof(int32_t) * (n_mesh + 1));
  memcpy(sc->v_off, v_off, sizeof(int32_t) * (n_mesh + 1));
  memcpy(sc->t_off, t_off, sizeof(int32_t) * (n_mesh + 1));
  memcpy(sc->f_off, f_off, sizeof(int32_t) * (n_mesh + 1));
  int nv = v_off[n_mesh], nt = t_off[n_mesh], nf = f_off[n_mesh];
  sc->verts = (float*)malloc(sizeof(float) * 3 * (size_t)(nv > 0 ? nv : 1));
  sc->tris = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)(nt > 0 ? nt : 1));
  sc->planes = (float*)malloc(sizeof(float) * 4 * (size_t)(nf > 0 ? nf : 1));
  memcpy(sc->verts, verts, sizeof(float) * 3 * (size_t)nv);
  memcpy(sc->tris, tris, sizeof(int32_t) * 3 * (size_t)nt);
  memcpy(sc->planes, planes, sizeof(float) * 4 * (size_t)nf);
  sc->max_v = 0;
  for (int m = 0; m < n_mesh; ++m) {
    int v = v_off[m + 1] - v_off[m];
    if (v > sc->max_v) sc->max_v = v;
    for (int t = t_off[m]; t < t_off[m + 1]; ++t)
      for (int k = 0; k < 3; ++k)
        if (tris[3 * t + k] < 0 || tris[3 * t + k] >= v) { orc_destroy(sc); return NULL; }
  }
  sc->P = n_poses;
  sc->poses = (float*)malloc(sizeof(float) * 4 * (size_t)n_poses);
  memcpy(sc->poses, poses, sizeof(float) * 4 * (size_t)n_poses);
  sc->K = K;
  sc->obj_mesh = (int32_t*)malloc(sizeof(int32_t) * (K > 0 ? K : 1));
  if (K) memcpy(sc->obj_mesh, obj_mesh, sizeof(int32_t) * K);
  sc->radius_mode = 0;
  sc->nthreads = 1;
  sc->sym = (uint8_t*)calloc((size_t)n_mesh + 1, 1);

  /* observed cloud I: one point per pixel with a return (Sec. III-A) */
  size_t npx = (size_t)sc->W * sc->H;
  sc->pix2pt = (int32_t*)malloc(sizeof(int32_t) * npx);
  int n = 0;
  for (size_t k = 0; k < npx; ++k) {
    sc->pix2pt[k] = -1;
    if (depth_obs && depth_obs[k] > 0.0f) ++n;
  }
  sc->nI = n;
  sc->I_pix = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  sc->I_cam = (double*)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
  sc->I_w = (double*)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
  n = 0;
  for (int v = 0; v < sc->H && depth_obs; ++v)
    for (int u = 0; u < sc->W; ++u) {
      size_t k = (size_t)v * sc->W + u;
      if (!(depth_obs[k] > 0.0f)) continue;
      double* pc = sc->I_cam + 3 * (size_t)n;
      double* pw = sc->I_w + 3 * (size_t)n;
      backproject(sc, u, v, (double)depth_obs[k], pc);
      double d[3] = {pc[0] - sc->t[0], pc[1] - sc->t[1], pc[2] - sc->t[2]};
      for (int r = 0; r < 3; ++r)
        pw[r] = sc->Rinv[3 * r] * d[0] + sc->Rinv[3 * r + 1] * d[1] + sc->Rinv[3 * r + 2] * d[2];
      sc->I_pix[n] = (int32_t)k;
      sc->pix2pt[k] = n;
      ++n;
    }
  return sc;
}

void orc_destroy(orc_scene* sc) {
  if (!sc) return;
  free(sc->v_off); free(sc->t_off); free(sc->f_off);
  free(sc->verts); free(sc->tris); free(sc->planes);
  free(sc->poses); free(sc->obj_mesh);
  free(sc->I_pix); free(sc->I_cam); free(sc->I_w); free(sc->pix2pt); free(sc->sym);
  free(sc);
}

int orc_set_mode(orc_scene* sc, int32_t radius_mode, int32_t nthreads) {
  if (!sc || radius_mode < 0 || radius_mode > 1 || nthreads < 1) return -1;
  sc->radius_mode = radius_mode;
  sc->nthreads = nthreads;
  return 0;
}

int32_t orc_num_points(const orc_scene* sc) { return sc ? sc->nI : -1; }

int orc_vertex_stage(const orc_scene* sc, int32_t mesh, int32_t pose, float* cam,
                     int32_t* uv) {
  if (!sc || mesh < 0 || mesh >= sc->n_mesh || pose < 0 || pose >= sc->P) return -1;
  int nv = sc->v_off[mesh + 1] - sc->v_off[mesh];
  int64_t* U = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)(nv > 0 ? nv : 1));
  int rc = vertex_stage_f32(sc, mesh, pose, cam, U, U + nv);
  for (int k = 0; k < nv; ++k) {
    uv[2 * k] = (int32_t)U[k];
    uv[2 * k + 1] = (int32_t)U[nv + k];
  }
  free(U);
  return rc;
}

int orc_render_objects(const orc_scene* sc, int32_t n, const int32_t* mesh,
                       const int32_t* pose, int32_t cull, double* depth) {
  if (!sc || n < 0) return -1;
  size_t npx = (size_t)sc->W * sc->H;
  float* cam = (float*)malloc(sizeof(float) * 3 * (size_t)(sc->max_v + 1));
  int64_t* U = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)(sc->max_v + 1));
  int rc = 0;
  for (int k = 0; k < n && !rc; ++k) {
    if (mesh[k] < 0 || mesh[k] >= sc->n_mesh || pose[k] < 0 || pose[k] >= sc->P) { rc = -1; break; }
    double* D = depth + (size_t)k * npx;
    for (size_t i = 0; i < npx; ++i) D[i] = INFINITY;
    rc = render_into(sc, mesh[k], pose[k], cull, D, cam, U, U + sc->max_v + 1);
  }
  free(cam);
  free(U);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* successor evaluation: Eq.(3) validity and Eq.(4) edge cost                */
/* ------------------------------------------------------------------------- */

typedef struct {
  double *DO, *DR, *RK;
  float* cam;
  int64_t* UV;
} scratch_t;

static void scratch_init(const orc_scene* sc, scratch_t* w) {
  size_t npx = (size_t)sc->W * sc->H;
  w->DO = (double*)malloc(sizeof(double) * npx);
  w->DR = (double*)malloc(sizeof(double) * npx);
  w->RK = (double*)malloc(sizeof(double) * npx);
  w->cam = (float*)malloc(sizeof(float) * 3 * (size_t)(sc->max_v + 1));
  w->UV = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)(sc->max_v + 1));
}

static void scratch_free(scratch_t* w) {
  free(w->DO); free(w->DR); free(w->RK); free(w->cam); free(w->UV);
}

typedef struct {
  const double* Dpar;    /* parent composite R_j, +inf = empty */
  const uint8_t* inVpar; /* per observed point: inside some parent volume */
  const uint8_t* nearVpar;
  int goal;
} parent_t;

/* One successor.  Writes status, cost, comps[5], flags[3]. */
static int eval_one(const orc_scene* sc, const parent_t* par, int mesh, int pose,
                    scratch_t* w, int32_t* status, int32_t* cost, int32_t* comps,
                    int32_t* flags) {
  const int W = sc->W, H = sc->H;
  const size_t npx = (size_t)W * H;
  for (size_t i = 0; i < npx; ++i) w->DO[i] = INFINITY;
  int rc = render_into(sc, mesh, pose, 1, w->DO, w->cam, w->UV, w->UV + sc->max_v + 1);
  if (rc) return rc;
  const double* Dp = par->Dpar;
  int valid = 1, ftie = 0;
  int32_t S = 0, nDR = 0;
  for (size_t i = 0; i < npx; ++i) {
    double z = w->DO[i];
    w->DR[i] = INFINITY;
    if (!(z < INFINITY)) continue;
    ++S;
    if (Dp[i] < INFINITY) {
      if (z < Dp[i]) valid = 0; /* the new object would occlude the parent scene */
      if (fabs(z - Dp[i]) <= FLAG_EPS) ftie = 1;
    } else {
      w->DR[i] = z; /* dR_{j+1}: points of the new object visible over R_j */
      ++nDR;
    }
  }
  int32_t nfd = 0, nfv = 0;
  comps[0] = S;
  comps[1] = nDR;
  flags[2] = ftie;
  if (!valid) {
    *status = 0;
    *cost = -1;
    comps[2] = comps[3] = comps[4] = -1;
    flags[0] = flags[1] = 0;
    return 0;
  }
  /* dJ_r: points of dR unexplained by I */
  int32_t dJr = 0;
  double q[3];
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      double z = w->DR[(size_t)v * W + u];
      if (!(z < INFINITY)) continue;
      backproject(sc, u, v, z, q);
      double m2 = min_d2_to_I(sc, q, u, v);
      if (m2 > sc->delta2) ++dJr;
      if (near_delta(sc, m2)) ++nfd;
    }
  /* dJ_o: observed points inside V(O_{j+1}) unexplained by dR; and at the goal
   * level the residual: observed points outside every volume that are unexplained
   * by the full render R_K = R_j with dR added.
   * Volume flags count only points whose membership flip would change this edge's
   * cost: near the candidate's boundary, "inside" contributes [unexplained by dR]
   * and "outside" contributes [outside the parent volumes and unexplained by R_K]
   * (0 below the goal level); near a parent's boundary (goal level, outside the
   * candidate) the flip toggles [unexplained by R_K]. */
  int32_t dJo = 0, res = 0;
  if (par->goal)
    for (size_t i = 0; i < npx; ++i) w->RK[i] = Dp[i] < INFINITY ? Dp[i] : w->DR[i];
  for (int k = 0; k < sc->nI; ++k) {
    const double* pc = sc->I_cam + 3 * (size_t)k;
    const int pix = sc->I_pix[k];
    const int up = pix % W, vp = pix / W;
    double vm = vol_margin(sc, mesh, pose, sc->I_w + 3 * (size_t)k);
    int inV = vm <= 0, nearV = fabs(vm) <= FLAG_EPS;
    int unexp_dr = 0, unexp_rk = 0;
    if (inV || nearV) {
      double m2 = min_d2_to_depth(sc, pc, up, vp, w->DR);
      unexp_dr = m2 > sc->delta2;
      if (near_delta(sc, m2)) ++nfd;
    }
    if (inV) dJo += unexp_dr;
    if (!par->goal) {
      if (nearV && unexp_dr) ++nfv;
      continue;
    }
    int inVp = par->inVpar[k], nearVp = par->nearVpar[k];
    if ((!inV && !inVp) || (nearV && !inVp) || (nearVp && !inV)) {
      double m2 = min_d2_to_depth(sc, pc, up, vp, w->RK);
      unexp_rk = m2 > sc->delta2;
      if (near_delta(sc, m2)) ++nfd;
    }
    if (!inV && !inVp) res += unexp_rk;
    if (nearV && unexp_dr != (inVp ? 0 : unexp_rk)) ++nfv;
    if (nearVp && !inV && unexp_rk) ++nfv;
  }
  comps[2] = dJr;
  comps[3] = dJo;
  comps[4] = res;
  flags[0] = nfd;
  flags[1] = nfv;
  *status = 1;
  *cost = dJr + dJo + res;
  return 0;
}

typedef struct {
  const orc_scene* sc;
  const parent_t* par;
  int n, tid, nth;
  const int32_t *cm, *cp;
  int32_t *st, *cost, *comps, *flags;
  int rc;
} job_t;

static void* eval_worker(void* arg) {
  job_t* jb = (job_t*)arg;
  scratch_t w;
  scratch_init(jb->sc, &w);
  jb->rc = 0;
  for (int i = jb->tid; i < jb->n; i += jb->nth) {
    int32_t cmp[5], flg[3];
    int rc = eval_one(jb->sc, jb->par, jb->cm[i], jb->cp[i], &w, jb->st + i, jb->cost + i,
                      cmp, flg);
    if (rc) { jb->rc = rc; break; }
    if (jb->comps) memcpy(jb->comps + 5 * (size_t)i, cmp, sizeof(cmp));
    if (jb->flags) memcpy(jb->flags + 3 * (size_t)i, flg, sizeof(flg));
  }
  scratch_free(&w);
  return NULL;
}

/* Parent materialisation: composite R_j and, for the goal level, which observed
 * points lie inside (or within the flag band of) some parent volume. */
typedef struct {
  parent_t p;
  double* D;
  uint8_t *inV, *nearV;
} parent_buf_t;

static int parent_build(const orc_scene* sc, int j, const int32_t* pm, const int32_t* pp,
                        parent_buf_t* pb) {
  size_t npx = (size_t)sc->W * sc->H;
  pb->D = (double*)malloc(sizeof(double) * npx);
  pb->inV = (uint8_t*)calloc((size_t)sc->nI + 1, 1);
  pb->nearV = (uint8_t*)calloc((size_t)sc->nI + 1, 1);
  for (size_t i = 0; i < npx; ++i) pb->D[i] = INFINITY;
  float* cam = (float*)malloc(sizeof(float) * 3 * (size_t)(sc->max_v + 1));
  int64_t* U = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)(sc->max_v + 1));
  int rc = 0;
  for (int k = 0; k < j && !rc; ++k)
    rc = render_into(sc, pm[k], pp[k], 1, pb->D, cam, U, U + sc->max_v + 1);
  free(cam);
  free(U);
  for (int i = 0; i < sc->nI; ++i)
    for (int k = 0; k < j; ++k) {
      double vm = vol_margin(sc, pm[k], pp[k], sc->I_w + 3 * (size_t)i);
      if (vm <= 0) pb->inV[i] = 1;
      if (fabs(vm) <= FLAG_EPS) pb->nearV[i] = 1;
    }
  pb->p.Dpar = pb->D;
  pb->p.inVpar = pb->inV;
  pb->p.nearVpar = pb->nearV;
  pb->p.goal = (j + 1 == sc->K);
  return rc;
}

static void parent_free(parent_buf_t* pb) {
  free(pb->D); free(pb->inV); free(pb->nearV);
}

static int eval_batch(const orc_scene* sc, const parent_t* par, int n, const int32_t* cm,
                      const int32_t* cp, int32_t* st, int32_t* cost, int32_t* comps,
                      int32_t* flags) {
  int nth = sc->nthreads < n ? sc->nthreads : n;
  if (nth < 1) nth = 1;
  job_t jobs[256];
  pthread_t th[256];
  if (nth > 256) nth = 256;
  for (int t = 0; t < nth; ++t) {
    job_t jb = {sc, par, n, t, nth, cm, cp, st, cost, comps, flags, 0};
    jobs[t] = jb;
  }
  if (nth == 1) {
    eval_worker(&jobs[0]);
  } else {
    for (int t = 0; t < nth; ++t) pthread_create(&th[t], NULL, eval_worker, &jobs[t]);
    for (int t = 0; t < nth; ++t) pthread_join(th[t], NULL);
  }
  for (int t = 0; t < nth; ++t)
    if (jobs[t].rc) return jobs[t].rc;
  return 0;
}

static int check_objects(const orc_scene* sc, int n, const int32_t* m, const int32_t* p) {
  for (int k = 0; k < n; ++k)
    if (m[k] < 0 || m[k] >= sc->n_mesh || p[k] < 0 || p[k] >= sc->P) return -1;
  return 0;
}

int orc_eval(const orc_scene* sc, int32_t j, const int32_t* par_mesh, const int32_t* par_pose,
             int32_t n, const int32_t* cand_mesh, const int32_t* cand_pose, int32_t* status,
             int32_t* cost, int32_t* comps, int32_t* flags) {
  if (!sc || j < 0 || j >= (sc->K > 0 ? sc->K : 1) || n < 0) return -1;
  if (check_objects(sc, j, par_mesh, par_pose) || check_objects(sc, n, cand_mesh, cand_pose))
    return -1;
  parent_buf_t pb;
  int rc = parent_build(sc, j, par_mesh, par_pose, &pb);
  if (!rc) rc = eval_batch(sc, &pb.p, n, cand_mesh, cand_pose, status, cost, comps, flags);
  parent_free(&pb);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* one-shot costs of a full assignment                                       */
/* ------------------------------------------------------------------------- */

/* ------------------------------------------------------------------------- */
/* overlap heuristic (Sec. IV-C)                                             */
/* ------------------------------------------------------------------------- */

/* h_overlap(s) = |I| - #{p in I : p in V_j}, V_j the union of the volumes of the j
 * placed objects: for the parent, and for each child that adds one candidate
 * object.  flags[c] counts the points whose membership in any of the volumes
 * involved is decided within FLAG_EPS of a boundary. */
int orc_overlap(const orc_scene* sc, int32_t j, const int32_t* pm, const int32_t* pp, int32_t n,
                const int32_t* cm, const int32_t* cp, int64_t* h_parent, int64_t* h_child,
                int32_t* flags) {
  if (!sc || j < 0 || n < 0 || (j > 0 && (!pm || !pp)) || (n > 0 && (!cm || !cp)))
    return -1;
  if (check_objects(sc, j, pm, pp) || check_objects(sc, n, cm, cp)) return -2;
  uint8_t* inVj = (uint8_t*)calloc((size_t)sc->nI + 1, 1);
  uint8_t* nearVj = (uint8_t*)calloc((size_t)sc->nI + 1, 1);
  if (!inVj || !nearVj) {
    free(inVj);
    free(nearVj);
    return -3;
  }
  int64_t inside = 0;
  for (int i = 0; i < sc->nI; ++i) {
    for (int k = 0; k < j; ++k) {
      const double vm = vol_margin(sc, pm[k], pp[k], sc->I_w + 3 * (size_t)i);
      if (vm <= 0) inVj[i] = 1;
      if (fabs(vm) <= FLAG_EPS) nearVj[i] = 1;
    }
    inside += inVj[i];
  }
  *h_parent = sc->nI - inside;
  for (int c = 0; c < n; ++c) {
    int64_t in_child = 0;
    int32_t fl = 0;
    for (int i = 0; i < sc->nI; ++i) {
      const double vm = vol_margin(sc, cm[c], cp[c], sc->I_w + 3 * (size_t)i);
      in_child += (inVj[i] || vm <= 0) ? 1 : 0;
      fl += (nearVj[i] || fabs(vm) <= FLAG_EPS) ? 1 : 0;
    }
    h_child[c] = sc->nI - in_child;
    flags[c] = fl;
  }
  free(inVj);
  free(nearVj);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* local ICP alignment (Sec. IV-E, compensating for discretization)           */
/* ------------------------------------------------------------------------- */

/* One linearised point-to-plane step (Chen and Medioni's ICP, restricted to the
 * table-plane motions).  For pairs (a_k, p_k) with unit normals n_k at p_k and
 * the centroid c of the a_k, a small rotation phi about the vertical axis through
 * c followed by a translation (tx, ty) leaves the residual n.(a + phi z x (a - c)
 * + t - p); the step minimises the sum of its squares, with the normal matrix
 * damped by 1e-6 of its diagonal (plus 1e-12) so that motions the pairs leave
 * unconstrained stay put.  out = (phi, tx', ty'): the same motion as a rotation
 * about the world z axis followed by the translation t' = c + t - R(phi) c. */
int orc_icp_step(int32_t n, const double* a, const double* p, const double* nrm, double* out) {
  if (n < 1 || !a || !p || !nrm || !out) return -1;
  double cx = 0, cy = 0;
  for (int k = 0; k < n; ++k) {
    cx += a[3 * k];
    cy += a[3 * k + 1];
  }
  cx /= n;
  cy /= n;
  double A[3][3] = {{0}}, b[3] = {0};
  for (int k = 0; k < n; ++k) {
    const double* ak = a + 3 * k;
    const double* pk = p + 3 * k;
    const double* nk = nrm + 3 * k;
    const double J[3] = {nk[1] * (ak[0] - cx) - nk[0] * (ak[1] - cy), nk[0], nk[1]};
    const double r = nk[0] * (ak[0] - pk[0]) + nk[1] * (ak[1] - pk[1]) + nk[2] * (ak[2] - pk[2]);
    for (int u = 0; u < 3; ++u) {
      for (int v = 0; v < 3; ++v) A[u][v] += J[u] * J[v];
      b[u] -= J[u] * r;
    }
  }
  for (int u = 0; u < 3; ++u) A[u][u] += 1e-6 * A[u][u] + 1e-12;
  /* Cramer's rule on the symmetric positive definite 3x3 system */
  const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                     A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                     A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  double x[3];
  for (int c = 0; c < 3; ++c) {
    double M[3][3];
    for (int u = 0; u < 3; ++u)
      for (int v = 0; v < 3; ++v) M[u][v] = v == c ? b[u] : A[u][v];
    x[c] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
            M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
            M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) / det;
  }
  const double co = cos(x[0]), si = sin(x[0]);
  out[0] = x[0];
  out[1] = cx + x[1] - (co * cx - si * cy);
  out[2] = cy + x[2] - (si * cx + co * cy);
  return 0;
}

static int near_half(double f) { /* f within ICP_FLAG_PX of a rounding boundary */
  const double r = f - floor(f);
  return fabs(r - 0.5) < ICP_FLAG_PX;
}

/* Surface normal of the observed point at pixel (u, v), world frame, unit length
 * and facing the camera: the cross product of the central differences of its four
 * pixel neighbours, which must all be observed and within `radius` of it.
 * Returns 0 when there is none; *near is set when a neighbour's distance lies
 * within ICP_FLAG_EPS of the radius. */
static int observed_normal(const orc_scene* sc, int u, int v, double radius, double* n,
                           int* near) {
  const int W = sc->W, H = sc->H;
  if (u < 1 || v < 1 || u > W - 2 || v > H - 2) return 0;
  const int c = sc->pix2pt[(size_t)v * W + u];
  const int nb[4] = {sc->pix2pt[(size_t)v * W + u + 1], sc->pix2pt[(size_t)v * W + u - 1],
                     sc->pix2pt[(size_t)(v + 1) * W + u], sc->pix2pt[(size_t)(v - 1) * W + u]};
  if (c < 0 || nb[0] < 0 || nb[1] < 0 || nb[2] < 0 || nb[3] < 0) return 0;
  const double* pc = sc->I_w + 3 * (size_t)c;
  int ok = 1;
  for (int k = 0; k < 4; ++k) {
    const double dk = sqrt(d2(pc, sc->I_w + 3 * (size_t)nb[k]));
    if (fabs(dk - radius) <= ICP_FLAG_EPS) *near = 1;
    if (dk > radius) ok = 0;
  }
  if (!ok) return 0;
  const double *px1 = sc->I_w + 3 * (size_t)nb[0], *px0 = sc->I_w + 3 * (size_t)nb[1];
  const double *py1 = sc->I_w + 3 * (size_t)nb[2], *py0 = sc->I_w + 3 * (size_t)nb[3];
  const double e1[3] = {px1[0] - px0[0], px1[1] - px0[1], px1[2] - px0[2]};
  const double e2[3] = {py1[0] - py0[0], py1[1] - py0[1], py1[2] - py0[2]};
  double m[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                 e1[0] * e2[1] - e1[1] * e2[0]};
  const double len = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
  if (!(len > 0)) return 0;
  /* the camera centre in the world frame is -Rinv t */
  double cw[3];
  for (int r = 0; r < 3; ++r)
    cw[r] = -(sc->Rinv[3 * r] * sc->t[0] + sc->Rinv[3 * r + 1] * sc->t[1] +
              sc->Rinv[3 * r + 2] * sc->t[2]);
  const double f = m[0] * (cw[0] - pc[0]) + m[1] * (cw[1] - pc[1]) + m[2] * (cw[2] - pc[2]);
  const double sg = f < 0 ? -1.0 : 1.0;
  for (int r = 0; r < 3; ++r) n[r] = sg * m[r] / len;
  return 1;
}

/* ICP of candidate (mesh, pose) against I over the non-occluded part of its
 * render, for `iters` rounds of projective association (the observed point at
 * the pixel nearest the projection of the moved model point, kept when it has a
 * normal and lies within `radius`) and a point-to-plane step.  Writes the
 * adjusted pose (x, y, cos, sin) and the match count of the last association;
 * status 0 when the candidate occludes the parent (no alignment: the grid pose
 * is returned). */
static int icp_one(const orc_scene* sc, const double* Dp, int mesh, int pose, int iters,
                   double radius, scratch_t* w, double* pose_out, int32_t* n_match,
                   int32_t* status, int32_t* flags) {
  const int W = sc->W, H = sc->H;
  const size_t npx = (size_t)W * H;
  for (size_t i = 0; i < npx; ++i) w->DO[i] = INFINITY;
  int rc = render_into(sc, mesh, pose, 1, w->DO, w->cam, w->UV, w->UV + sc->max_v + 1);
  if (rc) return rc;
  int valid = 1, fl = 0, nq = 0;
  for (size_t i = 0; i < npx; ++i) {
    const double z = w->DO[i];
    if (!(z < INFINITY)) continue;
    if (Dp[i] < INFINITY) {
      if (z < Dp[i]) valid = 0;
      if (fabs(z - Dp[i]) <= FLAG_EPS) fl = 1;
    } else {
      ++nq;
    }
  }
  const float* pz = sc->poses + 4 * (size_t)pose;
  for (int k = 0; k < 4; ++k) pose_out[k] = pz[k];
  *n_match = 0;
  if (!valid) {
    *status = 0;
    *flags = fl;
    return 0;
  }
  /* model points: the non-occluded part dR, in the world frame, back-projected from
   * the rendered depth as a float32 depth image holds it (reading: Sec. IV-E aligns
   * the rendered object, and a rendered depth image is float32 like the observed
   * one) */
  double* Q = (double*)malloc(sizeof(double) * 3 * (size_t)(nq + 1));
  double* A = (double*)malloc(sizeof(double) * 9 * (size_t)(nq + 1));
  if (!Q || !A) {
    free(Q); free(A);
    return -3;
  }
  double* Pm = A + 3 * (size_t)(nq + 1);
  double* Nm = Pm + 3 * (size_t)(nq + 1);
  int m = 0;
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      const size_t i = (size_t)v * W + u;
      if (!(w->DO[i] < INFINITY) || Dp[i] < INFINITY) continue;
      double q[3], d[3];
      backproject(sc, u, v, (double)(float)w->DO[i], q);
      for (int r = 0; r < 3; ++r) d[r] = q[r] - sc->t[r];
      for (int r = 0; r < 3; ++r)
        Q[3 * m + r] = sc->Rinv[3 * r] * d[0] + sc->Rinv[3 * r + 1] * d[1] + sc->Rinv[3 * r + 2] * d[2];
      ++m;
    }
  const float* M = sc->s.cam_from_world;
  const double r2 = radius * radius;
  double phi = 0, tx = 0, ty = 0;
  for (int it = 0; it < iters; ++it) {
    const double c = cos(phi), s = sin(phi);
    int nm = 0;
    for (int k = 0; k < m; ++k) {
      const double* q = Q + 3 * k;
      const double a[3] = {c * q[0] - s * q[1] + tx, s * q[0] + c * q[1] + ty, q[2]};
      double ac[3];
      for (int r = 0; r < 3; ++r)
        ac[r] = (double)M[4 * r] * a[0] + (double)M[4 * r + 1] * a[1] +
                (double)M[4 * r + 2] * a[2] + (double)M[4 * r + 3];
      if (!(ac[2] > 0)) continue;
      const double uf = sc->fx * ac[0] / ac[2] + sc->cx, vf = sc->fy * ac[1] / ac[2] + sc->cy;
      if (near_half(uf) || near_half(vf)) ++fl;
      const double iu = floor(uf + 0.5), iv = floor(vf + 0.5);
      if (iu < 0 || iu > W - 1 || iv < 0 || iv > H - 1) continue;
      const int pt = sc->pix2pt[(size_t)iv * W + (size_t)iu];
      if (pt < 0) continue;
      double nrm[3];
      int near = 0;
      const int has_n = observed_normal(sc, (int)iu, (int)iv, radius, nrm, &near);
      fl += near;
      if (!has_n) continue;
      const double* p = sc->I_w + 3 * (size_t)pt;
      const double dd = d2(a, p);
      if (fabs(sqrt(dd) - radius) <= ICP_FLAG_EPS) ++fl;
      if (dd > r2) continue;
      for (int r = 0; r < 3; ++r) {
        A[3 * nm + r] = a[r];
        Pm[3 * nm + r] = p[r];
        Nm[3 * nm + r] = nrm[r];
      }
      ++nm;
    }
    *n_match = nm;
    if (nm < 3) break;
    double st[3];
    orc_icp_step(nm, A, Pm, Nm, st);
    /* compose: the step after the motion so far */
    const double cd = cos(st[0]), sd = sin(st[0]);
    const double nx = cd * tx - sd * ty + st[1], ny = sd * tx + cd * ty + st[2];
    phi += st[0];
    tx = nx;
    ty = ny;
  }
  free(Q); free(A);
  /* adjusted pose: the motion applied after the grid placement */
  const double c = cos(phi), s = sin(phi);
  const double x = pz[0], y = pz[1], pc = pz[2], ps = pz[3];
  pose_out[0] = c * x - s * y + tx;
  pose_out[1] = s * x + c * y + ty;
  pose_out[2] = pc * c - ps * s;
  pose_out[3] = ps * c + pc * s;
  *status = 1;
  *flags = fl;
  return 0;
}

int orc_icp(const orc_scene* sc, int32_t j, const int32_t* pm, const int32_t* pp, int32_t n,
            const int32_t* cm, const int32_t* cp, int32_t iters, double radius, double* pose_out,
            int32_t* n_match, int32_t* status, int32_t* flags) {
  if (!sc || j < 0 || n < 0 || iters < 0 || !(radius > 0) || (j > 0 && (!pm || !pp)) ||
      (n > 0 && (!cm || !cp || !pose_out || !n_match || !status || !flags)))
    return -1;
  if (!sc->I_w) return -1;
  if (check_objects(sc, j, pm, pp) || check_objects(sc, n, cm, cp)) return -2;
  parent_buf_t pb;
  int rc = parent_build(sc, j, pm, pp, &pb);
  scratch_t w;
  scratch_init(sc, &w);
  for (int c = 0; c < n && !rc; ++c)
    rc = icp_one(sc, pb.D, cm[c], cp[c], iters, radius, &w, pose_out + 4 * (size_t)c,
                 n_match + c, status + c, flags + c);
  scratch_free(&w);
  parent_free(&pb);
  return rc;
}

static int cmp_pair(const int32_t* a, const int32_t* b) {
  if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
  if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
  return 0;
}

/* sorts K (mesh, pose) pairs in place into canonical order */
static void canon(int K, int32_t* pairs) {
  for (int a = 1; a < K; ++a)
    for (int b = a; b > 0 && cmp_pair(pairs + 2 * b, pairs + 2 * (b - 1)) < 0; --b) {
      int32_t t0 = pairs[2 * b], t1 = pairs[2 * b + 1];
      pairs[2 * b] = pairs[2 * b - 2];
      pairs[2 * b + 1] = pairs[2 * b - 1];
      pairs[2 * b - 2] = t0;
      pairs[2 * b - 1] = t1;
    }
}

static int cmp_key(int K, const int32_t* a, const int32_t* b) {
  for (int k = 0; k < K; ++k) {
    int c = cmp_pair(a + 2 * k, b + 2 * k);
    if (c) return c;
  }
  return 0;
}

int orc_jtree(const orc_scene* sc, int32_t K, const int32_t* mesh, const int32_t* pose,
              int64_t* out) {
  if (!sc || K < 1 || K > ORC_MAX_K || check_objects(sc, K, mesh, pose)) return -1;
  const int W = sc->W, H = sc->H;
  const size_t npx = (size_t)W * H;
  int32_t obj[2 * ORC_MAX_K];
  for (int k = 0; k < K; ++k) { obj[2 * k] = mesh[k]; obj[2 * k + 1] = pose[k]; }
  canon(K, obj);
  double* D = (double*)malloc(sizeof(double) * npx * (K + 2));
  double* RK = D + npx * K;
  double* OW = D + npx * (K + 1);
  int32_t m[ORC_MAX_K], p[ORC_MAX_K];
  for (int k = 0; k < K; ++k) { m[k] = obj[2 * k]; p[k] = obj[2 * k + 1]; }
  int rc = orc_render_objects(sc, K, m, p, 1, D);
  if (rc) { free(D); return rc; }
  int8_t* owner = (int8_t*)malloc(npx);
  int occ[ORC_MAX_K][ORC_MAX_K];
  memset(occ, 0, sizeof(occ));
  int ftie = 0;
  for (size_t i = 0; i < npx; ++i) {
    int best = -1;
    double bz = INFINITY;
    for (int k = 0; k < K; ++k) {
      double z = D[k * npx + i];
      if (z < bz) { bz = z; best = k; } /* strict: ties stay with the earlier object */
    }
    owner[i] = (int8_t)best;
    RK[i] = bz;
    for (int a = 0; a < K; ++a)
      for (int b = 0; b < K; ++b) {
        if (a == b) continue;
        double za = D[a * npx + i], zb = D[b * npx + i];
        if (za < zb && zb < INFINITY) occ[a][b] = 1;
        if (za < INFINITY && zb < INFINITY && fabs(za - zb) <= FLAG_EPS) ftie = 1;
      }
  }
  /* the order constraint of Eq.(3) can be met iff "a occludes b" is acyclic */
  int indeg[ORC_MAX_K] = {0}, done[ORC_MAX_K] = {0}, nd = 0;
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) indeg[b] += occ[a][b];
  for (int it = 0; it < K; ++it)
    for (int a = 0; a < K; ++a)
      if (!done[a] && indeg[a] == 0) {
        done[a] = 1;
        ++nd;
        for (int b = 0; b < K; ++b) indeg[b] -= occ[a][b];
      }
  int valid = (nd == K);
  int64_t nfd = 0, nfv = 0, Jr = 0, Jo_tree = 0, res = 0, Jo_raw = 0;
  double q[3];
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      double z = RK[(size_t)v * W + u];
      if (!(z < INFINITY)) continue;
      backproject(sc, u, v, z, q);
      double m2 = min_d2_to_I(sc, q, u, v);
      if (m2 > sc->delta2) ++Jr;
      if (near_delta(sc, m2)) ++nfd;
    }
  uint8_t* inAny = (uint8_t*)calloc((size_t)sc->nI + 1, 1);
  for (int k = 0; k < K; ++k) {
    for (size_t i = 0; i < npx; ++i) OW[i] = owner[i] == k ? RK[i] : INFINITY;
    for (int t = 0; t < sc->nI; ++t) {
      double vm = vol_margin(sc, m[k], p[k], sc->I_w + 3 * (size_t)t);
      if (fabs(vm) <= FLAG_EPS) ++nfv;
      if (vm > 0) continue;
      inAny[t] = 1;
      int pix = sc->I_pix[t];
      double m2 = min_d2_to_depth(sc, sc->I_cam + 3 * (size_t)t, pix % W, pix / W, OW);
      if (m2 > sc->delta2) ++Jo_tree;
      if (near_delta(sc, m2)) ++nfd;
    }
  }
  for (int t = 0; t < sc->nI; ++t) {
    int pix = sc->I_pix[t];
    double m2 = min_d2_to_depth(sc, sc->I_cam + 3 * (size_t)t, pix % W, pix / W, RK);
    int unexp = m2 > sc->delta2;
    if (near_delta(sc, m2)) ++nfd;
    Jo_raw += unexp;
    if (!inAny[t]) res += unexp;
  }
  out[0] = valid;
  out[1] = Jr + Jo_tree + res;
  out[2] = Jr + Jo_raw;
  out[3] = nfd;
  out[4] = nfv;
  out[5] = ftie;
  free(inAny);
  free(owner);
  free(D);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* searches                                                                  */
/* ------------------------------------------------------------------------- */

/* distinct mesh ids still to place, given the placed ones (multiset difference) */
int orc_set_symmetric(orc_scene* sc, int32_t mesh, int32_t symmetric) {
  if (!sc || mesh < 0 || mesh >= sc->n_mesh) return -1;
  sc->sym[mesh] = symmetric ? 1 : 0;
  return 0;
}

/* The poses a search tries for `mesh`: the subset itself, or for a rotationally
 * symmetric mesh (Sec. IV-E: only (x, y) matters) the first pose of the subset at
 * each distinct (x, y).  Returns the count written to out. */
static int mesh_subset(const orc_scene* sc, int mesh, int nsub, const int32_t* sub,
                       int32_t* out) {
  int n = 0;
  for (int b = 0; b < nsub; ++b) {
    int dup = 0;
    if (sc->sym[mesh]) {
      const float* q = sc->poses + 4 * (size_t)sub[b];
      for (int a = 0; a < n && !dup; ++a) {
        const float* r = sc->poses + 4 * (size_t)out[a];
        dup = (q[0] == r[0] && q[1] == r[1]);
      }
    }
    if (!dup) out[n++] = sub[b];
  }
  return n;
}

static int remaining_meshes(const orc_scene* sc, int j, const int32_t* pm, int32_t* out) {
  int32_t left[ORC_MAX_K];
  int nl = sc->K;
  memcpy(left, sc->obj_mesh, sizeof(int32_t) * sc->K);
  for (int k = 0; k < j; ++k)
    for (int a = 0; a < nl; ++a)
      if (left[a] == pm[k]) { left[a] = left[--nl]; break; }
  int nd = 0;
  for (int a = 0; a < nl; ++a) {
    int seen = 0;
    for (int b = 0; b < nd; ++b) seen |= (out[b] == left[a]);
    if (!seen) out[nd++] = left[a];
  }
  /* ascending ids, so candidate order is deterministic */
  for (int a = 1; a < nd; ++a)
    for (int b = a; b > 0 && out[b] < out[b - 1]; --b) {
      int32_t t = out[b]; out[b] = out[b - 1]; out[b - 1] = t;
    }
  return nd;
}

typedef struct {
  const orc_scene* sc;
  int nsub;
  const int32_t* sub;
  int64_t best_cost;
  int32_t best_key[2 * ORC_MAX_K];
  int have;
  int64_t n_eval, n_exp, n_goal;
  int rc;
} exh_t;

static void exh_rec(exh_t* E, int j, int32_t* pm, int32_t* pp, int64_t g) {
  const orc_scene* sc = E->sc;
  int32_t ids[ORC_MAX_K];
  int nd = remaining_meshes(sc, j, pm, ids);
  int cap = nd * E->nsub;
  int32_t* cm = (int32_t*)malloc(sizeof(int32_t) * 4 * (size_t)(cap + 1));
  int32_t *cp = cm + cap, *st = cm + 2 * cap, *cost = cm + 3 * cap;
  int n = 0;
  for (int a = 0; a < nd; ++a) {
    const int c = mesh_subset(sc, ids[a], E->nsub, E->sub, cp + n);
    for (int b = 0; b < c; ++b) cm[n + b] = ids[a];
    n += c;
  }
  parent_buf_t pb;
  int rc = parent_build(sc, j, pm, pp, &pb);
  if (!rc) rc = eval_batch(sc, &pb.p, n, cm, cp, st, cost, NULL, NULL);
  parent_free(&pb);
  if (rc) { E->rc = rc; free(cm); return; }
  E->n_eval += n;
  E->n_exp += 1;
  for (int i = 0; i < n && !E->rc; ++i) {
    if (!st[i]) continue;
    pm[j] = cm[i];
    pp[j] = cp[i];
    int64_t g2 = g + cost[i];
    if (j + 1 == sc->K) {
      int32_t key[2 * ORC_MAX_K];
      for (int k = 0; k < sc->K; ++k) { key[2 * k] = pm[k]; key[2 * k + 1] = pp[k]; }
      canon(sc->K, key);
      E->n_goal++;
      if (!E->have || g2 < E->best_cost ||
          (g2 == E->best_cost && cmp_key(sc->K, key, E->best_key) < 0)) {
        E->have = 1;
        E->best_cost = g2;
        memcpy(E->best_key, key, sizeof(int32_t) * 2 * sc->K);
      }
    } else {
      exh_rec(E, j + 1, pm, pp, g2);
    }
  }
  free(cm);
}

static int32_t* all_poses(const orc_scene* sc, int32_t* n_sub, const int32_t* sub) {
  if (sub && *n_sub > 0) return NULL;
  int32_t* a = (int32_t*)malloc(sizeof(int32_t) * sc->P);
  for (int i = 0; i < sc->P; ++i) a[i] = i;
  *n_sub = sc->P;
  return a;
}

int orc_search_exhaustive(const orc_scene* sc, int32_t n_sub, const int32_t* pose_sub,
                          int32_t* best_mesh, int32_t* best_pose, int64_t* stats) {
  if (!sc || sc->K < 1) return -1;
  int32_t* own = all_poses(sc, &n_sub, pose_sub);
  for (int i = 0; i < n_sub && !own; ++i)
    if (pose_sub[i] < 0 || pose_sub[i] >= sc->P) return -1;
  exh_t E;
  memset(&E, 0, sizeof(E));
  E.sc = sc;
  E.nsub = n_sub;
  E.sub = own ? own : pose_sub;
  int32_t pm[ORC_MAX_K], pp[ORC_MAX_K];
  exh_rec(&E, 0, pm, pp, 0);
  free(own);
  if (E.rc) return E.rc;
  stats[0] = E.have ? E.best_cost : -1;
  stats[1] = E.n_eval;
  stats[2] = E.n_exp;
  stats[3] = E.n_goal;
  if (!E.have) return 1;
  for (int k = 0; k < sc->K; ++k) {
    best_mesh[k] = E.best_key[2 * k];
    best_pose[k] = E.best_key[2 * k + 1];
  }
  return 0;
}

/* --- uniform-cost search over canonical states ------------------------------ */

typedef struct {
  int64_t g;
  int32_t j;
  int32_t key[2 * ORC_MAX_K]; /* canonical (mesh, pose) pairs of the placed objects */
} node_t;

typedef struct {
  node_t* nodes;
  int n, cap;
  int* heap;
  int hn, hcap;
  int* tab; /* open addressing: node index or -1 */
  int tcap;
} ucs_t;

static int node_less(const node_t* a, const node_t* b) {
  if (a->g != b->g) return a->g < b->g;
  if (a->j != b->j) return a->j > b->j; /* deeper first */
  return cmp_key(a->j, a->key, b->key) < 0;
}

static uint64_t key_hash(int j, const int32_t* key) {
  uint64_t h = 1469598103934665603ull ^ (uint64_t)j;
  for (int k = 0; k < 2 * j; ++k) {
    h ^= (uint32_t)key[k];
    h *= 1099511628211ull;
  }
  return h;
}

static void heap_push(ucs_t* U, int id) {
  if (U->hn == U->hcap) {
    U->hcap = U->hcap ? 2 * U->hcap : 1024;
    U->heap = (int*)realloc(U->heap, sizeof(int) * U->hcap);
  }
  int i = U->hn++;
  U->heap[i] = id;
  while (i > 0) {
    int p = (i - 1) / 2;
    if (!node_less(&U->nodes[U->heap[i]], &U->nodes[U->heap[p]])) break;
    int t = U->heap[i]; U->heap[i] = U->heap[p]; U->heap[p] = t;
    i = p;
  }
}

static int heap_pop(ucs_t* U) {
  int top = U->heap[0];
  U->heap[0] = U->heap[--U->hn];
  int i = 0;
  for (;;) {
    int l = 2 * i + 1, r = l + 1, m = i;
    if (l < U->hn && node_less(&U->nodes[U->heap[l]], &U->nodes[U->heap[m]])) m = l;
    if (r < U->hn && node_less(&U->nodes[U->heap[r]], &U->nodes[U->heap[m]])) m = r;
    if (m == i) break;
    int t = U->heap[i]; U->heap[i] = U->heap[m]; U->heap[m] = t;
    i = m;
  }
  return top;
}

/* finds the table slot of a state key (existing or empty) */
static int tab_slot(ucs_t* U, int j, const int32_t* key) {
  uint64_t h = key_hash(j, key);
  int mask = U->tcap - 1;
  int s = (int)(h & (uint64_t)mask);
  for (;;) {
    int id = U->tab[s];
    if (id < 0) return s;
    if (U->nodes[id].j == j && cmp_key(j, U->nodes[id].key, key) == 0) return s;
    s = (s + 1) & mask;
  }
}

static void tab_grow(ucs_t* U) {
  int oc = U->tcap;
  int* old = U->tab;
  U->tcap = oc ? 2 * oc : 1 << 12;
  U->tab = (int*)malloc(sizeof(int) * U->tcap);
  for (int i = 0; i < U->tcap; ++i) U->tab[i] = -1;
  for (int i = 0; i < oc; ++i)
    if (old[i] >= 0) {
      int s = tab_slot(U, U->nodes[old[i]].j, U->nodes[old[i]].key);
      U->tab[s] = old[i];
    }
  free(old);
}

int orc_search_ucs(const orc_scene* sc, int32_t n_sub, const int32_t* pose_sub,
                   int32_t* best_mesh, int32_t* best_pose, int64_t* stats) {
  if (!sc || sc->K < 1) return -1;
  int32_t* own = all_poses(sc, &n_sub, pose_sub);
  const int32_t* sub = own ? own : pose_sub;
  for (int i = 0; i < n_sub; ++i)
    if (sub[i] < 0 || sub[i] >= sc->P) { free(own); return -1; }
  ucs_t U;
  memset(&U, 0, sizeof(U));
  tab_grow(&U);
  /* per state: nodes[] holds the best g found; closed states have j = -1 - j */
  uint8_t* closed = NULL;
  int ccap = 0;
  U.cap = 1024;
  U.nodes = (node_t*)malloc(sizeof(node_t) * U.cap);
  memset(&U.nodes[0], 0, sizeof(node_t));
  U.n = 1;
  U.tab[tab_slot(&U, 0, U.nodes[0].key)] = 0;
  heap_push(&U, 0);
  int64_t n_eval = 0, n_exp = 0, n_goal = 0;
  int found = -1, rc = 0;
  /* heap entries carry their own g: duplicates are pushed as fresh nodes and the
   * table maps a key to its best node; stale entries are skipped on pop */
  while (U.hn > 0) {
    int id = heap_pop(&U);
    node_t cur = U.nodes[id];
    int s = tab_slot(&U, cur.j, cur.key);
    if (U.tab[s] != id) continue; /* superseded by a cheaper duplicate */
    if (id >= ccap) {
      int nc = ccap ? ccap : 1024;
      while (nc <= id) nc *= 2;
      closed = (uint8_t*)realloc(closed, nc);
      memset(closed + ccap, 0, nc - ccap);
      ccap = nc;
    }
    if (closed[id]) continue;
    closed[id] = 1;
    if (cur.j == sc->K) { found = id; break; }
    n_exp++;
    int32_t pm[ORC_MAX_K], pp[ORC_MAX_K], ids[ORC_MAX_K];
    for (int k = 0; k < cur.j; ++k) { pm[k] = cur.key[2 * k]; pp[k] = cur.key[2 * k + 1]; }
    int nd = remaining_meshes(sc, cur.j, pm, ids);
    int cap = nd * n_sub;
    int32_t* cm = (int32_t*)malloc(sizeof(int32_t) * 4 * (size_t)(cap + 1));
    int32_t *cp = cm + cap, *st = cm + 2 * cap, *cost = cm + 3 * cap;
    int n = 0;
    for (int a = 0; a < nd; ++a) {
      const int c = mesh_subset(sc, ids[a], n_sub, sub, cp + n);
      for (int b = 0; b < c; ++b) cm[n + b] = ids[a];
      n += c;
    }
    parent_buf_t pb;
    rc = parent_build(sc, cur.j, pm, pp, &pb);
    if (!rc) rc = eval_batch(sc, &pb.p, n, cm, cp, st, cost, NULL, NULL);
    parent_free(&pb);
    if (rc) { free(cm); break; }
    n_eval += n;
    for (int i = 0; i < n; ++i) {
      if (!st[i]) continue;
      node_t ch;
      ch.g = cur.g + cost[i];
      ch.j = cur.j + 1;
      memset(ch.key, 0, sizeof(ch.key));
      memcpy(ch.key, cur.key, sizeof(int32_t) * 2 * cur.j);
      ch.key[2 * cur.j] = cm[i];
      ch.key[2 * cur.j + 1] = cp[i];
      canon(ch.j, ch.key);
      if (ch.j == sc->K) n_goal++;
      if (2 * (U.n + 1) > U.tcap) tab_grow(&U);
      int sl = tab_slot(&U, ch.j, ch.key);
      int old = U.tab[sl];
      if (old >= 0) {
        if (old < ccap && closed[old]) continue;
        if (!node_less(&ch, &U.nodes[old])) continue;
      }
      if (U.n == U.cap) {
        U.cap *= 2;
        U.nodes = (node_t*)realloc(U.nodes, sizeof(node_t) * U.cap);
      }
      U.nodes[U.n] = ch;
      U.tab[sl] = U.n;
      heap_push(&U, U.n);
      U.n++;
    }
    free(cm);
  }
  free(own);
  if (!rc) {
    stats[0] = found >= 0 ? U.nodes[found].g : -1;
    stats[1] = n_eval;
    stats[2] = n_exp;
    stats[3] = n_goal;
    if (found >= 0)
      for (int k = 0; k < sc->K; ++k) {
        best_mesh[k] = U.nodes[found].key[2 * k];
        best_pose[k] = U.nodes[found].key[2 * k + 1];
      }
  }
  free(U.nodes); free(U.heap); free(U.tab); free(closed);
  if (rc) return rc;
  return found >= 0 ? 0 : 1;
}

/* --- brute force over joint assignments (independent of the tree) ---------- */

typedef struct {
  const orc_scene* sc;
  int nsub, tid, nth;
  const int32_t* sub;
  const int32_t* lists; /* per object k: its poses at lists + k * nsub, count cnt[k] */
  const int32_t* cnt;
  int64_t best;
  int32_t key[2 * ORC_MAX_K];
  int have;
  int64_t nvalid;
  int rc;
} bf_t;

static void* bf_worker(void* arg) {
  bf_t* B = (bf_t*)arg;
  const orc_scene* sc = B->sc;
  int K = sc->K;
  int64_t total = 1;
  for (int k = 0; k < K; ++k) total *= B->cnt[k];
  for (int64_t idx = B->tid; idx < total; idx += B->nth) {
    int32_t m[ORC_MAX_K], p[ORC_MAX_K];
    int64_t r = idx;
    for (int k = 0; k < K; ++k) {
      m[k] = sc->obj_mesh[k];
      p[k] = B->lists[(size_t)k * B->nsub + r % B->cnt[k]];
      r /= B->cnt[k];
    }
    int64_t out[6];
    int rc = orc_jtree(sc, K, m, p, out);
    if (rc) { B->rc = rc; return NULL; }
    if (!out[0]) continue;
    B->nvalid++;
    int32_t key[2 * ORC_MAX_K];
    for (int k = 0; k < K; ++k) { key[2 * k] = m[k]; key[2 * k + 1] = p[k]; }
    canon(K, key);
    if (!B->have || out[1] < B->best || (out[1] == B->best && cmp_key(K, key, B->key) < 0)) {
      B->have = 1;
      B->best = out[1];
      memcpy(B->key, key, sizeof(int32_t) * 2 * K);
    }
  }
  return NULL;
}

int orc_bruteforce_joint(const orc_scene* sc, int32_t n_sub, const int32_t* pose_sub,
                         int32_t* best_mesh, int32_t* best_pose, int64_t* stats) {
  if (!sc || sc->K < 1) return -1;
  int32_t* own = all_poses(sc, &n_sub, pose_sub);
  const int32_t* sub = own ? own : pose_sub;
  for (int i = 0; i < n_sub; ++i)
    if (sub[i] < 0 || sub[i] >= sc->P) { free(own); return -1; }
  int32_t* lists = (int32_t*)malloc(sizeof(int32_t) * (size_t)sc->K * (size_t)(n_sub + 1));
  int32_t cnt[ORC_MAX_K];
  for (int k = 0; k < sc->K; ++k)
    cnt[k] = mesh_subset(sc, sc->obj_mesh[k], n_sub, sub, lists + (size_t)k * n_sub);
  int nth = sc->nthreads > 256 ? 256 : sc->nthreads;
  bf_t B[256];
  pthread_t th[256];
  for (int t = 0; t < nth; ++t) {
    memset(&B[t], 0, sizeof(bf_t));
    B[t].sc = sc; B[t].nsub = n_sub; B[t].tid = t; B[t].nth = nth; B[t].sub = sub;
    B[t].lists = lists; B[t].cnt = cnt;
  }
  if (nth == 1) bf_worker(&B[0]);
  else {
    for (int t = 0; t < nth; ++t) pthread_create(&th[t], NULL, bf_worker, &B[t]);
    for (int t = 0; t < nth; ++t) pthread_join(th[t], NULL);
  }
  free(lists);
  free(own);
  int have = 0;
  int64_t best = 0, nvalid = 0;
  int32_t key[2 * ORC_MAX_K];
  for (int t = 0; t < nth; ++t) {
    if (B[t].rc) return B[t].rc;
    nvalid += B[t].nvalid;
    if (!B[t].have) continue;
    if (!have || B[t].best < best || (B[t].best == best && cmp_key(sc->K, B[t].key, key) < 0)) {
      have = 1;
      best = B[t].best;
      memcpy(key, B[t].key, sizeof(int32_t) * 2 * sc->K);
    }
  }
  stats[0] = have ? best : -1;
  stats[1] = nvalid;
  stats[2] = 0;
  stats[3] = 0;
  if (!have) return 1;
  for (int k = 0; k < sc->K; ++k) {
    best_mesh[k] = key[2 * k];
    best_pose[k] = key[2 * k + 1];
  }
  return 0;
}
