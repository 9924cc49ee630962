/*
 * perch_oracle.h -- the CPU oracle's own C interface.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, scalar definition of
 * what PERCH's successor evaluation computes (Narayanan & Likhachev, "PERCH:
 * Perception via Search for Multi-Object Recognition and Localization",
 * arXiv:1510.05613).  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg may load it.  It shares no source with the GPU library.
 *
 * Units are metres and radians.  Pixel (u, v) = (column, row); pixel centres sit
 * at integer coordinates.  Depth is the camera Z coordinate.  Floating point is
 * FP64 except the vertex stage, whose IEEE float32 operation order is part of the
 * rasterisation rule (both implementations take the same integer coverage
 * decisions from it).
 */
#ifndef PERCH_ORACLE_H
#define PERCH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t width, height;       /* image size in pixels                                 */
  float fx, fy, cx, cy;        /* pinhole intrinsics; pixel centre (u,v) at integers   */
  float cam_from_world[12];    /* row-major 3x4 [R | t]: p_cam = R p_world + t         */
  float delta;                 /* explanation radius: explained iff distance <= delta  */
} orc_sensor;

typedef struct orc_scene orc_scene;

/* Creates a scene.  All arrays are copied.  depth_obs (H*W, metres, 0 = no return)
 * may be NULL for a render-only scene.  Mesh m owns vertices [v_off[m], v_off[m+1]),
 * triangles [t_off[m], t_off[m+1]) (indices local to the mesh, outward
 * counter-clockwise) and planes [f_off[m], f_off[m+1]) given as (n, d) with the
 * solid being {p : n.p <= d for every plane}.  poses is n_poses x (x, y, cos, sin).
 * obj_mesh lists the known multiset of K mesh ids.  Returns NULL on bad input. */
orc_scene* orc_create(const orc_sensor* sensor, const float* depth_obs,
                      int32_t n_mesh, const int32_t* v_off, const int32_t* t_off,
                      const int32_t* f_off, const float* verts, const int32_t* tris,
                      const float* planes, int32_t n_poses, const float* poses,
                      int32_t K, const int32_t* obj_mesh);
void orc_destroy(orc_scene* sc);

/* radius_mode 0: exact pixel-window search (default); 1: all-pairs search.
 * nthreads: worker threads used by orc_eval and the searches (>= 1). */
int orc_set_mode(orc_scene* sc, int32_t radius_mode, int32_t nthreads);
int32_t orc_num_points(const orc_scene* sc);

/* Vertex stage of one mesh under one pose: cam (V x 3 float32) and the snapped
 * fixed-point screen coordinates UV (V x 2 int32, 1/256 pixel units). */
int orc_vertex_stage(const orc_scene* sc, int32_t mesh, int32_t pose, float* cam,
                     int32_t* uv);

/* Renders each listed object alone into depth[k*H*W ...] (FP64, +inf = uncovered).
 * cull = 1 rasterises front-facing triangles only (the rule), 0 rasterises all. */
int orc_render_objects(const orc_scene* sc, int32_t n, const int32_t* mesh,
                       const int32_t* pose, int32_t cull, double* depth);

/* Edge costs c(s, s') of n successors s' = s + (cand_mesh[i], cand_pose[i]) of the
 * parent s = {(par_mesh[k], par_pose[k]) : k < j}.  Goal level iff j + 1 == K.
 * status[i] = 1 valid / 0 invalid (cost -1).  comps (n x 5, nullable):
 * S, |dR|, dJ_r, dJ_o, residual.  flags (n x 3, nullable): n_flag_delta,
 * n_flag_vol, flag_valid. */
int orc_eval(const orc_scene* sc, int32_t j, const int32_t* par_mesh,
             const int32_t* par_pose, int32_t n, const int32_t* cand_mesh,
             const int32_t* cand_pose, int32_t* status, int32_t* cost,
             int32_t* comps, int32_t* flags);

/* One-shot costs of a full assignment of K objects (Eq. 2 evaluated from the
 * frontmost-owner partition, and the raw J of the problem statement).
 * out[0] valid (occlusion digraph acyclic), out[1] J_tree, out[2] J_raw,
 * out[3] n_flag_delta, out[4] n_flag_vol, out[5] flag_valid (depth ties). */
/* The overlap heuristic of Sec. IV-C, h_overlap(s) = |I| - #{p in I : p in V_j}:
 * h_parent for the parent of j objects, h_child[c] for each child adding candidate
 * (cand_mesh[c], cand_pose[c]); flags[c] = points decided within 1e-6 m of a
 * volume boundary. */
int orc_overlap(const orc_scene* sc, int32_t j, const int32_t* par_mesh,
                const int32_t* par_pose, int32_t n, const int32_t* cand_mesh,
                const int32_t* cand_pose, int64_t* h_parent, int64_t* h_child,
                int32_t* flags);

/* One linearised point-to-plane step over n pairs (a_k, p_k) with unit normals
 * nrm_k at p_k (3 doubles each, world frame): the small table-plane motion (a
 * rotation about the vertical axis through the centroid of the a_k, then a
 * translation) minimising sum (n.(moved a - p))^2 to first order, damped by 1e-6
 * of the normal matrix's diagonal plus 1e-12.  out = (phi, tx, ty) of the same
 * motion written as a rotation about the world z axis, then a translation. */
int orc_icp_step(int32_t n, const double* a, const double* p, const double* nrm, double* out);

/* Local ICP (Sec. IV-E) of each candidate's non-occluded part under the parent
 * s = {(par_mesh[k], par_pose[k]) : k < j}: `iters` rounds of projective
 * association (observed point at the pixel nearest the moved model point, kept
 * when it has a surface normal and lies within `radius` metres) and a
 * point-to-plane step (orc_icp_step).  The normal of an observed point is the
 * cross product of the central differences of its four pixel neighbours, all
 * observed and within `radius` of it, turned towards the camera.  pose_out (n x 4): adjusted
 * (x, y, cos, sin); n_match: matches of the last association; status 1 aligned,
 * 0 the candidate occludes the parent (grid pose returned); flags: associations
 * decided within 1e-4 px of a rounding boundary or 1e-6 m of the radius (match
 * or normal neighbourhood), plus 1 for a parent depth tie. */
int orc_icp(const orc_scene* sc, int32_t j, const int32_t* par_mesh, const int32_t* par_pose,
            int32_t n, const int32_t* cand_mesh, const int32_t* cand_pose, int32_t iters,
            double radius, double* pose_out, int32_t* n_match, int32_t* status,
            int32_t* flags);

int orc_jtree(const orc_scene* sc, int32_t K, const int32_t* mesh,
              const int32_t* pose, int64_t* out);

/* Searches over the tree restricted to the listed poses (pose_sub, n_sub).
 * best_mesh/best_pose receive the goal in canonical order (sorted by
 * (mesh, pose)).  stats: [0] cost, [1] successor evaluations, [2] expansions,
 * [3] goals seen.  Return 0 on success, 1 when no goal exists. */
/* Marks mesh as rotationally symmetric about the vertical axis (Sec. IV-E): the
 * searches below then try it only at the first pose of the subset at each distinct
 * (x, y). */
int orc_set_symmetric(orc_scene* sc, int32_t mesh, int32_t symmetric);

int orc_search_exhaustive(const orc_scene* sc, int32_t n_sub, const int32_t* pose_sub,
                          int32_t* best_mesh, int32_t* best_pose, int64_t* stats);
int orc_search_ucs(const orc_scene* sc, int32_t n_sub, const int32_t* pose_sub,
                   int32_t* best_mesh, int32_t* best_pose, int64_t* stats);
int orc_bruteforce_joint(const orc_scene* sc, int32_t n_sub, const int32_t* pose_sub,
                         int32_t* best_mesh, int32_t* best_pose, int64_t* stats);

#ifdef __cplusplus
}
#endif
#endif
