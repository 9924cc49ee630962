/*
 * perch.h -- C ABI of libperch.so: PERCH successor evaluation on AMD MI355X (gfx950).
 *
 * PERCH (Narayanan & Likhachev, arXiv:1510.05613) localises K known objects on a
 * table by searching the Monotone Scene Generation Tree (MSGT).  A tree state is a
 * set of placed objects O = (ID, x, y, theta) (Sec. III-A); a successor adds one
 * more object that must not occlude the scene rendered so far (Eq. 3); the edge
 * cost is the per-object explanation cost dJ_r + dJ_o (+ residual at the last
 * level) of Eq. (2)/(4), built on the point indicator of Eq. (1): a point is
 * unexplained by a cloud C iff its distance to every point of C exceeds delta.
 *
 * Conventions
 *   - Units: metres, radians.  World frame: table top is z = 0, z up.
 *   - Camera frame: x right, y down, z forward.  cam_from_world = [R | t] row-major
 *     3x4 float32, p_cam = R p_world + t (the known sensor pose, Sec. III).
 *   - Pixel (u, v) = (column, row); pixel centres at integer coordinates;
 *     u = fx X / Z + cx, v = fy Y / Z + cy.  Depth = camera Z.
 *   - Pose table row (x, y, cos theta, sin theta): model point m goes to
 *     (cos m_x - sin m_y + x, sin m_x + cos m_y + y, m_z).
 *   - Meshes are closed and convex, triangles counter-clockwise seen from outside,
 *     model frame resting on z = 0.  Their solid V(O) (Sec. III-A) is given as
 *     planes (n, d): inside iff n.p <= d for every plane.
 *   - A rendered cloud holds one point per covered pixel centre (front-facing
 *     triangles, vertices snapped to 1/256 px, top-left fill rule).
 *
 * Memory and streams
 *   - "host" pointers are read before the call returns; "device" pointers are
 *     borrowed, must live on the context's device, and are used in stream order
 *     on the context's HIP stream (asynchronously unless stated otherwise).
 *   - The library owns every buffer it allocates (observation, hash, meshes,
 *     pose table, parent buffers) and frees them in perch_destroy.
 *
 * Errors
 *   - Every call returns perch_status (0 = OK, < 0 = error); perch_last_error()
 *     gives a thread-local message.  No C++ exception crosses the ABI.  HIP
 *     failures map to PERCH_E_HIP with the HIP error string.
 *   - One thread may use a context at a time.
 */
#ifndef PERCH_H
#define PERCH_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PERCH_OK = 0,
  PERCH_E_ARG = -1,         /* bad argument (null, out of range, wrong size)        */
  PERCH_E_OOM = -2,         /* device allocation failed                              */
  PERCH_E_HIP = -3,         /* a HIP runtime call failed                             */
  PERCH_E_STATE = -4,       /* call order violated (e.g. eval before observation)    */
  PERCH_E_UNSUPPORTED = -5, /* input outside what the kernels handle                 */
  PERCH_E_BUDGET = -6       /* search budget exhausted; the incumbent is returned    */
} perch_status;

typedef struct perch_ctx perch_ctx;

/* An object state O = (ID, x, y, theta) of Sec. III-A, with (x, y, theta) given as
 * an index into the context's pose table. */
typedef struct {
  int32_t mesh_id;
  int32_t pose_idx;
} perch_object;

/* The sensor of the problem statement (Sec. III): intrinsics, 6-DoF pose and the
 * noise threshold delta of Eq. (1). */
typedef struct {
  int32_t width, height;    /* pixels                                               */
  float fx, fy, cx, cy;     /* pinhole intrinsics                                   */
  float cam_from_world[12]; /* row-major [R | t]                                    */
  float delta;              /* metres: explained iff distance <= delta              */
} perch_sensor;

/* Per-successor status values written by perch_eval_successors. */
#define PERCH_SUCC_VALID 1          /* R_j subset of R_{j+1} holds (Eq. 3)            */
#define PERCH_SUCC_INVALID 0        /* the new object occludes the parent scene        */
#define PERCH_SUCC_NEAR_PLANE -2    /* a vertex lies within 1 cm of the camera plane   */
#define PERCH_SUCC_TOO_WIDE -3      /* footprint wider than the configured z-tile      */
#define PERCH_SUCC_BAD_INPUT -4     /* mesh_id or pose_idx out of range                */

/* Creates a context on the current HIP device.  hip_stream: the hipStream_t all
 * work is ordered on (NULL = the null stream).  Synchronous. */
perch_status perch_create(const perch_sensor* sensor, void* hip_stream, perch_ctx** out);

/* Destroys the context and frees its device memory.  Synchronises its stream. */
void perch_destroy(perch_ctx* ctx);

/* Sets the observed depth image I of Sec. III (device, H*W float32 metres, 0 = no
 * return; the table and background already removed, as Sec. III assumes).  The
 * image is copied; the library back-projects it and builds the uniform voxel hash
 * used for the radius tests of Eq. (1).  Synchronous. */
perch_status perch_set_observation(perch_ctx* ctx, const float* depth_dev);

/* Adds (or replaces) mesh mesh_id of the model library (the 3D models of Sec. III).
 * All arrays are host memory: verts n_verts x 3, tris n_tris x 3 (0-based, local),
 * planes n_planes x 4.  Uploaded before the next evaluation.  mesh ids are dense
 * from 0. */
perch_status perch_add_mesh(perch_ctx* ctx, int32_t mesh_id, const float* verts,
                            int32_t n_verts, const int32_t* tris, int32_t n_tris,
                            const float* planes, int32_t n_planes);

/* Marks a mesh as rotationally symmetric about the vertical axis (Sec. IV-E: only
 * its (x, y) matters).  perch_search then tries it only at the first pose of the
 * pose list (table or subset, in order) at each distinct (x, y); not with the
 * learned search modes.  Identical objects need no flag: the object multiset
 * (perch_set_objects) lists the mesh id once per instance and the searches place
 * instances of one mesh as a set, not in every order. */
perch_status perch_set_symmetric(perch_ctx* ctx, int32_t mesh_id, int32_t symmetric);

/* Sets the discretised pose set (Sec. IV-E, the x/y/yaw grid): host, P x 4 rows
 * (x, y, cos theta, sin theta).  Empties the pose arena (perch_set_pose_arena). */
perch_status perch_set_poses(perch_ctx* ctx, const float* poses, int32_t P);

/* Reserves device room for `capacity` poses after the P grid poses: the arena
 * where perch_icp_children stores the poses it adjusts (indices P, P + 1, ...),
 * usable wherever a pose index is.  Empties the arena (earlier arena indices become
 * invalid) and forgets the materialised parent.  Synchronous. */
perch_status perch_set_pose_arena(perch_ctx* ctx, int32_t capacity);

/* Copies poses [first, first + n) of the table (grid, then arena) to host memory,
 * n x 4 floats (x, y, cos, sin).  Synchronous. */
perch_status perch_get_poses(perch_ctx* ctx, int32_t first, int32_t n, float* poses_host);

/* Most objects in a scene (and placed in a state). */
#define PERCH_MAX_OBJECTS 16

/* Sets the known multiset of K <= PERCH_MAX_OBJECTS mesh ids in the scene (Sec. III assumptions);
 * the goal level of the tree is K. */
perch_status perch_set_objects(perch_ctx* ctx, const int32_t* mesh_ids, int32_t K);

/* The hot path: evaluates n successors s' = s + cands[i] of the parent state
 * s = parent[0..j) (host array, j < K), i.e. Succ(s) membership (Eq. 3) and the
 * edge cost c(s, s') (Eq. 4).  cands_dev: device, n perch_object.  Outputs
 * (device, n int32 each): cost_dev (-1 unless valid), status_dev (PERCH_SUCC_*),
 * comps_dev (nullable, n x 5: silhouette pixels S, |dR|, dJ_r, dJ_o, residual;
 * all -1 unless the successor is valid).
 * The parent composite R_j (and, at the goal level, the set U of observed points
 * outside every parent volume and unexplained by R_j) is materialised first, on
 * the same stream.  Asynchronous. */
perch_status perch_eval_successors(perch_ctx* ctx, const perch_object* parent, int32_t j,
                                   const perch_object* cands_dev, int32_t n,
                                   int32_t* cost_dev, int32_t* status_dev,
                                   int32_t* comps_dev);

/* The same evaluation in two steps, for callers that evaluate the children of one
 * parent in several batches: perch_set_parent materialises R_j of parent[0..j)
 * (and U at the goal level); perch_eval_children evaluates successors of the
 * parent last set, with the outputs of perch_eval_successors.  Asynchronous. */
perch_status perch_set_parent(perch_ctx* ctx, const perch_object* parent, int32_t j);
perch_status perch_eval_children(perch_ctx* ctx, const perch_object* cands_dev, int32_t n,
                                 int32_t* cost_dev, int32_t* status_dev, int32_t* comps_dev);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc): perch_eval_successors with the
 * same arguments, outputs and kernels, but the parent composite R_j, the set U and
 * |U| live in a fixed device array of the library (one per GPU, held until the
 * process ends) instead of context buffers, and the call allocates nothing.
 * Limits: at most 1,048,576 pixels (W * H; PERCH_E_UNSUPPORTED beyond); the mesh
 * library must already be on the device (uploaded by an earlier perch_render,
 * perch_set_parent or perch_eval_successors; PERCH_E_STATE otherwise).  Every call
 * on one GPU shares the array: calls that overlap on one GPU (other streams or
 * threads) race and must be serialised by the caller.  The context's own parent
 * (perch_set_parent) is left as it was.  Asynchronous. */
perch_status perch_eval_successors_noalloc(perch_ctx* ctx, const perch_object* parent,
                                           int32_t j, const perch_object* cands_dev,
                                           int32_t n, int32_t* cost_dev, int32_t* status_dev,
                                           int32_t* comps_dev);

/* The paper's overlap heuristic (Sec. IV-C): h_overlap(s) = |I| - #{p in I : p in V_j},
 * the observed points outside the union V_j of the placed objects' volumes.  For
 * each successor of the parent last set, evaluates it as perch_eval_children does
 * (cost_dev, status_dev) and writes gain_dev[i] = #{p in I : p in V(O) and p not in
 * V_j}, so that h_overlap(child) = h_overlap(parent) - gain; -1 for a successor that
 * is not valid.  V(O) membership is decided as in exact arithmetic on the float32
 * inputs: float32 where a proven margin allows, FP64 otherwise.  gain_dev: device,
 * n int32.  Asynchronous. */
perch_status perch_overlap_gain(perch_ctx* ctx, const perch_object* cands_dev, int32_t n,
                                int32_t* cost_dev, int32_t* status_dev, int32_t* gain_dev);

/* Local ICP alignment (Sec. IV-E, compensating for discretization): for each
 * candidate (mesh, pose) of the parent last set, renders it, takes the part not
 * covered by the parent (dR) and runs `iters` ICP rounds against the observation:
 * each model point, moved by the motion so far, is paired with the observed point
 * at the pixel nearest its projection when that point has a surface normal (cross
 * product of its four pixel neighbours' differences, all observed and within
 * `radius`) and lies within `radius` metres (2 cm in the paper, Sec. V-B); one
 * point-to-plane step (Chen and Medioni) then solves for a rotation about the
 * vertical axis through the pairs' centroid and a table-plane translation (damped
 * 3 x 3 normal equations).  Fewer than 3 pairs end the rounds.  The adjusted pose
 * (the motion applied after the grid placement) goes to arena slot arena_used + i,
 * and adjusted_dev[i] = (mesh, P + arena_used + i) can be evaluated with
 * perch_eval_children.  status_dev: 1 aligned, 0 the candidate occludes the parent
 * (Eq. 3; grid pose kept), -2 vertex stage failed, -3 footprint larger than the
 * ICP tile, -4 candidate out of range; n_match_dev: pairs of the last round.
 * Candidates, outputs: device arrays of n.  PERCH_E_ARG when the arena lacks room
 * for n.  Asynchronous. */
perch_status perch_icp_children(perch_ctx* ctx, const perch_object* cands_dev, int32_t n,
                                int32_t iters, float radius, perch_object* adjusted_dev,
                                int32_t* n_match_dev, int32_t* status_dev);

/* Renders objects (host array objs[0..n)) to depth images (device output, float32,
 * +inf where uncovered): composite != 0 writes one H*W image holding the minimum
 * over the objects (the rendered scene R_n); composite == 0 writes n stand-alone
 * images.  Asynchronous. */
perch_status perch_render(perch_ctx* ctx, const perch_object* objs, int32_t n,
                          int32_t composite, float* depth_dev);

/* Tuning knobs of the successor kernel: threads per successor (64, 128, 256, 512
 * or 1024; until set, 512, and 1024 for launches of at most four successors per
 * compute unit while the z-tile is sized automatically), z-tile capacity in pixels (LDS; -1 = sized automatically
 * from the largest mesh so that two workgroups share a CU, the default), voxel cell
 * size in units of delta (>= 1), and the radius query behind dJ_r (0 = exact pixel
 * window over the observed depth, 1 = uniform voxel hash of the observed cloud).
 * Pass 0 (radius_mode: -1) to keep a value.  Results do not depend on them. */
perch_status perch_set_tuning(perch_ctx* ctx, int32_t threads, int32_t tile_px,
                              float cell_over_delta, int32_t radius_mode);

typedef struct {
  int32_t threads;        /* threads per successor                                   */
  int32_t tile_px;        /* z-tile pixels                                           */
  int32_t radius_mode;    /* 0 pixel window, 1 voxel hash                            */
  float cell_over_delta;  /* voxel cell size / delta (radius_mode 1)                 */
  float ms;               /* median time of the calibration batch                    */
} perch_tuning;

/* Autotuner: times every candidate setting of perch_set_tuning on the calibration
 * batch cands_dev[0..n) (device) under parent[0..j) (host), reps timed runs each,
 * checks that every setting reproduces the first one's outputs bit for bit, and
 * applies the fastest.  cache_path (nullable): JSON-lines cache keyed by device and
 * scene shape; a hit is applied without timing.  Synchronous. */
perch_status perch_autotune(perch_ctx* ctx, const perch_object* parent, int32_t j,
                            const perch_object* cands_dev, int32_t n, int32_t reps,
                            const char* cache_path, perch_tuning* best);

/* Observed point count |I| and the pixel window halo (host outputs). */
perch_status perch_get_info(perch_ctx* ctx, int32_t* n_points, int32_t* halo);

/* ---- batched evaluation across scenes and parents ---- */

/* A batch evaluates successors of many parents, possibly of different scenes
 * (contexts), in one persistent launch: workgroups pull (parent, mesh, pose) items
 * from an atomic queue, so meshes of very different sizes balance across the GPU.
 * The launch is captured once in a hipGraph and replayed while the work list and
 * outputs keep their addresses and size.  The contexts must stay alive and
 * unchanged while the batch uses them. */
typedef struct perch_batch perch_batch;

typedef struct {
  int32_t ctx;            /* index into the batch's contexts                       */
  int32_t j;              /* number of placed objects (j < K of that context)      */
  perch_object objs[PERCH_MAX_OBJECTS]; /* the parent state s = objs[0..j)         */
} perch_parent;

typedef struct {
  int32_t parent;         /* parent slot (index into the last perch_batch_set_parents) */
  int32_t mesh_id;
  int32_t pose_idx;
  int32_t reserved;
} perch_work;

/* hip_stream: the stream the batch orders its work on (NULL = null stream).
 * Synchronous. */
perch_status perch_batch_create(perch_ctx* const* ctxs, int32_t n_ctx, void* hip_stream,
                                perch_batch** out);
void perch_batch_destroy(perch_batch* b);
/* Materialises each parent (R_j, and U at its goal level) into its own slot
 * (host array).  Asynchronous. */
perch_status perch_batch_set_parents(perch_batch* b, const perch_parent* parents, int32_t n);
/* Evaluates n work items (device array) into cost/status/comps (device, as in
 * perch_eval_successors, indexed like the items).  Asynchronous. */
perch_status perch_batch_eval(perch_batch* b, const perch_work* items_dev, int32_t n,
                              int32_t* cost_dev, int32_t* status_dev, int32_t* comps_dev);
/* threads per workgroup (64/128/256/512, default 512), z-tile pixels (-1 = sized
 * automatically, the default), use_graph (0/1), persistent grid size (0 = one
 * workgroup per resident slot); 0 (use_graph, grid: -1) keeps a value. */
perch_status perch_batch_set_tuning(perch_batch* b, int32_t threads, int32_t tile_px,
                                    int32_t use_graph, int32_t grid);

typedef struct {
  int32_t threads;        /* threads per workgroup of the batched launch             */
  int32_t tile_px;        /* z-tile pixels                                           */
  int32_t radius_mode;    /* dJ_r query of every context: 0 pixel window, 1 voxel hash */
  float cell_over_delta;  /* voxel cell / delta of every context (radius_mode 1)     */
  float ms;               /* median time of the calibration launch with this setting */
  float default_ms;       /* the same for the setting in force before tuning (0 when */
                          /* taken from the cache)                                   */
} perch_batch_tuning;

/* Autotuner of the batched launch (the tile shapes and radius query of Sec. IV-E's
 * parallel successor generation): times each candidate setting (threads per
 * workgroup 512 / 256, z-tile sized automatically or 8,192 / 12,288 pixels, radius
 * query window or voxel hash with cells of 2 and 1 delta) on the calibration work
 * list items_dev[0..n) (device) over the parents last set, reps timed launches each
 * after a warm-up, checks that every setting reproduces the first one's costs and
 * statuses bit for bit, applies the fastest to the batch (and the radius query to
 * its contexts) and records it in the JSON-lines cache at cache_path (nullable)
 * keyed by device, contexts and work shape; a cache hit is applied without timing.
 * Needs perch_batch_set_parents first (PERCH_E_STATE).  Synchronous. */
perch_status perch_batch_autotune(perch_batch* b, const perch_work* items_dev, int32_t n,
                                  int32_t reps, const char* cache_path,
                                  perch_batch_tuning* best);

/* ---- learned successor-cost network (an inadmissible heuristic, Sec. IV-C) ---- */

/* A small CNN predicting log(1 + c(s, s')) of a successor from a 64 x 64 x 2 depth
 * crop (observed depth, parent composite) centred on the candidate's table point,
 * the candidate's mesh and its yaw: 4 x (3x3 conv, 32 channels, ReLU; strides 1, 2,
 * 2, 2), mean pooling of the 8 x 8 map and of its centre, a 16-d mesh embedding,
 * and a 64-unit head.  Convolutions run on bfloat16 MFMA with FP32 accumulation;
 * parameters are FP32 masters trained with Adam.  Parameters are one flat FP32
 * array in the order cW0 cb0 cW1 cb1 cW2 cb2 cW3 cb3 emb hW1 hb1 hw2 hb2 (conv
 * weights [32][(ky*3 + kx)*C_in + ci], C_in = 2 then 32; emb [n_mesh][16]; hW1
 * [64][82] over [pooled 64, embedding 16, cos, sin]). */
typedef struct perch_cnn perch_cnn;

typedef struct {
  int32_t crop;      /* crop index within the batch */
  int32_t mesh_id;
  float cos_yaw, sin_yaw;
} perch_cnn_pair;

/* max_crops / max_pairs: largest batch (device memory is sized for it).
 * Parameters start at zero: set them before use.  Synchronous. */
perch_status perch_cnn_create(int32_t n_mesh, int32_t max_crops, int32_t max_pairs,
                              void* hip_stream, perch_cnn** out);
void perch_cnn_destroy(perch_cnn* net);
int64_t perch_cnn_param_count(const perch_cnn* net);
/* The learned search's crops for this network sample every `step` pixels (1..64;
 * default 1): a network trained on crops of step s must be searched with step s. */
perch_status perch_cnn_set_crop_step(perch_cnn* net, int32_t step);
/* host FP32 parameters in / out (set also resets the Adam state).  Synchronous. */
perch_status perch_cnn_set_params(perch_cnn* net, const float* params, int64_t n);
perch_status perch_cnn_get_params(perch_cnn* net, float* params, int64_t n);
/* Crops of the context's current parent (perch_set_parent) for n table points
 * xy (host, n x 2 metres): device output n x 64 x 64 x 2 bfloat16 (NHWC, 16-byte
 * aligned: PERCH_E_ARG otherwise).  Synchronous. */
perch_status perch_cnn_crops(perch_ctx* ctx, const float* xy, int32_t n, uint16_t* crops_dev);
/* Predictions (device, n_pairs floats) of log(1 + cost); a pair whose crop or
 * mesh index is out of range gets NaN (and is ignored by training).  crops_dev
 * must be 16-byte aligned here and in the training calls (PERCH_E_ARG otherwise).
 * Asynchronous on the network's stream. */
perch_status perch_cnn_predict(perch_cnn* net, const uint16_t* crops_dev, int32_t n_crops,
                               const perch_cnn_pair* pairs_dev, int32_t n_pairs, float* pred_dev);
/* perch_cnn_predict's predictions for the crops perch_cnn_crops_step(ctx, xy, n,
 * the network's crop step) would make, without materialising them: the network's
 * first kernel samples the context's observation and current parent composite
 * itself (the values are bit-identical).  Runs on the context's stream.
 * Synchronous. */
perch_status perch_cnn_predict_scene(perch_cnn* net, perch_ctx* ctx, const float* xy, int32_t n,
                                     const perch_cnn_pair* pairs_dev, int32_t n_pairs,
                                     float* pred_dev);
/* The learned search's ranking step (Sec. IV-C: only the children the learned
 * heuristic ranks best enter the inadmissible queue).  pred_dev (device, read
 * only): n_meshes x n_poses predictions, child u * n_poses + b = mesh position u,
 * pose position b.  Writes to out_dev (device, k entries) {mesh_ids_dev[u],
 * pose_ids_dev[b]} of the k children with the smallest prediction, in increasing
 * prediction, equal predictions (-0 equal to +0) in increasing child index: the
 * first k of a stable sort.  Children of a mesh position u with allow_host[u] == 0
 * rank as +inf.  Needs 1 <= n_meshes <= 8 and 1 <= k <= n_meshes * n_poses.  Up
 * to 8192 children and k <= 1024 one workgroup selects them; beyond 8192 children,
 * while the 8192-child chunks' k candidates number at most 8192, each chunk's
 * workgroup selects its k best and one more workgroup merges them; otherwise a
 * device radix sort runs.  Both use temporary memory the context keeps.
 * Synchronous on the context's stream. */
perch_status perch_rank_children(perch_ctx* ctx, const float* pred_dev, int32_t n_poses,
                                 int32_t n_meshes, const int32_t* allow_host, int32_t k,
                                 const int32_t* mesh_ids_dev, const int32_t* pose_ids_dev,
                                 perch_object* out_dev);
/* One Adam step on the mean squared error against target_dev (device, log(1 +
 * cost)); loss_host (nullable) receives the batch loss before the step (then the
 * call is synchronous). */
perch_status perch_cnn_train_step(perch_cnn* net, const uint16_t* crops_dev, int32_t n_crops,
                                  const perch_cnn_pair* pairs_dev, const float* target_dev,
                                  int32_t n_pairs, float lr, float* loss_host);
/* Loss and gradients (host, perch_cnn_param_count floats) without a step.
 * Synchronous. */
perch_status perch_cnn_gradients(perch_cnn* net, const uint16_t* crops_dev, int32_t n_crops,
                                 const perch_cnn_pair* pairs_dev, const float* target_dev,
                                 int32_t n_pairs, float* grads_host, float* loss_host);

/* ---- tree search (Alg. 1: ComputePath over the implicit MSGT) ---- */

#define PERCH_SEARCH_EXHAUSTIVE 0 /* enumerate the whole tree, argmin (cost, key)        */
#define PERCH_SEARCH_UCS 1        /* best-first on g with duplicate detection (w = 1)    */
#define PERCH_SEARCH_FOCAL 2      /* anchor g-queue + depth-first inadmissible queue,    */
                                  /* goal accepted when g <= w * min g (Theorem 2)       */
#define PERCH_SEARCH_LEARNED 3    /* FOCAL whose inadmissible queue only receives the    */
                                  /* top-k children ranked by the learned network; the   */
                                  /* rest wait, keyed at g(parent), in the anchor queue  */
#define PERCH_SEARCH_MHA 4        /* Focal-MHA* with the paper's h_depth and h_overlap  */
                                  /* (Sec. IV-C) as two inadmissible queues, round robin */
#define PERCH_SEARCH_LEARNED_MHA 5 /* LEARNED with h_overlap as a second inadmissible    */
                                  /* queue over the children it evaluates               */

/* A discriminative pose estimate O' of one object (Sec. IV-C: e.g. from a feature-
 * or learning-based detector), for the pose-prior heuristic. */
typedef struct {
  int32_t mesh_id;
  float x, y, theta;           /* table-plane position (m) and yaw (rad)               */
} perch_pose_prior;

typedef struct {
  int32_t mode;                /* PERCH_SEARCH_*                                        */
  float w;                     /* suboptimality bound for FOCAL (>= 1)                  */
  int32_t anytime;             /* FOCAL: keep searching until the incumbent is optimal  */
  double budget_s;             /* wall-clock budget in seconds, 0 = none                */
  int64_t budget_expansions;   /* 0 = none                                              */
  const int32_t* pose_subset;  /* host; NULL = every pose of the table                  */
  int32_t n_pose_subset;
  perch_cnn* cnn;              /* LEARNED(_MHA): the network (created with capacity    */
                               /* for one crop per pose cell and one pair per child)   */
  int32_t topk;                /* LEARNED: children evaluated exactly per expansion    */
  int32_t icp_iters;           /* UCS/FOCAL/MHA: > 0 aligns every child by local ICP   */
                               /* (perch_icp_children) before its edge cost is taken;  */
                               /* the search empties the pose arena first and stops    */
                               /* as on a spent budget when it has no room for the     */
                               /* next expansion's children                            */
  float icp_radius;            /* ICP association radius in metres (0: 0.02)           */
  const perch_pose_prior* priors; /* MHA: pose estimates (host), n_priors > 0 adds a    */
  int32_t n_priors;            /* third inadmissible queue on h_prior(s) = sum over the */
                               /* placed objects of the distance to the nearest estimate*/
                               /* of the same mesh (metres + prior_rad_m per radian of  */
                               /* yaw, yaw ignored for symmetric meshes), plus          */
                               /* prior_slot_m per object still to place (Sec. IV-C)    */
  float prior_rad_m;           /* 0: 0.05 m per radian                                 */
  float prior_slot_m;          /* 0: 0.1 m                                             */
  int32_t batch;               /* LEARNED: states expanded per step (<= 1: one).  With */
                               /* B > 1 the search picks up to B states by its usual   */
                               /* rule, runs the network for all of them, and evaluates*/
                               /* every chosen child (and every popped lazy block) in  */
                               /* one persistent batched launch with one host          */
                               /* synchronisation; the network needs capacity for B    */
                               /* crops per pose cell and B pairs per child            */
} perch_search_opts;

#define PERCH_TRACE 64 /* entries of a search's anytime trace */

typedef struct {
  perch_object objs[PERCH_MAX_OBJECTS]; /* the goal, in insertion order (valid)      */
  int32_t K;
  int32_t found;               /* 1 if a goal was reached                               */
  int64_t cost;                /* sum of edge costs (Eq. 2)                             */
  int32_t edge_cost[PERCH_MAX_OBJECTS]; /* c(s_i, s_{i+1}) along the path          */
  int64_t n_expanded, n_evaluated, n_invalid;
  double t_total_s;            /* wall time of the call                                 */
  double t_best_s;             /* wall time until the returned cost was first reached   */
  int64_t lower_bound;         /* min g over the open list at exit (UCS/FOCAL)          */
  int64_t n_evaluated_best;    /* successors evaluated when the returned cost was first */
                               /* reached (a deterministic time-to-best-scene)          */
  int64_t n_merged;            /* ICP: valid children dropped because a sibling of the  */
                               /* same mesh was aligned into the same 1 mm x 1 mm x 0.5 */
                               /* degree cell at no higher cost                         */
  int32_t n_trace;             /* entries of the anytime trace below (<= 64)            */
  double trace_t[PERCH_TRACE]; /* seconds since the call: whenever the incumbent cost    */
  int64_t trace_cost[PERCH_TRACE]; /* improves, and every 0.25 s: incumbent cost (-1 =  */
  int64_t trace_lb[PERCH_TRACE];   /* none yet) and the anchor's lower bound min g      */
} perch_result;

/* ---- per-object pose regressor (discriminative pose priors, Sec. IV-C) ---- */

/* The estimator behind the pose-prior heuristic: Sec. IV-C lists, as a second kind
 * of inadmissible guidance, how far a state's objects lie from the poses a
 * discriminative estimator proposes.  The network has the successor-cost
 * network's convolution trunk (own weights) on 64 x 64 x 2 crops around anchor
 * points of the table, a 16-d mesh embedding and a 64-unit head with 3 + n_yaw
 * outputs per (crop, mesh) pair: objectness logit, offset (dx, dy) of the object
 * from the anchor in units of the anchor spacing, logits of the n_yaw yaw bins
 * (yaw 2 pi k / n_yaw).  Loss per pair: log(1 + e^s) - label s + label (10 |offset
 * error|^2 + cross-entropy of the yaw logits against a target spread evenly over
 * the bins that are congruent to the true one modulo the mesh's symmetry period);
 * the batch loss is the mean.  Parameters: one flat FP32 array cW0 cb0 cW1 cb1 cW2
 * cb2 cW3 cb3 (as perch_cnn) emb [n_mesh][16] W1 [64][80] (over [pooled 64,
 * embedding 16]) b1 [64] W2 [3 + n_yaw][64] b2 [3 + n_yaw]. */
typedef struct perch_posenet perch_posenet;

typedef struct {
  int32_t crop;      /* crop index within the batch */
  int32_t mesh_id;
} perch_posenet_pair;

typedef struct {
  float label;       /* 1: the object stands in this crop's anchor cell, else 0      */
  float dx, dy;      /* its offset from the anchor / spacing (used when label = 1)  */
  float yaw_bin;     /* true yaw bin (an integer value)                             */
  float period;      /* bins between yaws the mesh's symmetry makes equal: a       */
                     /* divisor of n_yaw (n_yaw: one bin, 1: every bin)            */
} perch_posenet_target;

/* 1 <= n_yaw <= 32.  Parameters start at zero: set them before use.  Synchronous. */
perch_status perch_posenet_create(int32_t n_mesh, int32_t n_yaw, int32_t max_crops,
                                  int32_t max_pairs, void* hip_stream, perch_posenet** out);
void perch_posenet_destroy(perch_posenet* net);
int64_t perch_posenet_param_count(const perch_posenet* net);
/* host FP32 parameters in / out (set also resets the Adam state).  Synchronous. */
perch_status perch_posenet_set_params(perch_posenet* net, const float* params, int64_t n);
perch_status perch_posenet_get_params(perch_posenet* net, float* params, int64_t n);
/* Crops as perch_cnn_crops, sampling every `step` pixels (step >= 1: the crop
 * spans 64 step pixels).  Synchronous. */
perch_status perch_cnn_crops_step(perch_ctx* ctx, const float* xy, int32_t n, int32_t step,
                                  uint16_t* crops_dev);
/* Raw outputs (device, n_pairs x (3 + n_yaw) floats); NaN rows for pairs whose
 * crop or mesh index is out of range.  crops_dev must be 16-byte aligned here, in
 * the training calls and in perch_posenet_estimate (PERCH_E_ARG otherwise).
 * Asynchronous on the network's stream. */
perch_status perch_posenet_predict(perch_posenet* net, const uint16_t* crops_dev,
                                   int32_t n_crops, const perch_posenet_pair* pairs_dev,
                                   int32_t n_pairs, float* out_dev);
/* One Adam step on the mean loss against target_dev (device, n_pairs entries);
 * loss_host (nullable) receives the batch loss before the step (then the call is
 * synchronous). */
perch_status perch_posenet_train_step(perch_posenet* net, const uint16_t* crops_dev,
                                      int32_t n_crops, const perch_posenet_pair* pairs_dev,
                                      const perch_posenet_target* target_dev, int32_t n_pairs,
                                      float lr, float* loss_host);
/* Loss and gradients (host, perch_posenet_param_count floats) without a step.
 * Synchronous. */
perch_status perch_posenet_gradients(perch_posenet* net, const uint16_t* crops_dev,
                                     int32_t n_crops, const perch_posenet_pair* pairs_dev,
                                     const perch_posenet_target* target_dev, int32_t n_pairs,
                                     float* grads_host, float* loss_host);
/* Pose estimates O' from crops_dev (device, one crop per anchor, n_anchors of them
 * at anchor_xy_host, n_anchors x 2 metres): for mesh mesh_ids_host[u] (u <
 * n_meshes), counts_host[u] estimates, picked by decreasing objectness (ties: the
 * lower anchor) among anchors at least nms_m from the mesh's earlier picks, each
 * decoded to (x, y) = anchor + spacing (dx, dy) and the yaw of its largest yaw
 * logit.  Writes them to out_host in query order (at most max_out; *n_out = the
 * number written; a mesh with fewer free anchors than its count gets fewer).
 * Needs n_anchors <= max_crops and n_anchors * n_meshes <= max_pairs, counts
 * 0..64.  Synchronous. */
perch_status perch_posenet_estimate(perch_posenet* net, const uint16_t* crops_dev,
                                    int32_t n_anchors, const float* anchor_xy_host, float spacing,
                                    float nms_m, const int32_t* mesh_ids_host,
                                    const int32_t* counts_host, int32_t n_meshes,
                                    perch_pose_prior* out_host, int32_t max_out, int32_t* n_out);

/* Runs the tree search of Alg. 1 on the context's scene: root = empty state, goal =
 * all K objects placed, successors and edge costs from perch_set_parent /
 * perch_eval_children on the GPU (one launch per expansion).  Synchronous.
 * Returns PERCH_E_BUDGET (with the incumbent in *out) when a budget runs out. */
perch_status perch_search(perch_ctx* ctx, const perch_search_opts* opts, perch_result* out);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* perch_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
