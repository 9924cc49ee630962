// perch_internal.h -- device-side data layout shared by the kernels and the host
// code of libperch.so (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace perch {

// Sensor in float32 (the vertex stage works in float32; see vstage()).
constexpr int kMaxObjects = 16;  // objects of a scene / a state (PERCH_MAX_OBJECTS)

struct Cam {
  int W, H;
  float fx, fy, cx, cy;
  float M[12];     // cam_from_world, row-major [R | t]
  float Winv[12];  // world_from_cam (rounded from the FP64 inverse of M)
  float delta, delta2;
  float inv_fx, inv_fy;
  double dfx, dfy, dcx, dcy;  // the same intrinsics widened to FP64 (depth planes)
  double dinv_fx, dinv_fy;
  double dWinv[12];  // world_from_cam in FP64 (near-boundary volume decisions)
  double dM[12];     // cam_from_world widened to FP64 (the ICP association)
  double ddelta2;    // delta^2 in FP64 of the float32 delta (near-threshold distance decisions)
  // Margin of the float32 distance test |q - p|^2 <= delta^2 (see delta_margin):
  // tau(z) = t_lin z + t_0 + 4 (t_a z + t_s)^2 for a fixed point at depth z.
  float t_lin, t_0, t_a, t_s;
};

// Uniform voxel hash of the observed cloud I (camera frame).  Cell (i, j, k) holds
// the points p with floor(p * inv_cell) == (i, j, k); the open-addressing table
// maps a packed cell key to its (start, count) run in pts.
struct Hash {
  const unsigned long long* keys;  // table keys, kEmptyKey when free
  const int2* cells;               // (start, count) per table slot
  const float4* pts;               // camera-frame points grouped by cell
  int mask;                        // table size - 1 (power of two)
  float inv_cell;
  float qpad;  // query half-width: delta with a rounding margin
};

constexpr unsigned long long kEmptyKey = ~0ull;
constexpr unsigned kInfBits = 0x7f800000u;  // +inf as float bits (empty z-buffer)

// Mesh library, flattened.  range[m] = (v_off, nv, t_off, nt); frange[m] = (f_off, nf).
struct Meshes {
  const float4* verts;
  const int4* tris;
  const float4* planes;
  const int4* range;
  const int2* frange;
  // 4 per mesh (model frame): the centre c of the vertices' box, its half-extents
  // (rounded up, so c +- them holds every vertex), the half-extents of a box about
  // c inside the volume V(O) (every point of it at least 1e-9 m inside every face
  // plane; -1 when there is none), and a zero pad
  const float4* aabb;
};

// Materialised parent state R_j (Sec. III-A): composite depth as float bits
// (+inf = empty), and at the goal level the bitmap U of observed pixels outside
// every parent volume and unexplained by R_j, with |U|.
struct Parent {
  const unsigned* depth;
  const unsigned* ubits;
  const int* ucount;
  const unsigned* vbits;  // observed pixels inside V_j (overlap heuristic), or null
  int has_parent;
  int goal;
};

struct EvalParams {
  int tile_px;  // z-tile capacity (pixels) in LDS
  int halo;     // largest pixel-window radius over the observed cloud
  int max_nv;   // largest vertex count in the library
  float dwin;   // window radius in metres (delta with a rounding margin)
  int n_mesh;   // candidates with mesh_id outside [0, n_mesh) or pose_idx outside
  int n_poses;  // [0, n_poses) are rejected with status -4
  int radius_mode;  // dJ_r query: 0 exact pixel window, 1 voxel hash
  int vpack;        // vertex cache: 0 int2 per vertex, 1 packed 16 + 16 bits (large meshes)
  // V(O) decisions: a float32 object-frame point more than vbox outside the mesh's
  // vertex box is outside; inside it, face-plane values of that float32 point decide
  // when they clear vtau32, then those of the FP64 object-frame point rounded to
  // float32 when they clear vtau, else FP64 decides.
  float vbox, vtau, vtau32;
};

// Everything a successor evaluation reads about one scene.
struct SceneDev {
  Cam cam;
  Meshes M;
  const float4* poses;
  const float* obs;         // observed depth (H*W)
  const float2* obs_range;  // per pixel (min, max) observed depth over the window halo
  Hash hs;
  EvalParams ep;
};

// One materialised parent of a batch, in scene `scene` of the batch.
struct ParentDev {
  const unsigned* depth;
  const unsigned* ubits;
  const int* ucount;
  int has_parent;
  int goal;
  int scene;
  int pad;
};

// ---- launchers (perch_kernels.hip) ----
void launch_fill_u32(unsigned* p, unsigned v, size_t n, hipStream_t s);
void launch_fill_i32(int* p, int v, size_t n, hipStream_t s);
// hash build: counts, table insert, scan, scatter
void launch_hash_insert(const Cam& cam, const float* depth, unsigned long long* keys,
                        int* counts, int mask, float inv_cell, int* n_points, hipStream_t s);
void launch_scan_cells(const int* counts, int2* cells, int n_slots, hipStream_t s);
void launch_hash_scatter(const Cam& cam, const float* depth, const unsigned long long* keys,
                         const int2* cells, int* fill, float4* pts, int mask, float inv_cell,
                         hipStream_t s);
void launch_render_object(const Cam& cam, const Meshes& M, const float4* poses, int mesh,
                          int pose, int n_tris, unsigned* depth_bits, hipStream_t s);
// The composite of j objects (mesh_pose: host, 2 j ints; j <= kMaxObjects) in one
// launch; max_tris = the largest triangle count among them.
void launch_render_objects(const Cam& cam, const Meshes& M, const float4* poses,
                           const int* mesh_pose, int j, int max_tris, unsigned* depth_bits,
                           hipStream_t s);
void launch_parent_u(const Cam& cam, const Meshes& M, const float4* poses, const float* obs,
                     const int* par_mesh_pose, int j, const unsigned* depth_bits,
                     unsigned* ubits, int* ucount, const EvalParams& ep, hipStream_t s);
void launch_bits_to_float(const unsigned* bits, float* out, size_t n, hipStream_t s);
void launch_obs_range(const Cam& cam, const float* obs, float2* out, int R, hipStream_t s);
// gain (optional): per valid successor, observed points inside V(O) and outside
// V_j (par.vbits), the decrease of the overlap heuristic; -1 for invalid ones.
hipError_t launch_eval(int threads, const SceneDev& S, const Parent& par, const int2* cands,
                       int n, int* cost, int* status, int* comps, int* gain, size_t lds_bytes,
                       hipStream_t s);
// vbits |= observed pixels inside the union of the j objects' volumes
void launch_parent_v(const Cam& cam, const Meshes& M, const float4* poses, const float* obs,
                     const int* par_mesh_pose, int j, unsigned* vbits, const EvalParams& ep,
                     hipStream_t s);
// What a batch's tables hold (flags of prepare/launch_eval_batch): some scene
// answers dJ_r by the voxel hash (radius mode 1), some parent is at its scene's goal
// level, some parent has a parent (is below the root).
constexpr int kBatchHash = 1, kBatchGoal = 2, kBatchParent = 4;
// Raises the kernel's LDS limit and reports resident workgroups per CU (call
// before launch_eval_batch, outside any graph capture).
hipError_t prepare_eval_batch(int threads, int vpack, int flags, size_t lds_bytes,
                              int* blocks_per_cu);
// grid = number of persistent workgroups (clamped to n)
hipError_t launch_eval_batch(int threads, int vpack, int flags, const SceneDev* scenes,
                             const ParentDev* parents, int n_parents, const int4* items, int n,
                             int* counter, int* cost, int* status, int* comps, size_t lds_bytes,
                             int grid, hipStream_t s);

// ---- local ICP (Sec. IV-E) ----
constexpr int kIcpThreads = 512;
struct IcpArgs {
  int iters;
  float radius;       // association radius (metres)
  const double4* pn;  // per pixel: world point (w = 1 with a normal), unit normal (FP64)
  float4* arena;      // adjusted poses, one per candidate
  int base;           // pose index of arena[0]
  int retry;          // 1: only candidates whose status is -3 (footprint beyond the
                      // previous pass's tile); the others exit at once
};
// pn (2 double4 per pixel) from the observation for association radius `radius`
void launch_obs_normals(const Cam& cam, const float* obs, float radius, double4* pn,
                        hipStream_t s);
// kIcpThreads threads per candidate; lds = vertex cache (int2, when vertex_cache)
// + tile + rings
hipError_t launch_icp(const SceneDev& S, const Parent& par, const int2* cands, int n,
                      const IcpArgs& ia, int2* out_obj, int* out_match, int* out_status,
                      bool vertex_cache, size_t lds, hipStream_t s);

// ---- learned search: device-side ranking of children (perch_select.hip) ----
constexpr int kMaxMeshes = 8;  // distinct meshes of one scene's object multiset (learned)
struct MeshMask {
  int allow[kMaxMeshes];  // 0: the mesh is placed already, its children rank last
};
// masked = pred, with +inf at u n_poses + b for every mesh position u < n_meshes
// with allow[u] == 0
void launch_mask_children(const float* pred, float* masked, int n_poses, int n_meshes,
                          MeshMask mask, hipStream_t s);
size_t select_temp_bytes(int n);
// Stable sort of n predicted costs with their indices (ascending; NaN last).
hipError_t sort_predictions(void* temp, size_t temp_bytes, const float* keys, float* keys_sorted,
                            const int* idx, int* idx_sorted, int n, hipStream_t s);
void launch_iota(int* idx, int n, hipStream_t s);
// cands[i] = (rest[id / n_poses], pose_ids[id % n_poses]) for id = idx_sorted[i], i < k
// One-workgroup top-k for small child counts: cands[0..k) = the children of the
// k smallest predictions (masked as above; ties by index), in that order, exactly
// what sorting and taking the first k gives.  False (nothing launched) when n or k
// exceed the limits below or k > n.
constexpr int kTopkMaxN = 8192;
constexpr int kTopkMaxK = 1024;
bool launch_select_topk(const float* pred, int n_poses, int n_meshes, MeshMask mask, int k,
                        const int* rest, const int* pose_ids, int2* cands, hipStream_t s);
// The same selection in two levels for more children: the number of kTopkMaxN-child
// chunks when their k candidates each fit one more selection (n > kTopkMaxN,
// k <= kTopkMaxK, chunks * k <= kTopkMaxN), else 0.  launch_select_topk2 then needs
// buf = chunks * k device entries.
int select_chunks(long n, int k);
void launch_select_topk2(const float* pred, int n_poses, int n_meshes, MeshMask mask, int k,
                         const int* rest, const int* pose_ids, int2* cands,
                         unsigned long long* buf, hipStream_t s);
void launch_child_cands(const int* idx_sorted, int k, const int* rest, int n_poses,
                        const int* pose_ids, int2* cands, hipStream_t s);
// Work items (slot, mesh, pose, 0) of a batched search step: items[i] = (slot,
// cands[i]) for i < k; or every (meshes.id[u], pose_ids[b]) child, mesh-major.
struct MeshList {
  int id[kMaxMeshes];
};
void launch_items_from_cands(const int2* cands, int k, int slot, int4* items, hipStream_t s);
void launch_items_all(int slot, const MeshList& meshes, int n_meshes, const int* pose_ids,
                      int n_poses, int4* items, hipStream_t s);

}  // namespace perch
