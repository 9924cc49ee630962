// perch_ctx.h -- the context object behind the C ABI (internal to libperch.so).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include <string>
#include <vector>

#include "../../include/perch.h"
#include "perch_internal.h"

namespace perch {

// Device memory the library holds (all contexts, batches and networks of the
// process).  With the environment variable PERCH_DEVICE_MEM_CAP set to a byte
// count, an allocation that would take the total above it fails as out of memory
// (PERCH_E_OOM) without reaching the runtime: a budget for processes that share a
// GPU, and the way the error path is tested.
bool dev_mem_admit(size_t n);
void dev_mem_account(long long delta);

// A device allocation owned by the context.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    const size_t want = n ? n : 16;
    if (!dev_mem_admit(want)) return hipErrorOutOfMemory;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) {
      bytes = n;
      dev_mem_account((long long)want);
    } else {
      p = nullptr;
    }
    return e;
  }
  void release() {
    if (p) {
      (void)hipFree(p);
      dev_mem_account(-(long long)(bytes ? bytes : 16));
    }
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

struct HostMesh {
  std::vector<float> verts;
  std::vector<int32_t> tris;
  std::vector<float> planes;
  bool set = false;
};

// Page-locked host memory owned by the context (fast, truly asynchronous copies).
struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipHostMalloc(&p, n ? n : 16, hipHostMallocDefault);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

inline int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Float32 error margins of the observed-point volume test for one scene (the
// derivation is in perch_api.cpp): vbox for the float32 vertex-box pre-test, vtau
// for the float32 face-plane values of the FP64 object-frame point.
void vol_margins(const Cam& cam, float obs_zmax, float pose_xy_max, float mesh_rmax,
                 float mesh_wmax, float& vbox, float& vtau, float& vtau32);

// Records a message for perch_last_error() and returns st.
perch_status fail(perch_status st, const char* fmt, ...);

// The largest batch (crops, pairs) the network was created for (perch_cnn_api.cpp).
perch_status cnn_capacity(const perch_cnn* c, int* max_crops, int* max_pairs);
// Pixel step of the crops the learned search takes for network c (1: every pixel).
int cnn_crop_step(const perch_cnn* c);

// Runs the learned network (forward pass and head) on stream s, the context's
// stream in the learned search (perch_cnn_api.cpp).
perch_status cnn_predict_on(perch_cnn* c, const uint16_t* crops, int n_crops, const void* pairs,
                            int n_pairs, float* pred, hipStream_t s);
// The same predictions for crops sampled inside the network's first kernel from the
// context's observation and current parent composite, one per descriptor of
// desc_dev (device CropDesc array, the network's crop step), on stream s.
perch_status cnn_predict_scene_on(perch_cnn* c, perch_ctx* ctx, const void* desc_dev,
                                  int n_crops, const void* pairs, int n_pairs, float* pred,
                                  hipStream_t s);

}  // namespace perch

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return perch::fail(e_ == hipErrorOutOfMemory ? PERCH_E_OOM : PERCH_E_HIP, "%s: %s", \
                         #expr, hipGetErrorString(e_));                                 \
  } while (0)


// Meshes of up to this many vertices keep full int2 snapped vertices in LDS; the
// vertex cache of larger ones is packed into 16 + 16 bits relative to the
// footprint (half the LDS, a second pass over the vertices).
constexpr int kInt2CacheMaxVerts = 5120;
inline int vertex_cache_packed(int max_nv) { return max_nv > kInt2CacheMaxVerts ? 1 : 0; }

// Dynamic LDS of the successor kernel: the snapped-vertex cache, the z-tile and
// one 128-entry triangle queue per wave.
inline size_t eval_lds_bytes(int max_nv, int tile_px, int threads) {
  const size_t vb = vertex_cache_packed(max_nv) ? sizeof(unsigned) : 2 * sizeof(int);
  return (size_t)max_nv * vb + (size_t)tile_px * sizeof(unsigned) +
         (size_t)(threads / 64) * 128 * sizeof(unsigned);
}

// Dynamic LDS and z-tile of the ICP kernel: one workgroup per CU, an int2 vertex
// cache for meshes of at most kInt2CacheMaxVerts vertices (larger ones recompute
// their snapped vertices), the largest tile (a multiple of 256 pixels) left over;
// footprints larger than it are not aligned.
inline bool icp_vertex_cache(int max_nv) { return max_nv <= kInt2CacheMaxVerts; }
inline size_t icp_fixed_lds(int max_nv) {
  return (icp_vertex_cache(max_nv) ? (size_t)max_nv * 2 * sizeof(int) : 0) +
         (size_t)(perch::kIcpThreads / 64) * 128 * sizeof(unsigned);
}
inline int icp_tile_px(int max_nv, int per_cu = 1) {
  const long budget = 160L * 1024 / per_cu - 4096 - (long)icp_fixed_lds(max_nv);
  return budget < 4L * 1024 ? 0 : (int)((budget / 4) & ~255L);
}

// Largest z-tile (a multiple of 256 pixels, at most 36,864) that lets two
// workgroups share a CU's 160 KB of LDS (four for 256 threads or fewer), else one;
// rows that do not fit are processed in bands.
inline int auto_tile_px(int max_nv, int threads) {
  const long fixed = (long)eval_lds_bytes(max_nv, 0, threads) + 2048;  // + static LDS
  const int per_cu[3] = {threads <= 256 ? 4 : 2, 2, 1};
  for (int k = 0; k < 3; ++k) {
    const long budget = (160L * 1024) / per_cu[k] - 256 - fixed;
    if (budget >= 4L * 4096) return (int)std::min(36864L, (budget / 4) & ~255L);
  }
  return 1024;
}

struct perch_ctx {
  using DevBuf = perch::DevBuf;
  using HostMesh = perch::HostMesh;
  using PinnedBuf = perch::PinnedBuf;
  using Cam = perch::Cam;
  using Meshes = perch::Meshes;
  using Hash = perch::Hash;
  using EvalParams = perch::EvalParams;
  Cam cam;
  hipStream_t stream = nullptr;
  int device = 0;
  // model library
  std::vector<HostMesh> meshes;
  std::vector<uint8_t> symmetric;  // per mesh id: searched over (x, y) only
  bool meshes_dirty = true;
  int max_nv = 0;
  DevBuf verts, tris, planes, range, frange, aabb;
  // pose table (device, and a host copy of the grid for the search driver): the P
  // grid poses, then room for arena_cap poses adjusted by the local ICP, of which
  // the first arena_used are taken
  DevBuf poses;
  std::vector<float> h_poses;
  int P = 0;
  int arena_cap = 0, arena_used = 0;
  int n_poses() const { return P + arena_used; }
  // known objects
  std::vector<int32_t> objects;
  // observation and hash
  DevBuf obs, obs_range;
  bool has_obs = false;
  int n_points = 0;
  DevBuf h_keys, h_cells, h_pts, h_counts;
  // observed points with surface normals for the local ICP, for one radius
  DevBuf icp_pn;
  long obs_serial = 0, icp_pn_obs = -1;
  float icp_pn_radius = -1.0f;
  int h_mask = 0;
  float cell_over_delta = 2.0f;
  // parent buffers (parent_j = level of the materialised parent, -1 = none)
  DevBuf par_depth, par_ubits, par_ucount;
  // overlap heuristic: observed pixels inside V_j of the materialised parent,
  // computed on first use (vbits_for == parent_serial)
  DevBuf par_vbits;
  std::vector<perch_object> parent_objs;
  long parent_serial = 0, vbits_for = -1;
  int parent_j = -1;
  // crop descriptors of the learned heuristic
  DevBuf cnn_desc;
  // search scratch: candidate list and outputs of one expansion
  DevBuf s_cands, s_out, s_adj;
  // learned search: crop descriptors, pair table, ranking buffers (kept between calls)
  DevBuf learned_bufs[11];
  PinnedBuf s_hcands, s_hout, s_hposes;
  // learned search with several states per step: a batch over this context, its
  // work items, outputs and the replicated crop / pair / prediction buffers
  perch_batch* s_batch = nullptr;
  DevBuf s_items, s_bout, s_bcrops, s_bpairs, s_bpred, s_bcands;
  PinnedBuf s_hitems, s_hbout;
  // tuning (tile_px 0 = sized automatically, see auto_tile_px)
  int threads = 512;
  bool threads_auto = true;  // threads never set explicitly: small launches widen
  int n_cus = 0;             // compute units of the context's device (0 = not queried)
  int tile_px = 0;
  int radius_mode = 0;
  EvalParams ep{};

  // Threads per successor for a launch of n successors: with automatic tuning, a
  // launch of at most four successors per CU (a search's per-expansion launches)
  // gives each successor a whole CU's 1,024 threads, which shortens the launch (a
  // 12-object search: -20 %); larger launches keep two 512-thread workgroups per CU.
  int launch_threads(int n) const {
    return threads_auto && tile_px == 0 && n > 0 && n <= 4 * n_cus ? 1024 : threads;
  }
  int tile_for(int nt) const { return tile_px > 0 ? tile_px : auto_tile_px(max_nv, nt); }

  // extents behind the float32 decision margins of the volume test (vol_margins)
  float obs_zmax = 0.0f;     // largest observed depth
  float pose_xy_max = 0.0f;  // largest |x| + |y| over the pose grid
  float mesh_rmax = 0.0f;    // largest distance of a mesh's vertex-box corner from its origin
  float mesh_wmax = 0.0f;    // largest |d| over the face planes (n, d)

  // ep with the volume-test margins of this scene (see perch::vol_margins).
  EvalParams eval_params() const {
    EvalParams e = ep;
    perch::vol_margins(cam, obs_zmax, pose_xy_max, mesh_rmax, mesh_wmax, e.vbox, e.vtau,
                       e.vtau32);
    return e;
  }

  int tile() const { return tile_px > 0 ? tile_px : auto_tile_px(max_nv, threads); }
  size_t eval_lds() const { return eval_lds_bytes(max_nv, tile(), threads); }

  Meshes dev_meshes() const {
    Meshes M;
    M.verts = verts.as<float4>();
    M.tris = tris.as<int4>();
    M.planes = planes.as<float4>();
    M.range = range.as<int4>();
    M.frange = frange.as<int2>();
    M.aabb = aabb.as<float4>();
    return M;
  }
  // Scene view for the kernels, with the context's tuning.
  perch::SceneDev scene_dev() const {
    perch::SceneDev S;
    S.cam = cam;
    S.M = dev_meshes();
    S.poses = poses.as<float4>();
    S.obs = obs.as<float>();
    S.obs_range = obs_range.as<float2>();
    S.hs = dev_hash();
    S.ep = eval_params();
    S.ep.tile_px = tile();
    S.ep.max_nv = max_nv;
    S.ep.vpack = vertex_cache_packed(max_nv);
    S.ep.n_mesh = (int)meshes.size();
    S.ep.n_poses = n_poses();
    S.ep.radius_mode = radius_mode;
    return S;
  }
  Hash dev_hash() const {
    Hash h;
    h.keys = h_keys.as<unsigned long long>();
    h.cells = h_cells.as<int2>();
    h.pts = h_pts.as<float4>();
    h.mask = h_mask;
    const float delta = cam.delta;
    h.qpad = delta * 1.001f + 1e-6f;
    h.inv_cell = 1.0f / (cell_over_delta * h.qpad);
    return h;
  }
};

// The composite depth (float bits) of parent slot `slot` of a batch, valid after
// perch_batch_set_parents (perch_batch.cpp).
const unsigned* batch_slot_depth(const perch_batch* b, int slot);

// Shared with the batch and search code (perch_api.cpp).
perch_status upload_meshes(perch_ctx* c);
perch_status materialise_into(perch_ctx* c, const perch_object* parent, int j, bool goal,
                              unsigned* depth, unsigned* ubits, int* ucount, hipStream_t st);
// The learned search's ranking step: out[0..k) = the children of the k smallest
// predictions (pred[u n_poses + b]; mesh positions with mask.allow[u] == 0 last),
// ties in index order, as {mesh_ids[u], pose_ids[b]}.  One workgroup selects up to
// kTopkMaxN children; beyond, a radix sort in the context's learned buffers.
// Asynchronous on st.
perch_status rank_children(perch_ctx* c, const float* pred, int n_poses, int n_meshes,
                           const perch::MeshMask& mask, int k, const int* mesh_ids,
                           const int* pose_ids, int2* out, hipStream_t st);
