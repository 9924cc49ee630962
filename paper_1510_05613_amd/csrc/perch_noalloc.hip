// perch_noalloc.hip -- perch_eval_successors without device allocation.
//
// The successor kernels of perch_eval_successors read a materialised parent: the
// composite depth R_j, and at the goal level the set U of observed points outside
// every parent volume and unexplained by R_j (bitmap and count).  The context
// allocates those buffers on first use; this entry point keeps them in a
// fixed-size array in device global memory instead, so that callers that cannot
// allocate (code under stream capture, serving loops, harnesses that forbid
// hipMalloc) can evaluate successors.  Each GPU the library runs on holds its own
// copy of the array until the process ends; every call on one GPU shares it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "perch_ctx.h"

using namespace perch;

namespace {

// Largest image (pixels) the scratch array holds: 1,048,576 (e.g. 1024 x 1024,
// 1280 x 800): parent depth 4 MiB, U bitmap 128 KiB, |U| in the last 256 bytes.
constexpr size_t kMaxPixels = size_t(1) << 20;
constexpr size_t kDepthBytes = kMaxPixels * sizeof(unsigned);
constexpr size_t kUbitsBytes = (kMaxPixels / 32) * sizeof(unsigned);
constexpr size_t kScratchBytes = kDepthBytes + kUbitsBytes + 256;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` per device, taken once per device with that device
// current.  The array's name in host code is a host-side stand-in and is never
// passed to a kernel or a copy.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

perch_status scratch_for(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(PERCH_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != dev) return fail(PERCH_E_STATE, "device %d is not current (%d is)", dev, cur);
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(PERCH_E_HIP, "hipGetSymbolAddress returned no address");
    g_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_ptr[dev]);
  return PERCH_OK;
}

}  // namespace

extern "C" perch_status perch_eval_successors_noalloc(perch_ctx* c, const perch_object* parent,
                                                      int32_t j, const perch_object* cands_dev,
                                                      int32_t n, int32_t* cost_dev,
                                                      int32_t* status_dev, int32_t* comps_dev) {
  if (!c) return fail(PERCH_E_ARG, "null context");
  if (n < 0 || (n > 0 && (!cands_dev || !cost_dev || !status_dev)))
    return fail(PERCH_E_ARG, "bad successor arrays");
  const size_t npx = (size_t)c->cam.W * c->cam.H;
  if (npx > kMaxPixels)
    return fail(PERCH_E_UNSUPPORTED,
                "image of %zu pixels exceeds the allocation-free limit of %zu pixels", npx,
                kMaxPixels);
  if (!c->has_obs) return fail(PERCH_E_STATE, "perch_set_observation not called");
  if (c->P <= 0) return fail(PERCH_E_STATE, "perch_set_poses not called");
  const int K = (int)c->objects.size();
  if (K < 1) return fail(PERCH_E_STATE, "perch_set_objects not called");
  if (j < 0 || j >= K || (j > 0 && !parent)) return fail(PERCH_E_ARG, "bad parent (j=%d, K=%d)", j, K);
  // uploading the library allocates: it must have happened in an earlier call
  if (c->meshes_dirty)
    return fail(PERCH_E_STATE,
                "mesh library not uploaded (perch_render, perch_set_parent or "
                "perch_eval_successors upload it)");
  for (int k = 0; k < j; ++k)
    if (parent[k].mesh_id < 0 || parent[k].mesh_id >= (int)c->meshes.size() ||
        parent[k].pose_idx < 0 || parent[k].pose_idx >= c->n_poses())
      return fail(PERCH_E_ARG, "parent object out of range");
  if (c->n_cus == 0)
    HIP_TRY(hipDeviceGetAttribute(&c->n_cus, hipDeviceAttributeMultiprocessorCount, c->device));
  const int nt = c->launch_threads(n);
  const int tile = c->tile_for(nt);
  const size_t lds = eval_lds_bytes(c->max_nv, tile, nt);
  if (lds > 160 * 1024 - 256)
    return fail(PERCH_E_UNSUPPORTED, "LDS need %zu B exceeds the CU (max_nv=%d, tile=%d)", lds,
                c->max_nv, tile);
  unsigned char* base = nullptr;
  perch_status st = scratch_for(c->device, &base);
  if (st) return st;
  unsigned* depth = reinterpret_cast<unsigned*>(base);
  unsigned* ubits = reinterpret_cast<unsigned*>(base + kDepthBytes);
  int* ucount = reinterpret_cast<int*>(base + kDepthBytes + kUbitsBytes);
  const bool goal = j + 1 == K;
  // clears what must start empty (depth +inf; U and |U| at the goal level) with fill
  // kernels, then renders the parent and builds U
  st = materialise_into(c, parent, j, goal, depth, ubits, ucount, c->stream);
  if (st) return st;
  if (n == 0) return PERCH_OK;
  Parent par;
  par.depth = depth;
  par.ubits = ubits;
  par.ucount = ucount;
  par.vbits = nullptr;
  par.has_parent = j > 0;
  par.goal = goal;
  SceneDev S = c->scene_dev();
  S.ep.tile_px = tile;
  HIP_TRY(launch_eval(nt, S, par, reinterpret_cast<const int2*>(cands_dev), n, cost_dev,
                      status_dev, comps_dev, nullptr, lds, c->stream));
  return PERCH_OK;
}
