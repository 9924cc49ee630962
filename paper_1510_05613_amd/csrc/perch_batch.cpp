// perch_batch.cpp -- batched successor evaluation across scenes and parents
// (arXiv:1510.05613 Sec. IV-E: successor generation is embarrassingly parallel).
//
// The paper farms successors out to CPU processes; here every successor of every
// parent of every scene in a batch goes into one persistent launch.  Parents are
// materialised into slots of their own; the kernel reads a scene table and a
// parent table from device memory and pulls (parent, mesh, pose) items from an
// atomic counter.  The launch (counter reset + persistent kernel) is captured in
// a hipGraph on a private stream and replayed on the caller's stream.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <string>
#include <vector>

#include "perch_ctx.h"

using namespace perch;

struct perch_batch {
  std::vector<perch_ctx*> ctxs;
  hipStream_t stream = nullptr;   // caller's stream
  hipStream_t capture = nullptr;  // private stream used only to capture graphs
  DevBuf scenes, parents, slot_depth, slot_ubits, slot_ucount, counter;
  int n_parents = 0;
  int flags = 0;  // kBatchHash | kBatchGoal | kBatchParent over the current tables
  int table_tile = -1;  // z-tile the uploaded scene table carries (-1: none uploaded)
  size_t npx_max = 0;
  int threads = 512;
  int tile_px = 0;  // 0 = sized automatically (auto_tile_px)
  int use_graph = 1;
  int grid = 0;
  // graph cache
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* g_items = nullptr;
  int g_n = -1;
  const void *g_cost = nullptr, *g_status = nullptr, *g_comps = nullptr;
  int g_threads = 0, g_tile = 0, g_grid = 0, g_parents = -1, g_flags = -1;
  const void* g_ptab = nullptr;

  std::vector<SceneDev> h_scenes;  // host copy of the scene table (kept: copies are async)
  int max_nv() const {
    int m = 0;
    for (perch_ctx* c : ctxs) m = std::max(m, c->max_nv);
    return m;
  }
  int tile() const { return tile_px > 0 ? tile_px : auto_tile_px(max_nv(), threads); }
  size_t lds_bytes() const { return eval_lds_bytes(max_nv(), tile(), threads); }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    g_items = nullptr;
  }
};

// Uploads the scene table with the tuning now in force (the z-tile the kernel
// places in LDS travels in each scene's parameters); *flags gets kBatchHash when a
// scene answers dJ_r by the voxel hash.  Asynchronous on the batch's stream.
static perch_status upload_scene_table(perch_batch* b, int* flags) {
  std::vector<SceneDev>& sd = b->h_scenes;
  sd.resize(b->ctxs.size());
  const int max_nv = b->max_nv();
  *flags = 0;
  for (size_t k = 0; k < b->ctxs.size(); ++k) {
    sd[k] = b->ctxs[k]->scene_dev();
    sd[k].ep.tile_px = b->tile();
    sd[k].ep.max_nv = max_nv;
    sd[k].ep.vpack = vertex_cache_packed(max_nv);
    *flags |= sd[k].ep.radius_mode == 1 ? kBatchHash : 0;
  }
  HIP_TRY(hipMemcpyAsync(b->scenes.p, sd.data(), sizeof(SceneDev) * sd.size(),
                         hipMemcpyHostToDevice, b->stream));
  b->table_tile = b->tile();
  return PERCH_OK;
}

const unsigned* batch_slot_depth(const perch_batch* b, int slot) {
  return b->slot_depth.as<unsigned>() + (size_t)slot * b->npx_max;
}

extern "C" {

perch_status perch_batch_create(perch_ctx* const* ctxs, int32_t n_ctx, void* hip_stream,
                                perch_batch** out) {
  if (!ctxs || !out || n_ctx < 1) return fail(PERCH_E_ARG, "bad context list");
  *out = nullptr;
  for (int k = 0; k < n_ctx; ++k) {
    perch_ctx* c = ctxs[k];
    if (!c) return fail(PERCH_E_ARG, "null context %d", k);
    if (!c->has_obs || c->P <= 0 || c->objects.empty())
      return fail(PERCH_E_STATE, "context %d lacks observation, poses or objects", k);
    perch_status st = upload_meshes(c);
    if (st) return st;
  }
  perch_batch* b = new perch_batch();
  b->ctxs.assign(ctxs, ctxs + n_ctx);
  b->stream = static_cast<hipStream_t>(hip_stream);
  for (perch_ctx* c : b->ctxs) b->npx_max = std::max(b->npx_max, (size_t)c->cam.W * c->cam.H);
  hipError_t e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
  if (e == hipSuccess) e = b->counter.ensure(sizeof(int));
  if (e == hipSuccess) e = b->scenes.ensure(sizeof(SceneDev) * n_ctx);
  if (e != hipSuccess) {
    if (b->capture) (void)hipStreamDestroy(b->capture);
    b->counter.release();
    b->scenes.release();
    delete b;
    return fail(e == hipErrorOutOfMemory ? PERCH_E_OOM : PERCH_E_HIP, "batch setup: %s",
                hipGetErrorString(e));
  }
  *out = b;
  return PERCH_OK;
}

void perch_batch_destroy(perch_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  b->drop_graph();
  for (DevBuf* d : {&b->scenes, &b->parents, &b->slot_depth, &b->slot_ubits, &b->slot_ucount,
                    &b->counter})
    d->release();
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
}

perch_status perch_batch_set_tuning(perch_batch* b, int32_t threads, int32_t tile_px,
                                    int32_t use_graph, int32_t grid) {
  if (!b) return fail(PERCH_E_ARG, "null batch");
  if (threads && threads != 64 && threads != 128 && threads != 256 && threads != 512)
    return fail(PERCH_E_ARG, "threads must be 64, 128, 256 or 512");
  if (tile_px && tile_px != -1 && (tile_px < 256 || tile_px > 36864))
    return fail(PERCH_E_ARG, "bad tile_px");
  if (threads) b->threads = threads;
  if (tile_px) b->tile_px = tile_px < 0 ? 0 : tile_px;
  if (use_graph >= 0) b->use_graph = use_graph ? 1 : 0;
  if (grid >= 0) b->grid = grid;
  return PERCH_OK;
}

perch_status perch_batch_set_parents(perch_batch* b, const perch_parent* parents, int32_t n) {
  if (!b || n < 0 || (n > 0 && !parents)) return fail(PERCH_E_ARG, "bad parent list");
  for (int k = 0; k < n; ++k) {
    const perch_parent& p = parents[k];
    if (p.ctx < 0 || p.ctx >= (int)b->ctxs.size()) return fail(PERCH_E_ARG, "parent %d: bad ctx", k);
    perch_ctx* c = b->ctxs[p.ctx];
    const int K = (int)c->objects.size();
    if (p.j < 0 || p.j >= K) return fail(PERCH_E_ARG, "parent %d: j=%d with K=%d", k, p.j, K);
    for (int o = 0; o < p.j; ++o)
      if (p.objs[o].mesh_id < 0 || p.objs[o].mesh_id >= (int)c->meshes.size() ||
          p.objs[o].pose_idx < 0 || p.objs[o].pose_idx >= c->n_poses())
        return fail(PERCH_E_ARG, "parent %d: object %d out of range", k, o);
    if (c->meshes_dirty) return fail(PERCH_E_STATE, "context %d meshes changed", p.ctx);
  }
  // the previous evaluation may still read the slots
  HIP_TRY(hipStreamSynchronize(b->stream));
  const size_t words = (b->npx_max + 31) / 32;
  HIP_TRY(b->slot_depth.ensure(std::max<size_t>(1, n) * b->npx_max * sizeof(unsigned)));
  HIP_TRY(b->slot_ubits.ensure(std::max<size_t>(1, n) * words * sizeof(unsigned)));
  HIP_TRY(b->slot_ucount.ensure(std::max<size_t>(1, n) * sizeof(int)));
  HIP_TRY(b->parents.ensure(std::max<size_t>(1, n) * sizeof(ParentDev)));
  std::vector<ParentDev> pd(std::max(1, n));
  int flags = 0;
  for (int k = 0; k < n; ++k) {
    const perch_parent& p = parents[k];
    perch_ctx* c = b->ctxs[p.ctx];
    unsigned* depth = b->slot_depth.as<unsigned>() + (size_t)k * b->npx_max;
    unsigned* ubits = b->slot_ubits.as<unsigned>() + (size_t)k * words;
    int* ucount = b->slot_ucount.as<int>() + k;
    const bool goal = p.j + 1 == (int)c->objects.size();
    perch_status st = materialise_into(c, p.objs, p.j, goal, depth, ubits, ucount, b->stream);
    if (st) return st;
    pd[k].depth = depth;
    pd[k].ubits = ubits;
    pd[k].ucount = ucount;
    pd[k].has_parent = p.j > 0;
    pd[k].goal = goal;
    flags |= (goal ? kBatchGoal : 0) | (p.j > 0 ? kBatchParent : 0);
    pd[k].scene = p.ctx;
    pd[k].pad = 0;
  }
  HIP_TRY(hipMemcpyAsync(b->parents.p, pd.data(), sizeof(ParentDev) * pd.size(),
                         hipMemcpyHostToDevice, b->stream));
  int hash = 0;
  perch_status st = upload_scene_table(b, &hash);
  if (st) return st;
  // the host vectors die here: the copies must complete first
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->n_parents = n;
  b->flags = flags | hash;
  return PERCH_OK;
}

perch_status perch_batch_eval(perch_batch* b, const perch_work* items_dev, int32_t n,
                              int32_t* cost_dev, int32_t* status_dev, int32_t* comps_dev) {
  if (!b) return fail(PERCH_E_ARG, "null batch");
  if (n < 0 || (n > 0 && (!items_dev || !cost_dev || !status_dev)))
    return fail(PERCH_E_ARG, "bad work arrays");
  if (n == 0) return PERCH_OK;
  if (b->table_tile < 0) return fail(PERCH_E_STATE, "perch_batch_set_parents not called");
  const size_t lds = b->lds_bytes();
  if (lds > 160 * 1024 - 256) return fail(PERCH_E_UNSUPPORTED, "LDS need %zu B too large", lds);
  if (b->table_tile != b->tile()) {
    // the tuning changed the z-tile since the scene table was written: the kernel
    // must place its tile in the LDS this launch gives it
    int hash = 0;
    perch_status st = upload_scene_table(b, &hash);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(b->stream));  // the host table is reused by the next upload
  }
  // resolve the persistent grid and the LDS limit outside any capture
  int grid = b->grid;
  {
    int dev = 0, cus = 0, per_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(prepare_eval_batch(b->threads, vertex_cache_packed(b->max_nv()), b->flags, lds,
                               &per_cu));
    if (grid <= 0) grid = std::max(1, cus * std::max(1, per_cu));
  }
  const int4* items = reinterpret_cast<const int4*>(items_dev);
  const SceneDev* scenes = b->scenes.as<SceneDev>();
  const ParentDev* parents = b->parents.as<ParentDev>();
  if (!b->use_graph) {
    HIP_TRY(launch_eval_batch(b->threads, vertex_cache_packed(b->max_nv()), b->flags, scenes,
                              parents, b->n_parents, items, n, b->counter.as<int>(), cost_dev,
                              status_dev, comps_dev, lds, grid, b->stream));
    return PERCH_OK;
  }
  const bool same = b->exec && b->g_items == items_dev && b->g_n == n && b->g_cost == cost_dev &&
                    b->g_status == status_dev && b->g_comps == comps_dev &&
                    b->g_threads == b->threads && b->g_tile == b->tile() && b->g_grid == grid &&
                    b->g_parents == b->n_parents && b->g_ptab == b->parents.p &&
                    b->g_flags == b->flags;
  if (!same) {
    b->drop_graph();
    HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_eval_batch(b->threads, vertex_cache_packed(b->max_nv()), b->flags,
                                     scenes, parents, b->n_parents, items, n,
                                     b->counter.as<int>(), cost_dev, status_dev, comps_dev, lds,
                                     grid, b->capture);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->capture, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(PERCH_E_HIP, "graph capture failed: %s",
                  hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->g_items = items_dev;
    b->g_n = n;
    b->g_cost = cost_dev;
    b->g_status = status_dev;
    b->g_comps = comps_dev;
    b->g_threads = b->threads;
    b->g_tile = b->tile();
    b->g_grid = grid;
    b->g_parents = b->n_parents;
    b->g_ptab = b->parents.p;
    b->g_flags = b->flags;
  }
  HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  return PERCH_OK;
}

}  // extern "C"

namespace {

std::string batch_fingerprint(const perch_batch* b, int n) {
  int dev = 0;
  hipDeviceProp_t prop;
  std::memset(&prop, 0, sizeof(prop));
  if (hipGetDevice(&dev) == hipSuccess) (void)hipGetDeviceProperties(&prop, dev);
  long long tris = 0, px = 0;
  for (const perch_ctx* c : b->ctxs) {
    for (const HostMesh& m : c->meshes) tris += (long long)m.tris.size() / 3;
    px += (long long)c->cam.W * c->cam.H;
  }
  char buf[512];
  snprintf(buf, sizeof buf, "batch|%s/%d|c%zu|px%lld|t%lld|v%d|p%d|n%d", prop.gcnArchName,
           prop.multiProcessorCount, b->ctxs.size(), px, tris, b->max_nv(), b->n_parents, n);
  return buf;
}

bool batch_cache_lookup(const char* path, const std::string& key, perch_batch_tuning* t) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  const std::string tag = "\"key\": \"" + key + "\"";
  while (std::getline(f, line)) {
    if (line.find(tag) == std::string::npos) continue;
    perch_batch_tuning r{};
    const char* q = strstr(line.c_str(), "\"threads\":");
    if (!q || sscanf(q, "\"threads\": %d, \"tile_px\": %d, \"radius_mode\": %d, "
                        "\"cell_over_delta\": %f, \"ms\": %f",
                     &r.threads, &r.tile_px, &r.radius_mode, &r.cell_over_delta, &r.ms) != 5)
      continue;
    *t = r;  // the last matching line wins
    found = true;
  }
  return found;
}

void batch_cache_store(const char* path, const std::string& key, const perch_batch_tuning& t) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << "{\"key\": \"" << key << "\", \"threads\": " << t.threads << ", \"tile_px\": " << t.tile_px
    << ", \"radius_mode\": " << t.radius_mode << ", \"cell_over_delta\": " << t.cell_over_delta
    << ", \"ms\": " << t.ms << "}\n";
}

// Applies a radius query (and cell size) to every context of the batch and
// rewrites the scene table and the kernel flags to match.
perch_status batch_apply_radius(perch_batch* b, int mode, float cell) {
  for (perch_ctx* c : b->ctxs) {
    perch_status st = perch_set_tuning(c, 0, 0, cell, mode);
    if (st) return st;
  }
  int hash = 0;
  perch_status st = upload_scene_table(b, &hash);
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->flags = (b->flags & ~kBatchHash) | hash;
  return PERCH_OK;
}

}  // namespace

extern "C" perch_status perch_batch_autotune(perch_batch* b, const perch_work* items_dev,
                                             int32_t n, int32_t reps, const char* cache_path,
                                             perch_batch_tuning* best) {
  if (!b || !best || !items_dev || n <= 0 || reps < 1) return fail(PERCH_E_ARG, "bad arguments");
  if (b->table_tile < 0) return fail(PERCH_E_STATE, "perch_batch_set_parents not called");
  const std::string key = batch_fingerprint(b, n);
  perch_batch_tuning t{};
  if (batch_cache_lookup(cache_path, key, &t)) {
    perch_status st = batch_apply_radius(b, t.radius_mode, t.cell_over_delta);
    if (!st) st = perch_batch_set_tuning(b, t.threads, t.tile_px, -1, -1);
    if (st) return st;
    t.default_ms = 0.0f;
    *best = t;
    return PERCH_OK;
  }
  DevBuf out;
  HIP_TRY(out.ensure((size_t)n * 2 * sizeof(int32_t)));
  int32_t* cost = out.as<int32_t>();
  int32_t* status = cost + n;
  std::vector<int32_t> ref, got((size_t)n * 2);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  struct Cfg {
    int threads, tile, mode;
    float cell;
  };
  // the setting in force first (the default), then the candidates
  const perch_ctx* c0 = b->ctxs[0];
  const Cfg keep{b->threads, b->tile_px > 0 ? b->tile_px : -1, c0->radius_mode,
                 c0->cell_over_delta};
  std::vector<Cfg> cfgs{keep};
  for (int th : {512, 256})
    for (int tile : {-1, 8192, 12288}) {
      cfgs.push_back({th, tile, 0, keep.cell});
      cfgs.push_back({th, tile, 1, 2.0f});
      cfgs.push_back({th, tile, 1, 1.0f});
    }
  perch_batch_tuning bestt{};
  bestt.ms = 1e30f;
  float default_ms = 0.0f;
  perch_status err = PERCH_OK;
  for (size_t k = 0; k < cfgs.size() && !err; ++k) {
    const Cfg& g = cfgs[k];
    err = batch_apply_radius(b, g.mode, g.cell);
    if (!err) err = perch_batch_set_tuning(b, g.threads, g.tile, -1, -1);
    if (err) break;
    if (b->lds_bytes() > 160 * 1024 - 2304) continue;  // with the static LDS
    err = perch_batch_eval(b, items_dev, n, cost, status, nullptr);  // warm-up (graph capture)
    if (err) break;
    std::vector<float> ms;
    for (int r = 0; r < reps && !err; ++r) {
      if (hipEventRecord(e0, b->stream) != hipSuccess) err = fail(PERCH_E_HIP, "event record");
      if (!err) err = perch_batch_eval(b, items_dev, n, cost, status, nullptr);
      if (!err && hipEventRecord(e1, b->stream) != hipSuccess) err = fail(PERCH_E_HIP, "event");
      if (!err && hipEventSynchronize(e1) != hipSuccess) err = fail(PERCH_E_HIP, "event sync");
      float v = 0;
      if (!err && hipEventElapsedTime(&v, e0, e1) != hipSuccess) err = fail(PERCH_E_HIP, "timing");
      ms.push_back(v);
    }
    if (err) break;
    if (hipMemcpy(got.data(), cost, got.size() * sizeof(int32_t), hipMemcpyDeviceToHost) !=
        hipSuccess) {
      err = fail(PERCH_E_HIP, "copy of tuning outputs failed");
      break;
    }
    if (ref.empty()) {
      ref = got;
    } else if (ref != got) {
      err = fail(PERCH_E_STATE, "setting threads=%d tile=%d mode=%d cell=%.1f changed the results",
                 g.threads, g.tile, g.mode, g.cell);
      break;
    }
    std::sort(ms.begin(), ms.end());
    const float med = ms[ms.size() / 2];
    if (k == 0) default_ms = med;
    if (med < bestt.ms) bestt = perch_batch_tuning{g.threads, b->tile(), g.mode, g.cell, med, 0.0f};
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  out.release();
  if (err || bestt.ms >= 1e30f) {
    (void)batch_apply_radius(b, keep.mode, keep.cell);
    (void)perch_batch_set_tuning(b, keep.threads, keep.tile, -1, -1);
    return err ? err : fail(PERCH_E_UNSUPPORTED, "no tuning candidate fits the LDS");
  }
  perch_status st = batch_apply_radius(b, bestt.radius_mode, bestt.cell_over_delta);
  if (!st) st = perch_batch_set_tuning(b, bestt.threads, bestt.tile_px, -1, -1);
  if (st) return st;
  bestt.default_ms = default_ms;
  batch_cache_store(cache_path, key, bestt);
  *best = bestt;
  return PERCH_OK;
}
