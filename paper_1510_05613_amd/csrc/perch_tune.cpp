// perch_tune.cpp -- autotuner for the successor kernel.
//
// Times every candidate setting (threads per successor, z-tile pixels, radius
// query of dJ_r and, for the voxel hash, its cell size) on a calibration batch of
// the caller's successors with HIP events, checks that each setting reproduces the
// first setting's outputs bit for bit (the settings change the schedule, never the
// result), applies the fastest to the context and records it in a JSON-lines cache
// keyed by device and scene shape.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "perch_ctx.h"

using namespace perch;

namespace {

std::string fingerprint(const perch_ctx* c, int j, int n) {
  int dev = 0;
  hipDeviceProp_t prop;
  std::memset(&prop, 0, sizeof(prop));
  if (hipGetDevice(&dev) == hipSuccess) (void)hipGetDeviceProperties(&prop, dev);
  long long tris = 0;
  for (const HostMesh& m : c->meshes) tris += (long long)m.tris.size() / 3;
  char buf[512];
  snprintf(buf, sizeof buf, "%s/%d|%dx%d|f%.1f|d%.4f|m%zu|t%lld|v%d|P%d|K%zu|j%d|n%d",
           prop.gcnArchName, prop.multiProcessorCount, c->cam.W, c->cam.H, c->cam.fx,
           c->cam.delta, c->meshes.size(), tris, c->max_nv, c->P, c->objects.size(), j, n);
  return buf;
}

bool cache_lookup(const char* path, const std::string& key, perch_tuning* t) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    const std::string tag = "\"key\": \"" + key + "\"";
    if (line.find(tag) == std::string::npos) continue;
    perch_tuning r{};
    const char* p = line.c_str();
    const char* q = strstr(p, "\"threads\":");
    if (!q || sscanf(q, "\"threads\": %d, \"tile_px\": %d, \"radius_mode\": %d, "
                        "\"cell_over_delta\": %f, \"ms\": %f",
                     &r.threads, &r.tile_px, &r.radius_mode, &r.cell_over_delta, &r.ms) != 5)
      continue;
    *t = r;  // the last matching line wins
    found = true;
  }
  return found;
}

void cache_store(const char* path, const std::string& key, const perch_tuning& t) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << "{\"key\": \"" << key << "\", \"threads\": " << t.threads << ", \"tile_px\": " << t.tile_px
    << ", \"radius_mode\": " << t.radius_mode << ", \"cell_over_delta\": " << t.cell_over_delta
    << ", \"ms\": " << t.ms << "}\n";
}

}  // namespace

extern "C" perch_status perch_autotune(perch_ctx* c, const perch_object* parent, int32_t j,
                                       const perch_object* cands_dev, int32_t n, int32_t reps,
                                       const char* cache_path, perch_tuning* best) {
  if (!c || !best || n <= 0 || !cands_dev || reps < 1) return fail(PERCH_E_ARG, "bad arguments");
  perch_status st = upload_meshes(c);
  if (st) return st;
  const std::string key = fingerprint(c, j, n);
  perch_tuning t{};
  if (cache_lookup(cache_path, key, &t)) {
    st = perch_set_tuning(c, t.threads, t.tile_px, t.cell_over_delta, t.radius_mode);
    if (st) return st;
    *best = t;
    return PERCH_OK;
  }
  st = perch_set_parent(c, parent, j);
  if (st) return st;
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
  std::vector<Cfg> cfgs;
  // tile -1: sized automatically for the thread count
  for (int th : {512, 256})
    for (int tile : {-1, 4096, 8192, 12288}) {
      cfgs.push_back({th, tile, 0, 2.0f});
      cfgs.push_back({th, tile, 1, 2.0f});
    }
  cfgs.push_back({512, -1, 1, 1.0f});
  const int keep_threads = c->threads, keep_tile = c->tile_px, keep_mode = c->radius_mode;
  const bool keep_auto = c->threads_auto;
  const float keep_cell = c->cell_over_delta;
  perch_tuning bestt{};
  bestt.ms = 1e30f;
  perch_status err = PERCH_OK;
  for (const Cfg& g : cfgs) {
    err = perch_set_tuning(c, g.threads, g.tile, g.cell, g.mode);
    if (err) break;
    // the cell change rebuilt the hash (and synchronised): materialise the parent again
    err = perch_set_parent(c, parent, j);
    if (err) break;
    if (c->eval_lds() > 160 * 1024 - 2304) continue;  // with the static LDS
    err = perch_eval_children(c, cands_dev, n, cost, status, nullptr);  // warm-up
    if (err) break;
    std::vector<float> ms;
    for (int r = 0; r < reps && !err; ++r) {
      if (hipEventRecord(e0, c->stream) != hipSuccess) err = fail(PERCH_E_HIP, "event record");
      if (!err) err = perch_eval_children(c, cands_dev, n, cost, status, nullptr);
      if (!err && hipEventRecord(e1, c->stream) != hipSuccess) err = fail(PERCH_E_HIP, "event");
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
    if (med < bestt.ms) bestt = perch_tuning{g.threads, c->tile(), g.mode, g.cell, med};
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  out.release();
  if (err || bestt.ms >= 1e30f) {
    (void)perch_set_tuning(c, keep_threads, keep_tile > 0 ? keep_tile : -1, keep_cell, keep_mode);
    c->threads_auto = keep_auto;
    return err ? err : fail(PERCH_E_UNSUPPORTED, "no tuning candidate fits the LDS");
  }
  st = perch_set_tuning(c, bestt.threads, bestt.tile_px, bestt.cell_over_delta, bestt.radius_mode);
  if (st) return st;
  cache_store(cache_path, key, bestt);
  *best = bestt;
  return PERCH_OK;
}
