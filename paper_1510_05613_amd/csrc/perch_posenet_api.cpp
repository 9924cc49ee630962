// perch_posenet_api.cpp -- C ABI of the per-object pose regressor (kernels in
// perch_posenet.hip and perch_cnn.hip, contract in include/perch.h).
#include <cstring>
#include <vector>

#include "perch_cnn.h"
#include "perch_ctx.h"

using namespace perch;
using namespace perch::cnn;

struct perch_posenet {
  int n_mesh = 0, n_yaw = 0, max_crops = 0, max_pairs = 0;
  hipStream_t stream = nullptr;
  int64_t n_params = 0;
  int step = 0;
  DevBuf params, grads, m, v;  // FP32, flat
  DevBuf act, dact, wb, feat, dfeat, hid, loss;
  DevBuf out, pairs, anchors, queries, res;  // estimate scratch
  Net net{};
  PoseParams P{}, G{};
  int64_t off[13];
};

namespace {

void pose_sizes(int n_mesh, int n_yaw, int64_t* sz) {
  int64_t k = 0;
  const int cin[4] = {2, kC, kC, kC};
  for (int l = 0; l < 4; ++l) {
    sz[k++] = (int64_t)kC * 9 * cin[l];
    sz[k++] = kC;
  }
  sz[k++] = (int64_t)n_mesh * kEmb;
  sz[k++] = (int64_t)kHid * kPoseIn;
  sz[k++] = kHid;
  sz[k++] = (int64_t)(3 + n_yaw) * kHid;
  sz[k++] = 3 + n_yaw;
}

void pose_views(float* base, const int64_t* off, Params& trunk, PoseParams& head) {
  trunk = Params{};
  for (int l = 0; l < 4; ++l) {
    trunk.cW[l] = base + off[2 * l];
    trunk.cb[l] = base + off[2 * l + 1];
  }
  head.emb = base + off[8];
  head.W1 = base + off[9];
  head.b1 = base + off[10];
  head.W2 = base + off[11];
  head.b2 = base + off[12];
}

void release_all(perch_posenet* c) {
  for (DevBuf* b : {&c->params, &c->grads, &c->m, &c->v, &c->act, &c->dact, &c->wb, &c->feat,
                    &c->dfeat, &c->hid, &c->loss, &c->out, &c->pairs, &c->anchors, &c->queries,
                    &c->res})
    b->release();
}

perch_status check_batch(perch_posenet* c, const uint16_t* crops, int32_t n_crops,
                         const perch_posenet_pair* pairs, int32_t n_pairs) {
  if (!c || !crops || !pairs || n_crops < 1 || n_pairs < 1)
    return fail(PERCH_E_ARG, "empty or null batch");
  if (reinterpret_cast<uintptr_t>(crops) % 16 != 0)
    return fail(PERCH_E_ARG, "crops must be 16-byte aligned");
  if (n_crops > c->max_crops || n_pairs > c->max_pairs)
    return fail(PERCH_E_ARG, "batch (%d crops, %d pairs) above the network's capacity (%d, %d)",
                n_crops, n_pairs, c->max_crops, c->max_pairs);
  return PERCH_OK;
}

perch_status run_backward(perch_posenet* c, const uint16_t* crops, int32_t n_crops,
                          const perch_posenet_pair* pairs, const perch_posenet_target* target,
                          int32_t n_pairs, float* loss_host) {
  HIP_TRY(hipMemsetAsync(c->grads.p, 0, c->n_params * sizeof(float), c->stream));
  HIP_TRY(hipMemsetAsync(c->dfeat.p, 0, (size_t)n_crops * kFeat * sizeof(float), c->stream));
  HIP_TRY(hipMemsetAsync(c->loss.p, 0, sizeof(float), c->stream));
  c->net.crops = crops;
  launch_forward(c->net, n_crops, c->stream);
  launch_pose_backward(c->net, c->P, c->G, c->n_yaw, n_crops, c->n_mesh,
                       reinterpret_cast<const PosePair*>(pairs),
                       reinterpret_cast<const PoseTarget*>(target), n_pairs, c->stream);
  HIP_TRY(hipGetLastError());
  if (loss_host) {
    float s = 0.0f;
    HIP_TRY(hipMemcpyAsync(&s, c->loss.p, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *loss_host = s / (float)n_pairs;
  }
  return PERCH_OK;
}

}  // namespace

static_assert(sizeof(perch_posenet_pair) == sizeof(PosePair), "pair layouts differ");
static_assert(sizeof(perch_posenet_target) == sizeof(PoseTarget), "target layouts differ");
static_assert(sizeof(perch_pose_prior) == sizeof(float4), "prior layout differs");

extern "C" {

perch_status perch_posenet_create(int32_t n_mesh, int32_t n_yaw, int32_t max_crops,
                                  int32_t max_pairs, void* hip_stream, perch_posenet** out) {
  if (!out || n_mesh < 1 || n_yaw < 1 || n_yaw > kMaxYaw || max_crops < 1 || max_pairs < 1 ||
      max_crops > 65536)
    return fail(PERCH_E_ARG, "bad pose network sizes");
  *out = nullptr;
  perch_posenet* c = new perch_posenet();
  c->n_mesh = n_mesh;
  c->n_yaw = n_yaw;
  c->max_crops = max_crops;
  c->max_pairs = max_pairs;
  c->stream = static_cast<hipStream_t>(hip_stream);
  int64_t sz[13];
  pose_sizes(n_mesh, n_yaw, sz);
  int64_t o = 0;
  for (int k = 0; k < 13; ++k) {
    c->off[k] = o;
    o += sz[k];
  }
  c->n_params = o;
  const size_t pb = (size_t)o * sizeof(float);
  const size_t per_crop = (size_t)kC * (64 * 64 + 32 * 32 + 16 * 16 + 8 * 8);
  const size_t kp[4] = {32, 288, 288, 288};
  const int no = 3 + n_yaw;
  hipError_t e = hipSuccess;
  for (DevBuf* b : {&c->params, &c->grads, &c->m, &c->v})
    if (e == hipSuccess) e = b->ensure(pb);
  if (e == hipSuccess) e = c->act.ensure(per_crop * max_crops * sizeof(bf16_t));
  if (e == hipSuccess) e = c->dact.ensure(per_crop * max_crops * sizeof(bf16_t));
  if (e == hipSuccess) e = c->wb.ensure((kp[0] + 3 * kp[1]) * kC * sizeof(bf16_t));
  if (e == hipSuccess) e = c->feat.ensure((size_t)max_crops * kFeat * sizeof(float));
  if (e == hipSuccess) e = c->dfeat.ensure((size_t)max_crops * kFeat * sizeof(float));
  if (e == hipSuccess) e = c->hid.ensure((size_t)(max_crops + n_mesh) * kHid * sizeof(float));
  if (e == hipSuccess) e = c->loss.ensure(sizeof(float));
  if (e == hipSuccess) e = c->out.ensure((size_t)max_pairs * no * sizeof(float));
  if (e == hipSuccess) e = c->pairs.ensure((size_t)max_pairs * sizeof(PosePair));
  if (e == hipSuccess) e = hipMemsetAsync(c->params.p, 0, pb, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->m.p, 0, pb, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->v.p, 0, pb, c->stream);
  if (e != hipSuccess) {
    release_all(c);
    delete c;
    return fail(e == hipErrorOutOfMemory ? PERCH_E_OOM : PERCH_E_HIP, "pose network setup: %s",
                hipGetErrorString(e));
  }
  Net& n = c->net;
  bf16_t* a = c->act.as<bf16_t>();
  bf16_t* d = c->dact.as<bf16_t>();
  const size_t sp[5] = {0, 64 * 64, 32 * 32, 16 * 16, 8 * 8};
  n.a[0] = n.d[0] = nullptr;
  for (int l = 1; l <= 4; ++l) {
    n.a[l] = a;
    n.d[l] = d;
    a += sp[l] * kC * max_crops;
    d += sp[l] * kC * max_crops;
  }
  bf16_t* w = c->wb.as<bf16_t>();
  for (int l = 0; l < 4; ++l) {
    n.Wb[l] = w;
    w += kp[l] * kC;
  }
  n.feat = c->feat.as<float>();
  n.dfeat = c->dfeat.as<float>();
  n.hid = c->hid.as<float>();
  n.loss = c->loss.as<float>();
  pose_views(c->params.as<float>(), c->off, n.P, c->P);
  pose_views(c->grads.as<float>(), c->off, n.G, c->G);
  launch_pack(n, c->stream);
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    release_all(c);
    delete c;
    return fail(PERCH_E_HIP, "pose network setup failed");
  }
  *out = c;
  return PERCH_OK;
}

void perch_posenet_destroy(perch_posenet* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  release_all(c);
  delete c;
}

int64_t perch_posenet_param_count(const perch_posenet* c) { return c ? c->n_params : -1; }

perch_status perch_posenet_set_params(perch_posenet* c, const float* host, int64_t n) {
  if (!c || !host || n != c->n_params) return fail(PERCH_E_ARG, "parameter count mismatch");
  HIP_TRY(hipMemcpyAsync(c->params.p, host, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemsetAsync(c->m.p, 0, n * sizeof(float), c->stream));
  HIP_TRY(hipMemsetAsync(c->v.p, 0, n * sizeof(float), c->stream));
  launch_pack(c->net, c->stream);
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->step = 0;
  return PERCH_OK;
}

perch_status perch_posenet_get_params(perch_posenet* c, float* host, int64_t n) {
  if (!c || !host || n != c->n_params) return fail(PERCH_E_ARG, "parameter count mismatch");
  HIP_TRY(hipMemcpyAsync(host, c->params.p, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return PERCH_OK;
}

perch_status perch_cnn_crops_step(perch_ctx* ctx, const float* xy, int32_t n, int32_t step,
                                  uint16_t* crops_dev) {
  if (!ctx || n < 0 || step < 1 || step > 64 || (n > 0 && (!xy || !crops_dev)))
    return fail(PERCH_E_ARG, "bad arguments");
  if (reinterpret_cast<uintptr_t>(crops_dev) % 16 != 0)
    return fail(PERCH_E_ARG, "crops must be 16-byte aligned");
  if (!ctx->has_obs) return fail(PERCH_E_STATE, "perch_set_observation not called");
  if (ctx->parent_j < 0) return fail(PERCH_E_STATE, "perch_set_parent not called");
  if (n == 0) return PERCH_OK;
  std::vector<CropDesc> d(n);
  const Cam& cam = ctx->cam;
  if (!crop_descriptors(cam.M, cam.fx, cam.fy, cam.cx, cam.cy, xy, n, d.data(), step))
    return fail(PERCH_E_ARG, "a crop centre lies behind the camera");
  HIP_TRY(ctx->cnn_desc.ensure(sizeof(CropDesc) * n));
  HIP_TRY(hipMemcpyAsync(ctx->cnn_desc.p, d.data(), sizeof(CropDesc) * n, hipMemcpyHostToDevice,
                         ctx->stream));
  launch_crops(ctx->obs.as<float>(), ctx->par_depth.as<unsigned>(), cam.W, cam.H,
               ctx->cnn_desc.as<CropDesc>(), n, crops_dev, ctx->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(ctx->stream));  // the host descriptors die here
  return PERCH_OK;
}

perch_status perch_posenet_predict(perch_posenet* c, const uint16_t* crops_dev, int32_t n_crops,
                                   const perch_posenet_pair* pairs_dev, int32_t n_pairs,
                                   float* out_dev) {
  perch_status st = check_batch(c, crops_dev, n_crops, pairs_dev, n_pairs);
  if (st) return st;
  if (!out_dev) return fail(PERCH_E_ARG, "null output");
  c->net.crops = crops_dev;
  launch_infer(c->net, n_crops, c->stream);
  launch_pose_predict(c->net, c->P, c->n_yaw, n_crops, c->n_mesh,
                      reinterpret_cast<const PosePair*>(pairs_dev), n_pairs, out_dev, c->stream);
  HIP_TRY(hipGetLastError());
  return PERCH_OK;
}

perch_status perch_posenet_gradients(perch_posenet* c, const uint16_t* crops_dev, int32_t n_crops,
                                     const perch_posenet_pair* pairs_dev,
                                     const perch_posenet_target* target_dev, int32_t n_pairs,
                                     float* grads_host, float* loss_host) {
  perch_status st = check_batch(c, crops_dev, n_crops, pairs_dev, n_pairs);
  if (st) return st;
  if (!target_dev || !grads_host) return fail(PERCH_E_ARG, "null argument");
  st = run_backward(c, crops_dev, n_crops, pairs_dev, target_dev, n_pairs, loss_host);
  if (st) return st;
  HIP_TRY(hipMemcpyAsync(grads_host, c->grads.p, c->n_params * sizeof(float),
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return PERCH_OK;
}

perch_status perch_posenet_train_step(perch_posenet* c, const uint16_t* crops_dev,
                                      int32_t n_crops, const perch_posenet_pair* pairs_dev,
                                      const perch_posenet_target* target_dev, int32_t n_pairs,
                                      float lr, float* loss_host) {
  perch_status st = check_batch(c, crops_dev, n_crops, pairs_dev, n_pairs);
  if (st) return st;
  if (!target_dev || !(lr > 0)) return fail(PERCH_E_ARG, "bad target or learning rate");
  st = run_backward(c, crops_dev, n_crops, pairs_dev, target_dev, n_pairs, loss_host);
  if (st) return st;
  c->step += 1;
  launch_adam(c->params.as<float>(), c->grads.as<float>(), c->m.as<float>(), c->v.as<float>(),
              (int)c->n_params, lr, c->step, c->stream);
  launch_pack(c->net, c->stream);
  HIP_TRY(hipGetLastError());
  return PERCH_OK;
}

perch_status perch_posenet_estimate(perch_posenet* c, const uint16_t* crops_dev,
                                    int32_t n_anchors, const float* anchor_xy_host, float spacing,
                                    float nms_m, const int32_t* mesh_ids_host,
                                    const int32_t* counts_host, int32_t n_meshes,
                                    perch_pose_prior* out_host, int32_t max_out, int32_t* n_out) {
  if (!c || !crops_dev || !anchor_xy_host || !mesh_ids_host || !counts_host || !n_out ||
      (max_out > 0 && !out_host))
    return fail(PERCH_E_ARG, "null argument");
  if (n_anchors < 1 || n_meshes < 1 || n_anchors > c->max_crops ||
      (int64_t)n_anchors * n_meshes > c->max_pairs)
    return fail(PERCH_E_ARG, "%d anchors x %d meshes above the network's capacity (%d, %d)",
                n_anchors, n_meshes, c->max_crops, c->max_pairs);
  if (!(spacing > 0.0f) || !(nms_m >= 0.0f)) return fail(PERCH_E_ARG, "bad spacing or nms_m");
  if (reinterpret_cast<uintptr_t>(crops_dev) % 16 != 0)
    return fail(PERCH_E_ARG, "crops must be 16-byte aligned");
  std::vector<PoseQuery> q(n_meshes);
  int total = 0;
  for (int u = 0; u < n_meshes; ++u) {
    if (mesh_ids_host[u] < 0 || mesh_ids_host[u] >= c->n_mesh || counts_host[u] < 0 ||
        counts_host[u] > 64)
      return fail(PERCH_E_ARG, "query %d: mesh %d, count %d", u, mesh_ids_host[u],
                  counts_host[u]);
    q[u] = PoseQuery{mesh_ids_host[u], counts_host[u], total, 0};
    total += counts_host[u];
  }
  *n_out = 0;
  if (total == 0) return PERCH_OK;
  const int np = n_anchors * n_meshes;
  std::vector<PosePair> pr(np);
  for (int u = 0; u < n_meshes; ++u)
    for (int a = 0; a < n_anchors; ++a) pr[(size_t)u * n_anchors + a] = PosePair{a, q[u].mesh};
  HIP_TRY(c->anchors.ensure(sizeof(float2) * n_anchors));
  HIP_TRY(c->queries.ensure(sizeof(PoseQuery) * n_meshes));
  HIP_TRY(c->res.ensure(sizeof(float4) * total));
  HIP_TRY(hipMemcpyAsync(c->pairs.p, pr.data(), sizeof(PosePair) * np, hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(c->anchors.p, anchor_xy_host, sizeof(float2) * n_anchors,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->queries.p, q.data(), sizeof(PoseQuery) * n_meshes,
                         hipMemcpyHostToDevice, c->stream));
  c->net.crops = crops_dev;
  launch_infer(c->net, n_anchors, c->stream);
  launch_pose_predict(c->net, c->P, c->n_yaw, n_anchors, c->n_mesh, c->pairs.as<PosePair>(), np,
                      c->out.as<float>(), c->stream);
  launch_pose_decode(c->out.as<float>(), c->n_yaw, n_anchors, c->anchors.as<float2>(), spacing,
                     nms_m, c->queries.as<PoseQuery>(), n_meshes, c->res.as<float4>(), c->stream);
  HIP_TRY(hipGetLastError());
  std::vector<float4> r(total);
  HIP_TRY(hipMemcpyAsync(r.data(), c->res.p, sizeof(float4) * total, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));  // pr, q and r die here
  int k = 0;
  for (int i = 0; i < total && k < max_out; ++i) {
    int mesh;
    std::memcpy(&mesh, &r[i].x, sizeof mesh);
    if (mesh < 0) continue;
    out_host[k++] = perch_pose_prior{mesh, r[i].y, r[i].z, r[i].w};
  }
  *n_out = k;
  return PERCH_OK;
}

}  // extern "C"
