// perch_cnn_api.cpp -- C ABI of the learned successor-cost network (see
// perch_cnn.hip for the kernels and include/perch.h for the contract).
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "perch_cnn.h"
#include "perch_ctx.h"

using namespace perch;
using namespace perch::cnn;

struct perch_cnn {
  int n_mesh = 0, max_crops = 0, max_pairs = 0;
  int crop_step = 1;  // pixel step of the crops the learned search takes for this network
  hipStream_t stream = nullptr;
  int64_t n_params = 0;
  int step = 0;
  DevBuf params, grads, m, v;  // FP32, flat
  DevBuf act, dact, wb, feat, dfeat, hid, loss;
  Net net{};
  int64_t off[13];  // offsets of the 13 tensors in the flat arrays
};

namespace {

void sizes(int n_mesh, int64_t* sz) {
  int64_t k = 0;
  const int cin[4] = {2, kC, kC, kC};
  for (int l = 0; l < 4; ++l) {
    sz[k++] = (int64_t)kC * 9 * cin[l];
    sz[k++] = kC;
  }
  sz[k++] = (int64_t)n_mesh * kEmb;
  sz[k++] = (int64_t)kHid * kIn;
  sz[k++] = kHid;
  sz[k++] = kHid;
  sz[k++] = 1;
}

Params views(float* base, const int64_t* off) {
  Params p;
  for (int l = 0; l < 4; ++l) {
    p.cW[l] = base + off[2 * l];
    p.cb[l] = base + off[2 * l + 1];
  }
  p.emb = base + off[8];
  p.hW1 = base + off[9];
  p.hb1 = base + off[10];
  p.hw2 = base + off[11];
  p.hb2 = base + off[12];
  return p;
}

}  // namespace

namespace perch {
namespace cnn {

bool crop_descriptors(const float M[12], float fx, float fy, float cx, float cy, const float* xy,
                      int n, CropDesc* out, int step) {
  // crop centre: the table point (x, y, 0) projected to the nearest pixel
  for (int k = 0; k < n; ++k) {
    double p[3];
    for (int r = 0; r < 3; ++r)
      p[r] = (double)M[4 * r] * xy[2 * k] + (double)M[4 * r + 1] * xy[2 * k + 1] + M[4 * r + 3];
    if (!(p[2] > 0.01)) return false;
    out[k].u0 = (int)std::lround(fx * p[0] / p[2] + cx);
    out[k].v0 = (int)std::lround(fy * p[1] / p[2] + cy);
    out[k].zref = (float)p[2];
    out[k].step = step;
  }
  return true;
}

}  // namespace cnn

int cnn_crop_step(const perch_cnn* c) { return c ? c->crop_step : 1; }

perch_status cnn_capacity(const perch_cnn* c, int* max_crops, int* max_pairs) {
  if (!c) return fail(PERCH_E_ARG, "null network");
  *max_crops = c->max_crops;
  *max_pairs = c->max_pairs;
  return PERCH_OK;
}

perch_status cnn_predict_on(perch_cnn* c, const uint16_t* crops, int n_crops, const void* pairs,
                            int n_pairs, float* pred, hipStream_t s) {
  if (!c || n_crops < 1 || n_pairs < 1 || n_crops > c->max_crops || n_pairs > c->max_pairs)
    return fail(PERCH_E_ARG, "batch (%d crops, %d pairs) above the network's capacity (%d, %d)",
                n_crops, n_pairs, c ? c->max_crops : 0, c ? c->max_pairs : 0);
  c->net.crops = crops;
  launch_infer_predict(c->net, n_crops, c->n_mesh, reinterpret_cast<const Pair*>(pairs), n_pairs,
                       pred, s);
  HIP_TRY(hipGetLastError());
  return PERCH_OK;
}

perch_status cnn_predict_scene_on(perch_cnn* c, perch_ctx* ctx, const void* desc_dev,
                                  int n_crops, const void* pairs, int n_pairs, float* pred,
                                  hipStream_t s) {
  if (!c || n_crops < 1 || n_pairs < 1 || n_crops > c->max_crops || n_pairs > c->max_pairs)
    return fail(PERCH_E_ARG, "batch (%d crops, %d pairs) above the network's capacity (%d, %d)",
                n_crops, n_pairs, c ? c->max_crops : 0, c ? c->max_pairs : 0);
  ImageCrops img;
  img.obs = ctx->obs.as<float>();
  img.pdepth = ctx->par_depth.as<unsigned>();
  img.W = ctx->cam.W;
  img.H = ctx->cam.H;
  img.desc = reinterpret_cast<const CropDesc*>(desc_dev);
  launch_infer_predict(c->net, n_crops, c->n_mesh, reinterpret_cast<const Pair*>(pairs), n_pairs,
                       pred, s, &img);
  HIP_TRY(hipGetLastError());
  return PERCH_OK;
}

}  // namespace perch

perch_status rank_children(perch_ctx* c, const float* pred, int n_poses, int n_meshes,
                           const MeshMask& mask, int k, const int* mesh_ids, const int* pose_ids,
                           int2* out, hipStream_t st) {
  if (k < 1 || (int64_t)k > (int64_t)n_poses * n_meshes || n_meshes > kMaxMeshes)
    return fail(PERCH_E_ARG, "ranking: k = %d of %d x %d children", k, n_meshes, n_poses);
  if (launch_select_topk(pred, n_poses, n_meshes, mask, k, mesh_ids, pose_ids, out, st))
    return PERCH_OK;
  const int n = n_poses * n_meshes;
  DevBuf &d_keys = c->learned_bufs[6], &d_idx = c->learned_bufs[7];
  if (const int chunks = select_chunks(n, k)) {
    HIP_TRY(d_keys.ensure(sizeof(unsigned long long) * chunks * k));
    launch_select_topk2(pred, n_poses, n_meshes, mask, k, mesh_ids, pose_ids, out,
                        d_keys.as<unsigned long long>(), st);
    return PERCH_OK;
  }
  DevBuf &d_idx2 = c->learned_bufs[8], &d_temp = c->learned_bufs[9];
  DevBuf& d_masked = c->learned_bufs[10];
  const size_t temp_bytes = select_temp_bytes(n);
  HIP_TRY(d_masked.ensure(sizeof(float) * n));
  HIP_TRY(d_keys.ensure(sizeof(float) * n));
  HIP_TRY(d_idx.ensure(sizeof(int) * n));
  HIP_TRY(d_idx2.ensure(sizeof(int) * n));
  HIP_TRY(d_temp.ensure(temp_bytes));
  launch_iota(d_idx.as<int>(), n, st);
  launch_mask_children(pred, d_masked.as<float>(), n_poses, n_meshes, mask, st);
  HIP_TRY(sort_predictions(d_temp.p, temp_bytes, d_masked.as<float>(), d_keys.as<float>(),
                           d_idx.as<int>(), d_idx2.as<int>(), n, st));
  launch_child_cands(d_idx2.as<int>(), k, mesh_ids, n_poses, pose_ids, out, st);
  return PERCH_OK;
}

extern "C" {

perch_status perch_cnn_create(int32_t n_mesh, int32_t max_crops, int32_t max_pairs,
                              void* hip_stream, perch_cnn** out) {
  if (!out || n_mesh < 1 || max_crops < 1 || max_pairs < 1 || max_crops > 65536)
    return fail(PERCH_E_ARG, "bad network sizes");
  *out = nullptr;
  perch_cnn* c = new perch_cnn();
  c->n_mesh = n_mesh;
  c->max_crops = max_crops;
  c->max_pairs = max_pairs;
  c->stream = static_cast<hipStream_t>(hip_stream);
  int64_t sz[13];
  sizes(n_mesh, sz);
  int64_t o = 0;
  for (int k = 0; k < 13; ++k) {
    c->off[k] = o;
    o += sz[k];
  }
  c->n_params = o;
  const size_t pb = (size_t)o * sizeof(float);
  const size_t per_crop = (size_t)kC * (64 * 64 + 32 * 32 + 16 * 16 + 8 * 8);  // a1..a4 elements
  const size_t kp[4] = {32, 288, 288, 288};
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
  if (e == hipSuccess) e = hipMemsetAsync(c->params.p, 0, pb, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->m.p, 0, pb, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->v.p, 0, pb, c->stream);
  if (e != hipSuccess) {
    for (DevBuf* b : {&c->params, &c->grads, &c->m, &c->v, &c->act, &c->dact, &c->wb, &c->feat,
                      &c->dfeat, &c->loss})
      b->release();
    delete c;
    return fail(e == hipErrorOutOfMemory ? PERCH_E_OOM : PERCH_E_HIP, "network setup: %s",
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
  n.P = views(c->params.as<float>(), c->off);
  n.G = views(c->grads.as<float>(), c->off);
  launch_pack(n, c->stream);
  *out = c;
  return PERCH_OK;
}

void perch_cnn_destroy(perch_cnn* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (DevBuf* b : {&c->params, &c->grads, &c->m, &c->v, &c->act, &c->dact, &c->wb, &c->feat,
                    &c->dfeat, &c->hid, &c->loss})
    b->release();
  delete c;
}

int64_t perch_cnn_param_count(const perch_cnn* c) { return c ? c->n_params : -1; }

perch_status perch_cnn_set_crop_step(perch_cnn* c, int32_t step) {
  if (!c || step < 1 || step > 64) return fail(PERCH_E_ARG, "bad crop step");
  c->crop_step = step;
  return PERCH_OK;
}

perch_status perch_cnn_set_params(perch_cnn* c, const float* host, int64_t n) {
  if (!c || !host || n != c->n_params) return fail(PERCH_E_ARG, "parameter count mismatch");
  HIP_TRY(hipMemcpyAsync(c->params.p, host, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemsetAsync(c->m.p, 0, n * sizeof(float), c->stream));
  HIP_TRY(hipMemsetAsync(c->v.p, 0, n * sizeof(float), c->stream));
  launch_pack(c->net, c->stream);
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->step = 0;
  return PERCH_OK;
}

perch_status perch_cnn_get_params(perch_cnn* c, float* host, int64_t n) {
  if (!c || !host || n != c->n_params) return fail(PERCH_E_ARG, "parameter count mismatch");
  HIP_TRY(hipMemcpyAsync(host, c->params.p, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return PERCH_OK;
}

perch_status perch_cnn_crops(perch_ctx* ctx, const float* xy, int32_t n, uint16_t* crops_dev) {
  if (!ctx || n < 0 || (n > 0 && (!xy || !crops_dev))) return fail(PERCH_E_ARG, "bad arguments");
  if (reinterpret_cast<uintptr_t>(crops_dev) % 16 != 0)
    return fail(PERCH_E_ARG, "crops must be 16-byte aligned");
  if (!ctx->has_obs) return fail(PERCH_E_STATE, "perch_set_observation not called");
  if (ctx->parent_j < 0) return fail(PERCH_E_STATE, "perch_set_parent not called");
  if (n == 0) return PERCH_OK;
  std::vector<CropDesc> d(n);
  const Cam& cam = ctx->cam;
  if (!crop_descriptors(cam.M, cam.fx, cam.fy, cam.cx, cam.cy, xy, n, d.data()))
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

perch_status perch_cnn_predict_scene(perch_cnn* net, perch_ctx* ctx, const float* xy, int32_t n,
                                     const perch_cnn_pair* pairs_dev, int32_t n_pairs,
                                     float* pred_dev) {
  if (!net || !ctx || !xy || !pairs_dev || !pred_dev || n < 1 || n_pairs < 1)
    return fail(PERCH_E_ARG, "bad arguments");
  if (!ctx->has_obs) return fail(PERCH_E_STATE, "perch_set_observation not called");
  if (ctx->parent_j < 0) return fail(PERCH_E_STATE, "perch_set_parent not called");
  std::vector<CropDesc> d(n);
  const Cam& cam = ctx->cam;
  if (!crop_descriptors(cam.M, cam.fx, cam.fy, cam.cx, cam.cy, xy, n, d.data(), net->crop_step))
    return fail(PERCH_E_ARG, "a crop centre lies behind the camera");
  HIP_TRY(ctx->cnn_desc.ensure(sizeof(CropDesc) * n));
  HIP_TRY(hipMemcpyAsync(ctx->cnn_desc.p, d.data(), sizeof(CropDesc) * n, hipMemcpyHostToDevice,
                         ctx->stream));
  perch_status st = cnn_predict_scene_on(net, ctx, ctx->cnn_desc.p, n, pairs_dev, n_pairs,
                                         pred_dev, ctx->stream);
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(ctx->stream));  // the host descriptors die here
  return PERCH_OK;
}

perch_status perch_rank_children(perch_ctx* ctx, const float* pred_dev, int32_t n_poses,
                                 int32_t n_meshes, const int32_t* allow_host, int32_t k,
                                 const int32_t* mesh_ids_dev, const int32_t* pose_ids_dev,
                                 perch_object* out_dev) {
  if (!ctx || !pred_dev || !allow_host || !mesh_ids_dev || !pose_ids_dev || !out_dev)
    return fail(PERCH_E_ARG, "null argument");
  if (n_poses < 1 || n_meshes < 1 || n_meshes > kMaxMeshes)
    return fail(PERCH_E_ARG, "need 1 <= n_poses and 1 <= n_meshes <= %d", kMaxMeshes);
  if ((int64_t)n_poses * n_meshes > INT32_MAX) return fail(PERCH_E_ARG, "too many children");
  const int n = n_poses * n_meshes;
  if (k < 1 || k > n) return fail(PERCH_E_ARG, "need 1 <= k <= %d", n);
  MeshMask mask{};
  for (int u = 0; u < n_meshes; ++u) mask.allow[u] = allow_host[u] ? 1 : 0;
  perch_status st = rank_children(ctx, pred_dev, n_poses, n_meshes, mask, k, mesh_ids_dev,
                                  pose_ids_dev, reinterpret_cast<int2*>(out_dev), ctx->stream);
  if (st) return st;
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return PERCH_OK;
}

static perch_status check_batch(perch_cnn* c, const uint16_t* crops, int32_t n_crops,
                                const perch_cnn_pair* pairs, int32_t n_pairs) {
  if (!c || !crops || !pairs || n_crops < 1 || n_pairs < 1)
    return fail(PERCH_E_ARG, "empty or null batch");
  if (reinterpret_cast<uintptr_t>(crops) % 16 != 0)
    return fail(PERCH_E_ARG, "crops must be 16-byte aligned");
  if (n_crops > c->max_crops || n_pairs > c->max_pairs)
    return fail(PERCH_E_ARG, "batch (%d crops, %d pairs) above the network's capacity (%d, %d)",
                n_crops, n_pairs, c->max_crops, c->max_pairs);
  return PERCH_OK;
}

perch_status perch_cnn_predict(perch_cnn* c, const uint16_t* crops_dev, int32_t n_crops,
                               const perch_cnn_pair* pairs_dev, int32_t n_pairs, float* pred_dev) {
  perch_status st = check_batch(c, crops_dev, n_crops, pairs_dev, n_pairs);
  if (st) return st;
  if (!pred_dev) return fail(PERCH_E_ARG, "null output");
  c->net.crops = crops_dev;
  launch_infer_predict(c->net, n_crops, c->n_mesh, reinterpret_cast<const Pair*>(pairs_dev),
                       n_pairs, pred_dev, c->stream);
  HIP_TRY(hipGetLastError());
  return PERCH_OK;
}

static perch_status run_backward(perch_cnn* c, const uint16_t* crops, int32_t n_crops,
                                 const perch_cnn_pair* pairs, const float* target, int32_t n_pairs,
                                 float* loss_host) {
  HIP_TRY(hipMemsetAsync(c->grads.p, 0, c->n_params * sizeof(float), c->stream));
  HIP_TRY(hipMemsetAsync(c->dfeat.p, 0, (size_t)n_crops * kFeat * sizeof(float), c->stream));
  HIP_TRY(hipMemsetAsync(c->loss.p, 0, sizeof(float), c->stream));
  c->net.crops = crops;
  launch_forward(c->net, n_crops, c->stream);
  launch_backward(c->net, n_crops, c->n_mesh, reinterpret_cast<const Pair*>(pairs), target,
                  n_pairs, c->stream);
  HIP_TRY(hipGetLastError());
  if (loss_host) {
    float s = 0.0f;
    HIP_TRY(hipMemcpyAsync(&s, c->loss.p, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *loss_host = s / (float)n_pairs;
  }
  return PERCH_OK;
}

perch_status perch_cnn_gradients(perch_cnn* c, const uint16_t* crops_dev, int32_t n_crops,
                                 const perch_cnn_pair* pairs_dev, const float* target_dev,
                                 int32_t n_pairs, float* grads_host, float* loss_host) {
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

perch_status perch_cnn_train_step(perch_cnn* c, const uint16_t* crops_dev, int32_t n_crops,
                                  const perch_cnn_pair* pairs_dev, const float* target_dev,
                                  int32_t n_pairs, float lr, float* loss_host) {
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

}  // extern "C"
