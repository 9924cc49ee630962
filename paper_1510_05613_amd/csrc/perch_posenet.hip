// perch_posenet.hip -- head kernels of the per-object pose regressor (gfx950).
//
// The paper names discriminative pose estimates as a second kind of guidance for
// its multi-heuristic search: an inadmissible heuristic that measures how far a
// state's placed objects lie from the poses a discriminative estimator proposes
// (arXiv:1510.05613 Sec. IV-C, "Heuristics").  This regressor is that estimator.
// It shares the convolution trunk (bfloat16 MFMA kernels of perch_cnn.hip) with the
// successor-cost network but has its own weights; one crop is taken around each
// anchor point of a coarse grid on the table, and for every (crop, mesh) pair the
// head predicts
//   - an objectness logit: does the object of this mesh stand in the anchor's cell,
//   - the object's offset (dx, dy) from the anchor in units of the anchor spacing,
//   - logits over the n_yaw yaw bins of the pose grid.
// Loss per pair: logistic loss of the objectness + label * (kPoseWxy * squared
// offset error + kPoseWyaw * cross-entropy of the yaw logits against a target
// spread evenly over the bins the mesh's symmetry makes equivalent); the mean over
// the pairs.  Head arithmetic, loss and gradients are FP32.
#include <hip/hip_runtime.h>

#include "perch_cnn.h"

namespace perch {
namespace cnn {

__device__ __forceinline__ bool pose_pair_ok(const PosePair& pr, int n_crops, int n_mesh) {
  return pr.crop >= 0 && pr.crop < n_crops && pr.mesh >= 0 && pr.mesh < n_mesh;
}

// First layer split by input: block b < n_crops holds crop b's feature term of every
// hidden unit, A[b][r] = sum_i W1[r][i] feat[b][i]; block n_crops + m holds mesh m's
// term, B[m][r] = b1[r] + sum_e W1[r][64 + e] emb[m][e].
__global__ void __launch_bounds__(kHid)
    k_pose_parts(const float* feat, const PoseParams P, int n_crops, float* hid) {
  __shared__ float x[kFeat];
  const int b = blockIdx.x, r = threadIdx.x;
  const bool crop = b < n_crops;
  const int m = b - n_crops;
  if (crop) x[r] = feat[b * kFeat + r];
  else if (r < kEmb) x[r] = P.emb[m * kEmb + r];
  __syncthreads();
  const float* w = P.W1 + r * kPoseIn;
  float z = crop ? 0.0f : P.b1[r];
  if (crop)
    for (int i = 0; i < kFeat; ++i) z = fmaf(w[i], x[i], z);
  else
    for (int e = 0; e < kEmb; ++e) z = fmaf(w[kFeat + e], x[e], z);
  hid[b * kHid + r] = z;
}

// One pair per thread: the 3 + n_yaw outputs (NaN for an out-of-range pair).
__global__ void k_pose_pairs(const float* hid, const PoseParams P, int n_yaw,
                             const PosePair* pairs, int n_pairs, int n_crops, int n_mesh,
                             float* out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_pairs) return;
  const int no = 3 + n_yaw;
  const PosePair pr = pairs[q];
  float* o = out + (size_t)q * no;
  if (!pose_pair_ok(pr, n_crops, n_mesh)) {
    for (int k = 0; k < no; ++k) o[k] = __uint_as_float(0x7fc00000u);
    return;
  }
  const float* a = hid + pr.crop * kHid;
  const float* bm = hid + (n_crops + pr.mesh) * kHid;
  float h[kHid];
  for (int r = 0; r < kHid; ++r) h[r] = fmaxf(a[r] + bm[r], 0.0f);
  for (int k = 0; k < no; ++k) {
    const float* w = P.W2 + k * kHid;
    float y = P.b2[k];
    for (int r = 0; r < kHid; ++r) y = fmaf(w[r], h[r], y);
    o[k] = y;
  }
}

// Loss and head gradients for 64 pairs per workgroup (one thread per pair): the
// pair's head input, hidden activations and output gradients go to LDS, and the
// weight gradients are reduced over the workgroup's pairs before one atomic add.
__global__ void __launch_bounds__(64)
    k_pose_bwd(const float* feat, const PoseParams P, int n_yaw, const PosePair* pairs,
               const PoseTarget* target, int n_pairs, int n_crops, int n_mesh, PoseParams G,
               float* dfeat, float* loss_sum) {
  constexpr int kNo = 3 + kMaxYaw;
  __shared__ float sh[64][kPoseIn];  // head input per pair
  __shared__ float sr1[64][kHid];    // relu(z1) per pair
  __shared__ float sdz[64][kHid];    // d loss / d z1 per pair
  __shared__ float sdo[64][kNo];     // d loss / d output per pair
  const int t = threadIdx.x;
  const int q = blockIdx.x * 64 + t;
  const int no = 3 + n_yaw;
  const PosePair pr = q < n_pairs ? pairs[q] : PosePair{-1, -1};
  const bool live = q < n_pairs && pose_pair_ok(pr, n_crops, n_mesh);
  if (live) {
    for (int i = 0; i < kFeat; ++i) sh[t][i] = feat[pr.crop * kFeat + i];
    for (int e = 0; e < kEmb; ++e) sh[t][kFeat + e] = P.emb[pr.mesh * kEmb + e];
    for (int r = 0; r < kHid; ++r) {
      float z = P.b1[r];
      for (int i = 0; i < kPoseIn; ++i) z = fmaf(P.W1[r * kPoseIn + i], sh[t][i], z);
      sr1[t][r] = fmaxf(z, 0.0f);
      sdz[t][r] = z;  // pre-activation for now
    }
    // the outputs wait in sdo[t] and are overwritten by their gradients
    float* y = sdo[t];
    for (int k = 0; k < no; ++k) {
      float v = P.b2[k];
      for (int r = 0; r < kHid; ++r) v = fmaf(P.W2[k * kHid + r], sr1[t][r], v);
      y[k] = v;
    }
    const PoseTarget tg = target[q];
    const float inv_n = 1.0f / (float)n_pairs;
    // objectness: log(1 + e^s) - label s, gradient sigmoid(s) - label
    const float s = y[0];
    float L = fmaxf(s, 0.0f) - tg.label * s + log1pf(expf(-fabsf(s)));
    y[0] = (1.0f / (1.0f + expf(-s)) - tg.label) * inv_n;
    if (tg.label > 0.0f) {
      const float ex = y[1] - tg.dx, ey = y[2] - tg.dy;
      L += kPoseWxy * (ex * ex + ey * ey);
      y[1] = 2.0f * kPoseWxy * ex * inv_n;
      y[2] = 2.0f * kPoseWxy * ey * inv_n;
      // yaw: log-sum-exp minus the mean logit over the equivalent bins
      float m = -INFINITY;
      for (int k = 0; k < n_yaw; ++k) m = fmaxf(m, y[3 + k]);
      float se = 0.0f;
      for (int k = 0; k < n_yaw; ++k) se += expf(y[3 + k] - m);
      const int per = max(1, (int)tg.period), kb = (int)tg.yaw_bin;
      const int n_eq = max(1, n_yaw / per);
      float tz = 0.0f;
      for (int k = 0; k < n_yaw; ++k)
        if ((k - kb) % per == 0) tz += y[3 + k];
      L += kPoseWyaw * (m + logf(se) - tz / (float)n_eq);
      for (int k = 0; k < n_yaw; ++k) {
        const float tk = ((k - kb) % per == 0) ? 1.0f / (float)n_eq : 0.0f;
        y[3 + k] = kPoseWyaw * (expf(y[3 + k] - m) / se - tk) * inv_n;
      }
    } else {
      for (int k = 1; k < no; ++k) y[k] = 0.0f;
    }
    for (int k = no; k < kNo; ++k) y[k] = 0.0f;
    atomicAdd(loss_sum, L);
    for (int r = 0; r < kHid; ++r) {
      float g = 0.0f;
      for (int k = 0; k < no; ++k) g = fmaf(P.W2[k * kHid + r], sdo[t][k], g);
      sdz[t][r] = sdz[t][r] > 0.0f ? g : 0.0f;
    }
  } else {
    for (int i = 0; i < kPoseIn; ++i) sh[t][i] = 0.0f;
    for (int r = 0; r < kHid; ++r) {
      sr1[t][r] = 0.0f;
      sdz[t][r] = 0.0f;
    }
    for (int k = 0; k < kNo; ++k) sdo[t][k] = 0.0f;
  }
  __syncthreads();
  // input gradients: features per crop, embedding per mesh
  if (live) {
    for (int i = 0; i < kPoseIn; ++i) {
      float g = 0.0f;
      for (int r = 0; r < kHid; ++r) g = fmaf(P.W1[r * kPoseIn + i], sdz[t][r], g);
      if (i < kFeat)
        atomicAdd(&dfeat[pr.crop * kFeat + i], g);
      else
        atomicAdd(&G.emb[pr.mesh * kEmb + (i - kFeat)], g);
    }
  }
  // weight gradients reduced over the workgroup's pairs
  for (int e = t; e < kHid * kPoseIn; e += 64) {
    const int r = e / kPoseIn, i = e % kPoseIn;
    float g = 0.0f;
    for (int u = 0; u < 64; ++u) g = fmaf(sdz[u][r], sh[u][i], g);
    atomicAdd(&G.W1[e], g);
  }
  for (int e = t; e < no * kHid; e += 64) {
    const int k = e / kHid, r = e % kHid;
    float g = 0.0f;
    for (int u = 0; u < 64; ++u) g = fmaf(sdo[u][k], sr1[u][r], g);
    atomicAdd(&G.W2[e], g);
  }
  {
    float g = 0.0f;
    for (int u = 0; u < 64; ++u) g += sdz[u][t];  // kHid == blockDim.x
    atomicAdd(&G.b1[t], g);
  }
  if (t < no) {
    float g = 0.0f;
    for (int u = 0; u < 64; ++u) g += sdo[u][t];
    atomicAdd(&G.b2[t], g);
  }
}

// One workgroup per query: `count` picks by decreasing objectness among anchors not
// within nms_m of an earlier pick (ties: the lower anchor index), each decoded to
// (mesh, x, y, theta) with theta = 2 pi k / n_yaw of its largest yaw logit (ties:
// the lower bin).
__global__ void __launch_bounds__(256)
    k_pose_decode(const float* out, int n_yaw, int n_anchors, const float2* anchors,
                  float spacing, float nms_m, const PoseQuery* queries, float4* res) {
  __shared__ float s_best[256];
  __shared__ int s_arg[256];
  __shared__ int s_pick[64];
  const PoseQuery qr = queries[blockIdx.x];
  const int t = threadIdx.x;
  const int no = 3 + n_yaw;
  const float* o = out + (size_t)blockIdx.x * n_anchors * no;
  const int count = min(qr.count, 64);
  for (int c = 0; c < count; ++c) {
    float best = -INFINITY;
    int arg = -1;
    for (int a = t; a < n_anchors; a += 256) {
      bool free = true;
      for (int p = 0; p < c && free; ++p) {
        const float2 u = anchors[a], v = anchors[s_pick[p]];
        const float dx = u.x - v.x, dy = u.y - v.y;
        free = dx * dx + dy * dy >= nms_m * nms_m;
      }
      const float sc = o[(size_t)a * no];
      if (free && (arg < 0 || sc > best)) {  // a grows: the first maximum stays
        best = sc;
        arg = a;
      }
    }
    s_best[t] = best;
    s_arg[t] = arg;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) {
        const int a2 = s_arg[t + w];
        const bool take = a2 >= 0 && (s_arg[t] < 0 || s_best[t + w] > s_best[t] ||
                                      (s_best[t + w] == s_best[t] && a2 < s_arg[t]));
        if (take) {
          s_best[t] = s_best[t + w];
          s_arg[t] = a2;
        }
      }
      __syncthreads();
    }
    const int a = s_arg[0];
    if (t == 0) {
      s_pick[c] = a < 0 ? 0 : a;
      float4 r = make_float4(__int_as_float(qr.mesh), 0.0f, 0.0f, 0.0f);
      if (a >= 0) {
        const float* y = o + (size_t)a * no;
        int kb = 0;
        for (int k = 1; k < n_yaw; ++k)
          if (y[3 + k] > y[3 + kb]) kb = k;
        r.y = anchors[a].x + spacing * y[1];
        r.z = anchors[a].y + spacing * y[2];
        r.w = 6.28318530717958648f * (float)kb / (float)n_yaw;
      } else {
        r.x = __int_as_float(-1);  // fewer free anchors than instances
      }
      res[qr.first + c] = r;
    }
    __syncthreads();
  }
}

void launch_pose_predict(const Net& net, const PoseParams& P, int n_yaw, int n_crops, int n_mesh,
                         const PosePair* pairs, int n_pairs, float* out, hipStream_t s) {
  if (n_pairs <= 0) return;
  hipLaunchKernelGGL(k_pose_parts, dim3(n_crops + n_mesh), dim3(kHid), 0, s, net.feat, P, n_crops,
                     net.hid);
  hipLaunchKernelGGL(k_pose_pairs, dim3((n_pairs + 127) / 128), dim3(128), 0, s, net.hid, P,
                     n_yaw, pairs, n_pairs, n_crops, n_mesh, out);
}

void launch_pose_backward(const Net& net, const PoseParams& P, const PoseParams& G, int n_yaw,
                          int n_crops, int n_mesh, const PosePair* pairs,
                          const PoseTarget* target, int n_pairs, hipStream_t s) {
  hipLaunchKernelGGL(k_pose_bwd, dim3((n_pairs + 63) / 64), dim3(64), 0, s, net.feat, P, n_yaw,
                     pairs, target, n_pairs, n_crops, n_mesh, G, net.dfeat, net.loss);
  launch_trunk_backward(net, n_crops, s);
}

void launch_pose_decode(const float* out, int n_yaw, int n_anchors, const float2* anchors,
                        float spacing, float nms_m, const PoseQuery* q, int n_q, float4* res,
                        hipStream_t s) {
  if (n_q > 0)
    hipLaunchKernelGGL(k_pose_decode, dim3(n_q), dim3(256), 0, s, out, n_yaw, n_anchors, anchors,
                       spacing, nms_m, q, res);
}

}  // namespace cnn
}  // namespace perch
