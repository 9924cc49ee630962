// perch_cnn.h -- layout of the learned successor-cost network (internal).
#pragma once
#include <hip/hip_runtime.h>

namespace perch {
namespace cnn {

typedef unsigned short bf16_t;  // bfloat16 bits

constexpr int kCrop = 64;                // crop side (pixels)
constexpr int kC = 32;                   // channels of every conv layer
constexpr int kEmb = 16;                 // mesh embedding
constexpr int kFeat = 2 * kC;            // pooled features (whole map + centre)
constexpr int kHid = 64;                 // head hidden units
constexpr int kIn = kFeat + kEmb + 2;    // head input: features, embedding, cos, sin

struct CropDesc {
  int u0, v0;  // crop centre pixel
  float zref;  // camera depth of the table point under the candidate
  int step;    // pixel step between crop samples (0 or 1: every pixel)
};

struct Pair {
  int crop;  // crop index within the batch
  int mesh;
  float cos_yaw, sin_yaw;
};

// Views of one flat FP32 parameter (or gradient) array, in the order
// cW0 cb0 cW1 cb1 cW2 cb2 cW3 cb3 emb hW1 hb1 hw2 hb2, conv weights as
// [co][(ky * 3 + kx) * C_in + ci].
struct Params {
  float* cW[4];
  float* cb[4];
  float* emb;
  float* hW1;
  float* hb1;
  float* hw2;
  float* hb2;
};

struct Net {
  const bf16_t* crops;  // input of the current call, [n][64][64][2]
  bf16_t* a[5];         // a[l] = output of conv l (l = 1..4), NHWC, 32 channels
  bf16_t* d[5];         // d[l] = gradient at the pre-activation of conv l
  bf16_t* Wb[4];        // bfloat16 conv weights [32][KP]
  float* feat;          // [n][64]
  float* dfeat;
  float* hid;           // inference: [n_crops + n_mesh][64] partial first-layer sums
  float* loss;          // sum of squared errors
  Params P, G;
};

void launch_crops(const float* obs, const unsigned* pdepth, int W, int H, const CropDesc* desc,
                  int n, bf16_t* out, hipStream_t s);
// Crop centres of table points (x, y): nearest pixel of the projection and the
// camera depth of the point; false when a point lies behind the camera.
bool crop_descriptors(const float M[12], float fx, float fy, float cx, float cy, const float* xy,
                      int n, CropDesc* out, int step = 1);
// Forward pass of the trunk for training: every activation a[1..4] is kept for the
// backward pass.
void launch_forward(const Net& net, int n_crops, hipStream_t s);
// The same forward pass for inference (bit-identical features): conv1 + conv2 and
// conv3 + conv4 + pooling run as two fused kernels; of the activations only a[2]
// is written.
void launch_infer(const Net& net, int n_crops, hipStream_t s);
// Crops sampled inside the first network kernel instead of read from net.crops:
// the observation, the parent composite (float bits, +inf empty) and one descriptor
// per crop, as launch_crops takes them.
struct ImageCrops {
  const float* obs;
  const unsigned* pdepth;
  int W, H;
  const CropDesc* desc;
};
// Predictions of n_pairs (crop, mesh, yaw) pairs in three launches: launch_infer's
// two kernels, the second of which also computes the first head layer's per-crop and
// per-mesh terms, then one thread per pair adds them and the yaw terms.  img: the
// crops are sampled from the images (bit-identical to launch_crops' crops).
void launch_infer_predict(const Net& net, int n_crops, int n_mesh, const Pair* pairs,
                          int n_pairs, float* pred, hipStream_t s,
                          const ImageCrops* img = nullptr);
// Pairs whose crop index is outside [0, n_crops) or mesh outside [0, n_mesh) are
// ignored by the backward pass and predicted as NaN.
void launch_backward(const Net& net, int n_crops, int n_mesh, const Pair* pairs,
                     const float* target, int n_pairs, hipStream_t s);
// The trunk's backward pass from net.dfeat (pooled-feature gradients of n_crops
// crops): conv weight and bias gradients into net.G, activations' gradients in net.d.
void launch_trunk_backward(const Net& net, int n_crops, hipStream_t s);
void launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, int step,
                 hipStream_t s);
void launch_pack(const Net& net, hipStream_t s);

// ---- per-object pose regressor (the same trunk, its own weights and head) ----
// Head: [feat (64), mesh embedding (16)] -> 64 (ReLU) -> 3 + n_yaw outputs:
// objectness logit, position offset (dx, dy) from the crop's table point in units
// of the anchor spacing, and logits of the n_yaw yaw bins (yaw 2 pi k / n_yaw).
constexpr int kPoseIn = kFeat + kEmb;
constexpr int kMaxYaw = 32;
constexpr float kPoseWxy = 10.0f;  // weight of the position term of the loss
constexpr float kPoseWyaw = 1.0f;  // weight of the yaw term

struct PoseParams {
  float* emb;  // [n_mesh][16]
  float* W1;   // [64][80]
  float* b1;   // [64]
  float* W2;   // [3 + n_yaw][64]
  float* b2;   // [3 + n_yaw]
};

struct PosePair {
  int crop, mesh;
};

// Targets per pair: label (1: this crop's anchor holds the object), dx, dy (used
// when label is 1), the true yaw bin and the period (in bins) of the mesh's yaw
// symmetry: the target yaw distribution is uniform over the bins congruent to the
// true one modulo the period.
struct PoseTarget {
  float label, dx, dy, yaw_bin, period;
};

// Pose queries of the decoder: mesh, instances wanted, first output slot.
struct PoseQuery {
  int mesh, count, first, pad;
};

// hid must hold (n_crops + n_mesh) x 64 floats.
void launch_pose_predict(const Net& net, const PoseParams& P, int n_yaw, int n_crops, int n_mesh,
                         const PosePair* pairs, int n_pairs, float* out, hipStream_t s);
void launch_pose_backward(const Net& net, const PoseParams& P, const PoseParams& G, int n_yaw,
                          int n_crops, int n_mesh, const PosePair* pairs,
                          const PoseTarget* target, int n_pairs, hipStream_t s);
// Per query q: out rows q * n_anchors .. + n_anchors - 1 are its pairs; picks
// `count` anchors by decreasing objectness (ties: lower index), each at least
// nms_m from the earlier picks, and writes (mesh, x, y, theta) per pick.
void launch_pose_decode(const float* out, int n_yaw, int n_anchors, const float2* anchors,
                        float spacing, float nms_m, const PoseQuery* q, int n_q, float4* res,
                        hipStream_t s);

}  // namespace cnn
}  // namespace perch
