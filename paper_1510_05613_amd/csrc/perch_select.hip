// perch_select.hip -- device-side ranking of a state's children for the learned
// search (arXiv:1510.05613 Sec. IV-C: an inadmissible queue fed by a learned
// heuristic): the predicted costs are sorted with their child indices (a stable
// LSD radix sort, so equal predictions keep index order) and the first k indices
// become (mesh, pose) candidates for the exact evaluation, without a round trip
// through the host.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "perch_internal.h"

namespace perch {

namespace {

__global__ void k_iota(int* idx, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) idx[i] = i;
}

__global__ void k_mask_children(float* pred, int n_poses, int n, MeshMask mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !mask.allow[i / n_poses]) pred[i] = __builtin_inff();
}

// child index i = (position of the mesh in the list) * P + (position of the pose)
__global__ void k_child_cands(const int* idx_sorted, int k, const int* rest, int n_poses,
                              const int* pose_ids, int2* cands) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const int id = idx_sorted[i];
  cands[i] = make_int2(rest[id / n_poses], pose_ids[id % n_poses]);
}

}  // namespace

size_t select_temp_bytes(int n) {
  size_t bytes = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const float*)nullptr,
                                           (float*)nullptr, (const int*)nullptr, (int*)nullptr,
                                           n);
  return bytes;
}

hipError_t sort_predictions(void* temp, size_t temp_bytes, const float* keys, float* keys_sorted,
                            const int* idx, int* idx_sorted, int n, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, keys_sorted, idx, idx_sorted,
                                            n, 0, 32, s);
}

void launch_iota(int* idx, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_iota, dim3((n + 255) / 256), dim3(256), 0, s, idx, n);
}

void launch_mask_children(float* pred, int n_poses, int n_meshes, MeshMask mask, hipStream_t s) {
  const int n = n_poses * n_meshes;
  if (n > 0)
    hipLaunchKernelGGL(k_mask_children, dim3((n + 255) / 256), dim3(256), 0, s, pred, n_poses, n,
                       mask);
}

void launch_child_cands(const int* idx_sorted, int k, const int* rest, int n_poses,
                        const int* pose_ids, int2* cands, hipStream_t s) {
  if (k > 0)
    hipLaunchKernelGGL(k_child_cands, dim3((k + 255) / 256), dim3(256), 0, s, idx_sorted, k,
                       rest, n_poses, pose_ids, cands);
}

}  // namespace perch
