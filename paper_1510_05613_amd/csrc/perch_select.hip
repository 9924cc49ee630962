// perch_select.hip -- device-side ranking of a state's children for the learned
// search (arXiv:1510.05613 Sec. IV-C: an inadmissible queue fed by a learned
// heuristic): the k children with the smallest predicted cost (equal predictions
// in index order, -0 equal to +0) become (mesh, pose) candidates for the exact
// evaluation, in that order, without a round trip through the host.  Up to
// kTopkMaxN children one workgroup selects them (radix select plus a rank count);
// beyond that the predictions are sorted with their indices (a stable LSD radix
// sort) and the first k taken.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "perch_internal.h"

namespace perch {

namespace {

__global__ void k_iota(int* idx, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) idx[i] = i;
}

__global__ void k_mask_children(const float* pred, float* masked, int n_poses, int n,
                                MeshMask mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) masked[i] = mask.allow[i / n_poses] ? pred[i] : __builtin_inff();
}

// child index i = (position of the mesh in the list) * P + (position of the pose)
__global__ void k_child_cands(const int* idx_sorted, int k, const int* rest, int n_poses,
                              const int* pose_ids, int2* cands) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const int id = idx_sorted[i];
  cands[i] = make_int2(rest[id / n_poses], pose_ids[id % n_poses]);
}

// Work items of a batched step: ranked candidates of parent slot `slot`.
__global__ void k_items_from_cands(const int2* cands, int k, int slot, int4* items) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) items[i] = make_int4(slot, cands[i].x, cands[i].y, 0);
}

// Work items of a batched step: every child (meshes[u], pose_ids[b]) of parent slot
// `slot`, u < n_meshes, b < n_poses, mesh-major.
__global__ void k_items_all(int slot, MeshList meshes, int n_meshes, const int* pose_ids,
                            int n_poses, int4* items) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)n_meshes * n_poses) return;
  const int u = (int)(i / n_poses), b = (int)(i - (long)u * n_poses);
  items[i] = make_int4(slot, meshes.id[u], pose_ids[b], 0);
}

// Order-preserving map of a float to an unsigned key (negative values flipped,
// positive ones with the sign bit set); -0 maps like +0.
__device__ inline unsigned order_key(float v) {
  unsigned b = __float_as_uint(v);
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Inclusive prefix sum over one 64-lane wavefront.
__device__ inline unsigned wave_incl_scan(unsigned x, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned v = __shfl_up(x, off, 64);
    if (lane >= off) x += v;
  }
  return x;
}

// Adds one to hist[d] for every active lane of the wavefront.  Predictions close in
// value share their leading digits, so most lanes of a pass usually fall in one bin:
// the lanes with the first active lane's digit are counted with one atomic, the
// others add theirs one by one.
__device__ inline void hist_add(unsigned* hist, bool act, unsigned d, int lane) {
  const unsigned long long m = __ballot(act);
  if (m == 0ull) return;
  const int first = __builtin_ctzll(m);
  const unsigned d0 = __shfl(d, first, 64);
  const bool same = act && d == d0;
  const unsigned long long ms = __ballot(same);
  if (lane == first)
    atomicAdd(&hist[d0], (unsigned)__popcll(ms));
  else if (act && !same)
    atomicAdd(&hist[d], 1u);
}

constexpr int kSelThreads = 1024;
constexpr int kSelPer = kTopkMaxN / kSelThreads;  // keys held per thread, in registers

// Selection modes: kSelAll, one workgroup over every child, writes cands; kSelChunk,
// workgroup c over children [c L, c L + L) (L = kTopkMaxN), writes its first k (or
// all of them when fewer) as (key << 32 | child) to buf[c k ..] in rank order,
// sentinel entries (all ones) after them; kSelMerge, one workgroup over the chunks'
// buf entries, writes cands.  The k smallest (key, child) of the children are among
// their chunks' k smallest, and the merge's position order among equal keys is the
// children's index order (chunks cover increasing children, each in rank order), so
// the two levels give what one selection over all children gives.
enum { kSelAll = 0, kSelChunk = 1, kSelMerge = 2 };

// Thread t holds the keys of positions [t*per, t*per + per) of the workgroup's
// range.  Four 8-bit radix-select passes (most significant digit first) find T, the
// k-th smallest key, and how many keys equal to T the first k hold; a block scan of
// the per-thread tie counts gives each tie its position-order rank; the k chosen
// (key, position) pairs go to LDS, and each one's rank among them is its output slot.
template <int MODE>
__global__ void __launch_bounds__(kSelThreads) k_select_topk(
    const float* __restrict__ pred, const unsigned long long* __restrict__ buf_in, int n_poses,
    int n, MeshMask mask, int k, const int* __restrict__ rest, const int* __restrict__ pose_ids,
    int2* __restrict__ cands, unsigned long long* __restrict__ buf_out) {
  __shared__ unsigned hist[256];
  __shared__ unsigned s_wsum[kSelThreads / 64];
  __shared__ unsigned long long s_sel[kTopkMaxK];
  __shared__ unsigned s_prefix, s_krem, s_nsel;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int base = MODE == kSelChunk ? blockIdx.x * kTopkMaxN : 0;  // first child of the range
  const int nl = MODE == kSelChunk ? min(kTopkMaxN, n - base) : n;  // positions in the range
  const int kl = min(k, nl);                                          // keys to select
  const int per = (nl + kSelThreads - 1) / kSelThreads;  // <= kSelPer, checked by the host
  const int i0 = tid * per;
  unsigned r[kSelPer];
#pragma unroll
  for (int j = 0; j < kSelPer; ++j) {
    const int i = i0 + j;
    r[j] = 0xFFFFFFFFu;
    if (j < per && i < nl) {
      if (MODE == kSelMerge) {
        r[j] = (unsigned)(buf_in[i] >> 32);
      } else {
        const int c = base + i;
        r[j] = mask.allow[c / n_poses] ? order_key(pred[c]) : order_key(__builtin_inff());
      }
    }
  }
  if (tid == 0) {
    s_prefix = 0u;
    s_krem = (unsigned)kl;
    s_nsel = 0u;
  }
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    if (tid < 256) hist[tid] = 0u;
    __syncthreads();
    const unsigned pre = s_prefix;
    const unsigned hmask = pass ? (0xFFFFFFFFu << (shift + 8)) : 0u;
#pragma unroll
    for (int j = 0; j < kSelPer; ++j)
      hist_add(hist, j < per && i0 + j < nl && (r[j] & hmask) == pre, (r[j] >> shift) & 255u, lane);
    __syncthreads();
    if (wave == 0) {
      const unsigned h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2],
                     h3 = hist[4 * lane + 3];
      const unsigned sum = h0 + h1 + h2 + h3;
      const unsigned incl = wave_incl_scan(sum, lane);
      const unsigned krem = s_krem;
      unsigned acc = incl - sum;
      if (acc < krem && incl >= krem) {  // exactly one lane holds the k-th key's digit
        const unsigned h[4] = {h0, h1, h2, h3};
        int b = 0;
        while (acc + h[b] < krem) acc += h[b++];
        s_prefix = pre | ((unsigned)(4 * lane + b) << shift);
        s_krem = krem - acc;
      }
    }
    __syncthreads();
  }
  const unsigned T = s_prefix, krem = s_krem;
  unsigned ties = 0;
#pragma unroll
  for (int j = 0; j < kSelPer; ++j) ties += (j < per && i0 + j < nl && r[j] == T) ? 1u : 0u;
  const unsigned wincl = wave_incl_scan(ties, lane);
  if (lane == 63) s_wsum[wave] = wincl;
  __syncthreads();
  unsigned tb = wincl - ties;
  for (int w = 0; w < wave; ++w) tb += s_wsum[w];
#pragma unroll
  for (int j = 0; j < kSelPer; ++j) {
    const int i = i0 + j;
    if (j >= per || i >= nl) continue;
    bool take = r[j] < T;
    if (r[j] == T) take = tb++ < krem;
    if (take) s_sel[atomicAdd(&s_nsel, 1u)] = ((unsigned long long)r[j] << 32) | (unsigned)i;
  }
  __syncthreads();
  for (int t = tid; t < k; t += kSelThreads) {
    if (MODE == kSelChunk && t >= kl) {  // fewer children than k in this chunk
      buf_out[(size_t)blockIdx.x * k + t] = ~0ull;
      continue;
    }
    const unsigned long long me = s_sel[t];
    int rank = 0;
    for (int q = 0; q < kl; ++q) rank += s_sel[q] < me ? 1 : 0;
    const unsigned pos = (unsigned)(me & 0xFFFFFFFFull);
    if (MODE == kSelChunk) {
      buf_out[(size_t)blockIdx.x * k + rank] = (me & 0xFFFFFFFF00000000ull) | (unsigned)(base + pos);
    } else {
      const int id = MODE == kSelMerge ? (int)(unsigned)(buf_in[pos] & 0xFFFFFFFFull) : (int)pos;
      cands[rank] = make_int2(rest[id / n_poses], pose_ids[id % n_poses]);
    }
  }
}

}  // namespace

bool launch_select_topk(const float* pred, int n_poses, int n_meshes, MeshMask mask, int k,
                        const int* rest, const int* pose_ids, int2* cands, hipStream_t s) {
  const long n = (long)n_poses * n_meshes;
  if (n <= 0 || n > kTopkMaxN || k <= 0 || k > kTopkMaxK || k > n) return false;
  hipLaunchKernelGGL(k_select_topk<kSelAll>, dim3(1), dim3(kSelThreads), 0, s, pred, nullptr,
                     n_poses, (int)n, mask, k, rest, pose_ids, cands, nullptr);
  return true;
}

int select_chunks(long n, int k) {
  if (n <= kTopkMaxN || k <= 0 || k > kTopkMaxK || k > n) return 0;
  const long c = (n + kTopkMaxN - 1) / kTopkMaxN;
  return c * k <= kTopkMaxN ? (int)c : 0;
}

void launch_select_topk2(const float* pred, int n_poses, int n_meshes, MeshMask mask, int k,
                         const int* rest, const int* pose_ids, int2* cands,
                         unsigned long long* buf, hipStream_t s) {
  const int n = n_poses * n_meshes, c = select_chunks(n, k);
  hipLaunchKernelGGL(k_select_topk<kSelChunk>, dim3(c), dim3(kSelThreads), 0, s, pred, nullptr,
                     n_poses, n, mask, k, nullptr, nullptr, nullptr, buf);
  hipLaunchKernelGGL(k_select_topk<kSelMerge>, dim3(1), dim3(kSelThreads), 0, s, nullptr, buf,
                     n_poses, c * k, mask, k, rest, pose_ids, cands, nullptr);
}

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

void launch_mask_children(const float* pred, float* masked, int n_poses, int n_meshes,
                          MeshMask mask, hipStream_t s) {
  const int n = n_poses * n_meshes;
  if (n > 0)
    hipLaunchKernelGGL(k_mask_children, dim3((n + 255) / 256), dim3(256), 0, s, pred, masked,
                       n_poses, n, mask);
}

void launch_child_cands(const int* idx_sorted, int k, const int* rest, int n_poses,
                        const int* pose_ids, int2* cands, hipStream_t s) {
  if (k > 0)
    hipLaunchKernelGGL(k_child_cands, dim3((k + 255) / 256), dim3(256), 0, s, idx_sorted, k,
                       rest, n_poses, pose_ids, cands);
}

void launch_items_from_cands(const int2* cands, int k, int slot, int4* items, hipStream_t s) {
  if (k > 0)
    hipLaunchKernelGGL(k_items_from_cands, dim3((k + 255) / 256), dim3(256), 0, s, cands, k,
                       slot, items);
}

void launch_items_all(int slot, const MeshList& meshes, int n_meshes, const int* pose_ids,
                      int n_poses, int4* items, hipStream_t s) {
  const long n = (long)n_meshes * n_poses;
  if (n > 0)
    hipLaunchKernelGGL(k_items_all, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, slot,
                       meshes, n_meshes, pose_ids, n_poses, items);
}

}  // namespace perch
