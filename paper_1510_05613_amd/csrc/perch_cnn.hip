// perch_cnn.hip -- learned successor-cost network: inference and training kernels
// for gfx950 (bfloat16 MFMA, FP32 accumulation).
//
// The paper proposes learned, possibly inadmissible heuristics for its
// multi-heuristic search (arXiv:1510.05613 Sec. IV-C and the conclusion).  This
// network predicts log(1 + c(s, s')) of a successor from a 64 x 64 x 2 depth crop
// (observed depth and the parent's composite, relative to the table point under
// the candidate), the candidate's mesh and its yaw:
//   4 x [3x3 conv, 32 channels, ReLU] (strides 1, 2, 2, 2) -> mean over the 8 x 8
//   map and over its centre 2 x 2 -> [64 + 16-d mesh embedding + cos, sin yaw]
//   -> 64 (ReLU) -> 1.
// Convolutions are implicit GEMMs on v_mfma_f32_32x32x16_bf16: forward (pixels x
// out-channels), input gradient (pixels x in-channels) and weight gradient
// (out-channels x taps*in-channels, reduced over pixels).  Activations and the
// gradients fed to the MFMAs are bfloat16; accumulation, pooling, the head, the
// loss and Adam are FP32.  Tensors are NHWC.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "perch_cnn.h"

namespace perch {
namespace cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// bfloat16 bits of f, rounded to nearest even (inputs are finite)
__device__ __forceinline__ bf16_t f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// Row of the 32 x 32 MFMA result held in accumulator element e of lane l:
// 8 (e / 4) + 4 (l / 32) + e % 4; its column is l % 32.
__device__ __forceinline__ int acc_row(int e, int lane) {
  return 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
}

// ---------------------------------------------------------------------------
// crops
// ---------------------------------------------------------------------------

// bfloat16(lo) | bfloat16(hi) << 16, rounded to nearest even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ unsigned pack_bf16(float lo, float hi) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(unsigned, v);
}

// The two channels of a crop sample at a pixel: (z - zref) / 0.25 clipped to
// [-1, 1] for the observed depth z (1 where z <= 0: no return) and for the parent
// depth with float bits k (1 where +inf: no parent point); 1 outside the image.
// Shared by k_crops and the crops k_conv12_fwd samples itself.
__device__ __forceinline__ unsigned crop_sample(float z, unsigned k, bool in_image, float zref) {
  const float a = in_image && z > 0.0f
                      ? __builtin_amdgcn_fmed3f((z - zref) * 4.0f, -1.0f, 1.0f) : 1.0f;
  const float b = in_image && k != 0x7f800000u
                      ? __builtin_amdgcn_fmed3f((__uint_as_float(k) - zref) * 4.0f, -1.0f, 1.0f)
                      : 1.0f;
  return pack_bf16(a, b);
}

// One crop per workgroup: 64 x 64 samples every `step` pixels around (u0, v0);
// channel 0 the observed depth, channel 1 the parent composite, both as (z - zref)
// / 0.25 clipped to [-1, 1], +1 where there is no return / no parent point or
// outside the image.
__global__ void __launch_bounds__(1024)
    k_crops(const float* obs, const unsigned* pdepth, int W, int H, const CropDesc* desc, int n,
            bf16_t* out) {
  const int c = blockIdx.x;
  if (c >= n) return;
  const CropDesc d = desc[c];
  const int st = d.step > 1 ? d.step : 1;
  unsigned* o = reinterpret_cast<unsigned*>(out) + (size_t)c * kCrop * kCrop;  // both channels
#pragma unroll 4
  for (int t = threadIdx.x; t < kCrop * kCrop; t += blockDim.x) {
    const int cy = t / kCrop, cx = t % kCrop;
    const int u = d.u0 + (cx - kCrop / 2) * st, v = d.v0 + (cy - kCrop / 2) * st;
    const bool inb = u >= 0 && u < W && v >= 0 && v < H;
    const size_t px = inb ? (size_t)v * W + u : 0;
    o[t] = crop_sample(obs[px], pdepth ? pdepth[px] : 0x7f800000u, inb, d.zref);
  }
}

// ---------------------------------------------------------------------------
// convolution forward: out[m][co] = relu(b[co] + sum_k patch[m][k] W[co][k])
// ---------------------------------------------------------------------------

template <int CIN>
struct KDim {
  static constexpr int K = 9 * CIN;                  // taps x input channels
  static constexpr int KP = (K + 15) / 16 * 16;      // padded to the MFMA depth
  static constexpr int LDSROW = KP + 8;              // LDS row stride (bank spread)
};

// Eight consecutive k of the im2col patch of output pixel (n, oy, ox); branch-free
// (out-of-range reads are redirected to element 0 and zeroed).
template <int CIN, int S, int HIN>
__device__ __forceinline__ uint4 patch8(const bf16_t* __restrict__ in, bool valid, int n, int oy,
                                        int ox, int k0) {
  if (CIN % 8 == 0) {
    const int tap = k0 / CIN, ci0 = k0 % CIN;
    const int iy = oy * S + tap / 3 - 1, ix = ox * S + tap % 3 - 1;
    const bool ok = valid && tap < 9 && iy >= 0 && iy < HIN && ix >= 0 && ix < HIN;
    const size_t off = ok ? (((size_t)n * HIN + iy) * HIN + ix) * CIN + ci0 : 0;
    const uint4 v = *reinterpret_cast<const uint4*>(in + off);
    return ok ? v : make_uint4(0u, 0u, 0u, 0u);
  } else if (CIN == 2) {
    // four taps of both channels: one 4-byte load per tap (k = 2 tap + ci)
    unsigned v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int tap = k0 / 2 + q;
      const int iy = oy * S + tap / 3 - 1, ix = ox * S + tap % 3 - 1;
      const bool ok = valid && tap < 9 && iy >= 0 && iy < HIN && ix >= 0 && ix < HIN;
      const size_t off = ok ? (((size_t)n * HIN + iy) * HIN + ix) * 2 : 0;
      const unsigned x = *reinterpret_cast<const unsigned*>(in + off);
      v[q] = ok ? x : 0u;
    }
    return make_uint4(v[0], v[1], v[2], v[3]);
  } else {
    unsigned v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 + q;
      const int tap = k / CIN, ci = k % CIN;
      const int iy = oy * S + tap / 3 - 1, ix = ox * S + tap % 3 - 1;
      const bool ok = valid && k < 9 * CIN && iy >= 0 && iy < HIN && ix >= 0 && ix < HIN;
      const size_t off = ok ? (((size_t)n * HIN + iy) * HIN + ix) * CIN + ci : 0;
      const unsigned x = in[off];
      v[q] = ok ? x : 0u;
    }
    return make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16),
                      v[6] | (v[7] << 16));
  }
}

// Forward tiles are computed transposed, out^T = W x patch^T: the weights are the
// MFMA's A operand (lane l: W[l % 32][16 kc + 8 (l / 32) .. + 8]) and the im2col
// patches its B operand (lane l: pixel l % 32), so lane l ends with pixel l % 32's
// channels 8 g + 4 (l / 32) + i in accumulator element 4 g + i (g, i = 0..3).  The
// accumulation chain starts from the bias, and the ReLU and bfloat16 rounding give
// four packed 8-byte stores per lane.

// The bias of the lane's accumulator elements: acc[4 g + i] = b[8 g + 4 (lane / 32) + i]
// (b: 16-byte aligned, 32 channel biases).
__device__ __forceinline__ f32x16 bias_acc(const float* b, int lane) {
  const int h4 = 4 * (lane >> 5);
  f32x16 a;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const float4 v = *reinterpret_cast<const float4*>(b + 8 * g + h4);
    a[4 * g] = v.x;
    a[4 * g + 1] = v.y;
    a[4 * g + 2] = v.z;
    a[4 * g + 3] = v.w;
  }
  return a;
}

// bf16(relu(lo)) | bf16(relu(hi)) << 16: the ReLU after the rounding, as a signed
// 16-bit max with 0 (a negative value, -0 included, has its sign bit set), gives
// the same bits as rounding the ReLU's result.
__device__ __forceinline__ unsigned pack_relu_bf16(float lo, float hi) {
  typedef short short2_t __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  typedef float float2_t __attribute__((ext_vector_type(2)));
  const float2_t f = {lo, hi};
  const short2_t v = __builtin_bit_cast(short2_t, __builtin_convertvector(f, bf16x2_t));
  const short2_t z = {0, 0};
  return __builtin_bit_cast(unsigned, __builtin_elementwise_max(v, z));
}

// dst[8 g + 4 (lane / 32) .. + 4] of the lane's pixel = bf16(relu(acc)).
template <typename Ptr>
__device__ __forceinline__ void store_relu_bf16(const f32x16& acc, int lane, Ptr dst) {
  const int h4 = 4 * (lane >> 5);
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const uint2 v = make_uint2(pack_relu_bf16(acc[4 * g], acc[4 * g + 1]),
                               pack_relu_bf16(acc[4 * g + 2], acc[4 * g + 3]));
    *reinterpret_cast<uint2*>(dst + 8 * g + h4) = v;
  }
}

// An empty use of v's registers: the compiler waits for v's load here.
__device__ __forceinline__ void settle(const uint4& v) {
  asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
}

// Workgroup barrier ordering LDS accesses only: global stores stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ f32x16 mfma_bf16(uint4 a, uint4 b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a), as_bf16x8(b), c, 0, 0, 0);
}

// Each wave keeps the 32 output channels' weights as MFMA fragments in registers
// (KP / 16 of them, loaded once), then walks 32-pixel output tiles tile = wave,
// wave + total waves, ...: per tile KP / 16 MFMA steps whose patch fragments are read
// straight from the input, in increasing k as a single accumulation chain (the same
// sums in the same order for any grid).
template <int CIN, int S, int HIN>
__global__ void __launch_bounds__(256)
    k_conv_fwd(const bf16_t* __restrict__ in, const bf16_t* __restrict__ Wb,
               const float* __restrict__ bias, bf16_t* __restrict__ out, int n_img) {
  using D = KDim<CIN>;
  constexpr int HO = HIN / S, NPIX = HO * HO, NK = D::KP / 16;
  __shared__ __align__(16) float sb[kC];
  if (threadIdx.x < kC) sb[threadIdx.x] = bias[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int co = lane & 31, kh = 8 * (lane >> 5);
  const int total = n_img * NPIX;
  const int n_tiles = (total + 31) / 32;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int n_waves = gridDim.x * 4;
  if (wave >= n_tiles) return;
  uint4 wf[NK];  // W[co][16 kc + kh .. + 8] (rows of KP elements, 16-byte aligned)
#pragma unroll
  for (int kc = 0; kc < NK; ++kc)
    wf[kc] = *reinterpret_cast<const uint4*>(Wb + (size_t)co * D::KP + kc * 16 + kh);
  for (int t = wave; t < n_tiles; t += n_waves) {
    const int m = t * 32 + (lane & 31);
    const bool mv = m < total;
    const int n = m / NPIX, pix = m % NPIX, oy = pix / HO, ox = pix % HO;
    f32x16 acc = bias_acc(sb, lane);
#pragma unroll
    for (int kc = 0; kc < NK; ++kc)
      acc = mfma_bf16(wf[kc], patch8<CIN, S, HIN>(in, mv, n, oy, ox, kc * 16 + kh), acc);
    if (mv) store_relu_bf16(acc, lane, out + (size_t)m * kC);
  }
}

// ---------------------------------------------------------------------------
// inference: conv1 and conv2 fused over bands of conv2 output rows
// ---------------------------------------------------------------------------

// conv1's 64 x 64 x 32 activation never reaches HBM: a work item is one crop's band
// of kBandRows conv2 output rows.  The item's 2 kBandRows + 3 input rows are staged
// in LDS (loaded during the previous item), conv1 computes the 2 kBandRows + 1 rows
// that the band's stride-2 3 x 3 windows read into an LDS band, and conv2 reads its
// patches from there.  Both LDS tiles carry zero padding (a column left of the image,
// and right of it for the input; conv1's row -1), so no patch read is masked.
// Tiles, fragments, the accumulation chain, bias, ReLU and rounding are those of
// k_conv_fwd for each layer (a conv1 tile is half a row, a conv2 tile one output
// row), so the output equals the two unfused launches bit for bit.  Work items are
// taken grid-stride; each wave loads both layers' weight fragments once.
constexpr int kBandRows = 4;                // conv2 output rows per work item (one per wave)
constexpr int kBandIn = 2 * kBandRows + 1;  // conv1 rows a band reads
constexpr int kInRows = kBandIn + 2;        // input rows those read
constexpr int kInSlots = 72;                // input row: col x at slot x + 4, pads at 3 and 68
constexpr int kBandSlots = kCrop + 1;       // band row: col x at slot x + 1, pad at 0
constexpr int kPixStride = kC + 8;          // bfloat16 per LDS pixel (80 B spreads the banks)
constexpr int kConv12Items = kCrop / 2 / kBandRows;  // work items per crop

// Where k_conv12_fwd's input comes from: a crop tensor, or (IMG) the observation and
// the parent composite, sampled per crop descriptor exactly as k_crops does.
struct CropSource {
  const bf16_t* crops;     // [n][64][64][2] (without IMG)
  const float* obs;        // H x W observed depth (IMG)
  const unsigned* pdepth;  // H x W parent composite, float bits, +inf empty (IMG)
  int W, H;
  const CropDesc* desc;    // one per crop (IMG)
};

template <bool IMG>
__global__ void __launch_bounds__(256)
    k_conv12_fwd(const CropSource src, const bf16_t* __restrict__ W1,
                 const float* __restrict__ b1, const bf16_t* __restrict__ W2,
                 const float* __restrict__ b2, bf16_t* __restrict__ out, int n_img) {
  constexpr int NK1 = KDim<2>::KP / 16, KP1 = KDim<2>::KP;
  constexpr int NK2 = KDim<kC>::KP / 16, KP2 = KDim<kC>::KP;
  constexpr int H2 = kCrop / 2;
  constexpr int IN_U4 = kInRows * kCrop * 2 * 2 / 16;  // 16-byte pieces of an item's input
  __shared__ __align__(16) unsigned sin[kInRows * kInSlots];  // two bfloat16 channels per slot
  __shared__ __align__(16) bf16_t band[kBandIn * kBandSlots * kPixStride];
  __shared__ __align__(16) float sb[kC];  // conv2's bias
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int co = lane & 31, kh = 8 * (lane >> 5), h = lane >> 5;
  const int tap_base = h ? kInSlots + 1 : 0, tap_2 = h ? kInSlots - 1 : 2;
  if (tid < kC) sb[tid] = b2[tid];
  f32x16 bias1;  // conv1's bias, kept in registers for its eighteen tiles per item
#pragma unroll
  for (int e = 0; e < 16; ++e) bias1[e] = b1[8 * (e >> 2) + 4 * h + (e & 3)];
  for (int r = tid; r < kInRows; r += blockDim.x) sin[r * kInSlots + 3] = sin[r * kInSlots + 68] = 0u;
  for (int i = tid; i < kBandIn * kPixStride / 8; i += blockDim.x)  // slot 0 of every band row
    *reinterpret_cast<uint4*>(band + (i / (kPixStride / 8)) * kBandSlots * kPixStride +
                              8 * (i % (kPixStride / 8))) = make_uint4(0u, 0u, 0u, 0u);
  uint4 w1[NK1], w2[NK2];
#pragma unroll
  for (int kc = 0; kc < NK1; ++kc)
    w1[kc] = *reinterpret_cast<const uint4*>(W1 + (size_t)co * KP1 + kc * 16 + kh);
#pragma unroll
  for (int kc = 0; kc < NK2; ++kc)
    w2[kc] = *reinterpret_cast<const uint4*>(W2 + (size_t)co * KP2 + kc * 16 + kh);
  const int n_items = n_img * kConv12Items;
  // Four samples (16 bytes) of item `it`'s input rows, issued by every thread: a
  // 16-byte load clamped into the crop tensor, or (IMG) the four pixels' observed and
  // parent depths, clamped into the image; `ok` says whether the row is the crop's
  // (else conv1's zero padding).  The samples are formed when they go to LDS.
  uint4 pre;
  float pz[4], zref = 0.0f;
  unsigned pk[4], inimg = 0u;
  bool pre_ok;
  auto fetch = [&](int it) {
    const int itc = min(it, n_items - 1), n = itc / kConv12Items;
    const int yi = 2 * (itc % kConv12Items) * kBandRows - 2 + (tid % IN_U4) / 16;
    const int yc = min(max(yi, 0), kCrop - 1);
    pre_ok = it < n_items && yi == yc;
    if constexpr (IMG) {
      const CropDesc d = src.desc[n];
      const int st = d.step > 1 ? d.step : 1;
      const int v = d.v0 + (yc - kCrop / 2) * st;
      zref = d.zref;
      inimg = 0u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int u = d.u0 + (4 * (tid % 16) + q - kCrop / 2) * st;
        const bool inb = u >= 0 && u < src.W && v >= 0 && v < src.H;
        const size_t px = inb ? (size_t)v * src.W + u : 0;
        pz[q] = src.obs[px];
        pk[q] = src.pdepth[px];
        inimg |= inb ? 1u << q : 0u;
      }
    } else {
      pre = *reinterpret_cast<const uint4*>(
          src.crops + (((size_t)n * kCrop + yc) * kCrop + 4 * (tid % 16)) * 2);
    }
  };
  fetch(blockIdx.x);
  // the weight fragments land before the loop, whose waits then count only its own
  // loads and stores (a weight load pending at the loop entry would make the
  // compiler wait for every outstanding store in each iteration)
#pragma unroll
  for (int kc = 0; kc < NK1; ++kc) settle(w1[kc]);
#pragma unroll
  for (int kc = 0; kc < NK2; ++kc) settle(w2[kc]);
#pragma unroll
  for (int e = 0; e < 16; ++e) asm volatile("" ::"v"(bias1[e]));
  // the input of the next item goes to LDS during conv2 (conv1 is done with it),
  // long after its load was issued
  auto stage = [&]() {
    if (tid < IN_U4) {
      uint4 v = pre;
      if constexpr (IMG)
        v = make_uint4(crop_sample(pz[0], pk[0], inimg & 1u, zref),
                       crop_sample(pz[1], pk[1], inimg & 2u, zref),
                       crop_sample(pz[2], pk[2], inimg & 4u, zref),
                       crop_sample(pz[3], pk[3], inimg & 8u, zref));
      *reinterpret_cast<uint4*>(sin + (tid / 16) * kInSlots + 4 + 4 * (tid % 16)) =
          pre_ok ? v : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  stage();
  for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int n = item / kConv12Items, r0 = (item % kConv12Items) * kBandRows;
    const int y0 = 2 * r0 - 1;  // conv1 row of band row 0
    lds_barrier();
    fetch(item + gridDim.x);
    // conv1: two 32-pixel tiles per band row; row -1 is conv2's zero padding
    for (int t = wave; t < 2 * kBandIn; t += 4) {
      const int yl = t >> 1, ox = (t & 1) * 32 + (lane & 31);
      bf16_t* dst = band + (yl * kBandSlots + ox + 1) * kPixStride;
      if (y0 + yl < 0) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
          *reinterpret_cast<uint2*>(dst + 8 * g + 4 * h) = make_uint2(0u, 0u);
        continue;
      }
      // tap (ky, kx) of input (y0 + yl + ky - 1, ox + kx - 1): sin row yl + ky, slot
      // ox + kx + 3.  k = 2 tap + channel: lanes 0-31 hold taps 0-3 and 8 (offsets
      // 0, 1, 2, 72, 146), lanes 32-63 taps 4-7 (73, 74, 144, 145)
      const unsigned* sp = sin + yl * kInSlots + ox + 3;
      const unsigned* sq = sp + tap_base;
      const uint4 p0 = make_uint4(sq[0], sq[1], sq[tap_2], sq[kInSlots]);
      const unsigned t8 = sp[2 * kInSlots + 2];
      const uint4 p1 = make_uint4(h ? 0u : t8, 0u, 0u, 0u);
      f32x16 acc = bias1;
      acc = mfma_bf16(w1[0], p0, acc);
      acc = mfma_bf16(w1[1], p1, acc);
      store_relu_bf16(acc, lane, dst);
    }
    lds_barrier();
    stage();
    // conv2: output row r0 + wave; tap (ky, kx) of pixel ox reads band row
    // 2 wave + ky, slot 2 ox + kx
    {
      const int oy = r0 + wave, ox = lane & 31;
      const bf16_t* bp = band + (2 * wave * kBandSlots + 2 * ox) * kPixStride + kh;
      f32x16 acc = bias_acc(sb, lane);
#pragma unroll
      for (int kc = 0; kc < NK2; ++kc) {
        const int tap = kc / 2, ky = tap / 3, kx = tap % 3;
        const uint4 a = *reinterpret_cast<const uint4*>(
            bp + (ky * kBandSlots + kx) * kPixStride + 16 * (kc % 2));
        acc = mfma_bf16(w2[kc], a, acc);
      }
      store_relu_bf16(acc, lane, out + (((size_t)n * H2 + oy) * H2 + ox) * kC);
    }
  }
}

// conv3, conv4 and the pooling fused per crop for inference: a3 (16 x 16) and a4
// (8 x 8) stay in LDS, only the 64 pooled features are written.  conv3's tiles
// (two output rows, one per wave of the 512-thread workgroup) and conv4's (four
// rows) are k_conv_fwd's, the pooling sums in k_pool_fwd's order, so the features
// equal the unfused launches' bit for bit.  Both layers' weight fragments are read
// from LDS copies, which leaves a wave the registers to issue all eighteen patch
// loads of its conv3 tile at once.  a3 in LDS has a zero row and column before the
// image (slot (y + 1) 17 + x + 1).
//
// HEAD: also the first head layer's per-crop term of every hidden unit from the
// pooled features, hid[n][r] = sum_i hW1[r][i] feat[n][i], and (workgroups m <
// n_mesh) the per-mesh term hid[n_img + m][r] = hb1[r] + sum_e hW1[r][64 + e]
// emb[m][e], in k_head_parts' order.
constexpr int kConv34Threads = 512;

template <bool HEAD>
__global__ void __launch_bounds__(kConv34Threads)
    k_conv34_pool(const bf16_t* __restrict__ a2, const bf16_t* __restrict__ W3,
                  const float* __restrict__ b3, const bf16_t* __restrict__ W4,
                  const float* __restrict__ b4, float* __restrict__ feat, int n_img,
                  const Params P, int n_mesh, float* __restrict__ hid) {
  constexpr int NK = KDim<kC>::KP / 16, KP = KDim<kC>::KP, WROW = KP + 8;
  __shared__ __align__(16) bf16_t s3[17 * 17 * kPixStride];
  __shared__ __align__(16) bf16_t s4[8 * 8 * kC];
  __shared__ __align__(16) bf16_t sw[2][kC * WROW];
  __shared__ __align__(16) float sb[2 * kC];
  __shared__ float sfeat[kFeat];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int co = lane & 31, kh = 8 * (lane >> 5);
  if (HEAD && tid < kHid)
    for (int m = blockIdx.x; m < n_mesh; m += gridDim.x) {
      const float* w = P.hW1 + tid * kIn + kFeat;
      float z = P.hb1[tid];
      for (int e = 0; e < kEmb; ++e) z = fmaf(w[e], P.emb[m * kEmb + e], z);
      hid[(n_img + m) * kHid + tid] = z;
    }
  if (tid < 2 * kC) sb[tid] = tid < kC ? b3[tid] : b4[tid - kC];
  for (int i = tid; i < 2 * kC * KP / 8; i += blockDim.x) {
    const int l = i / (kC * KP / 8), j = i % (kC * KP / 8), r = j / (KP / 8), c8 = j % (KP / 8);
    *reinterpret_cast<uint4*>(&sw[l][r * WROW + c8 * 8]) =
        *reinterpret_cast<const uint4*>((l ? W4 : W3) + (size_t)r * KP + c8 * 8);
  }
  for (int i = tid; i < 33 * kPixStride / 8; i += blockDim.x) {  // row 0 and column 0
    const int slot = i / (kPixStride / 8), q = i % (kPixStride / 8);
    const int sl = slot < 17 ? slot : (slot - 16) * 17;
    *reinterpret_cast<uint4*>(s3 + sl * kPixStride + 8 * q) = make_uint4(0u, 0u, 0u, 0u);
  }
  lds_barrier();
  const bf16_t* wrow3 = &sw[0][co * WROW + kh];
  const bf16_t* wrow4 = &sw[1][co * WROW + kh];
  for (int n = blockIdx.x; n < n_img; n += gridDim.x) {
    // conv3: tile `wave` (pixels 32 wave ..), patches from a2 in global memory
    {
      const int m = wave * 32 + (lane & 31), oy = m / 16, ox = m % 16;
      uint4 pf[NK];
#pragma unroll
      for (int kc = 0; kc < NK; ++kc) pf[kc] = patch8<kC, 2, 32>(a2, true, n, oy, ox, kc * 16 + kh);
      f32x16 acc = bias_acc(sb, lane);
#pragma unroll
      for (int kc = 0; kc < NK; ++kc)
        acc = mfma_bf16(*reinterpret_cast<const uint4*>(wrow3 + kc * 16), pf[kc], acc);
      store_relu_bf16(acc, lane, s3 + ((oy + 1) * 17 + ox + 1) * kPixStride);
    }
    lds_barrier();
    // conv4: two tiles; tap (ky, kx) of pixel (oy, ox) reads slot (2 oy + ky) 17 + 2 ox + kx
    if (wave < 2) {
      const int m = wave * 32 + (lane & 31), oy = m / 8, ox = m % 8;
      const bf16_t* bp = s3 + (2 * oy * 17 + 2 * ox) * kPixStride + kh;
      f32x16 acc = bias_acc(sb + kC, lane);
#pragma unroll
      for (int kc = 0; kc < NK; ++kc) {
        const int tap = kc / 2, ky = tap / 3, kx = tap % 3;
        const uint4 a = *reinterpret_cast<const uint4*>(bp + (ky * 17 + kx) * kPixStride + 16 * (kc % 2));
        acc = mfma_bf16(*reinterpret_cast<const uint4*>(wrow4 + kc * 16), a, acc);
      }
      store_relu_bf16(acc, lane, s4 + m * kC);
    }
    lds_barrier();
    // pooling (one lane per channel); s4 is rewritten only after the next crop's
    // first barrier, which these lanes reach after this loop
    if (tid < kC) {
      float sm = 0.0f, sc = 0.0f;
      for (int p = 0; p < 64; ++p) {
        const float v = bf2f(s4[p * kC + tid]);
        sm += v;
        const int y = p / 8, x = p % 8;
        if (y >= 3 && y <= 4 && x >= 3 && x <= 4) sc += v;
      }
      feat[n * kFeat + tid] = sm / 64.0f;
      feat[n * kFeat + kC + tid] = sc / 4.0f;
      if (HEAD) {
        sfeat[tid] = sm / 64.0f;
        sfeat[kC + tid] = sc / 4.0f;
      }
    }
    if (HEAD) {
      // sfeat is rewritten only after the next crop's first two barriers
      lds_barrier();
      if (tid < kHid) {
        const float* w = P.hW1 + tid * kIn;
        float z = 0.0f;
        for (int i = 0; i < kFeat; ++i) z = fmaf(w[i], sfeat[i], z);
        hid[n * kHid + tid] = z;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// convolution input gradient: din[m][ci] = mask(m, ci) sum_{tap, co} dpre[o(m,tap)][co] W[co][tap][ci]
// ---------------------------------------------------------------------------

// The layers with an input gradient have stride 2, so an input pixel (iy, ix)
// receives from tap (ky, kx) only when iy + 1 - ky and ix + 1 - kx are even: one
// tap row for even iy (ky = 1), two for odd iy (ky = 0, 2), and the same for the
// columns.  Tiles therefore hold 32 pixels of one parity class (iy % 2, ix % 2) of
// one image, at (iy, ix) = (2 a + py, 2 b + px) for 32 consecutive (a, b), and run
// the MFMAs of their 1, 2 or 4 taps only (the taps that only add zeros are left out;
// the sums keep the increasing tap order).
template <int S, int HIN>
__global__ void __launch_bounds__(256)
    k_conv_dgrad(const bf16_t* __restrict__ dpre, const bf16_t* __restrict__ Wb,
                 const bf16_t* __restrict__ act_in, bf16_t* __restrict__ din, int n_img) {
  static_assert(S == 2, "input gradients of stride-2 layers only");
  constexpr int HO = HIN / 2, CLS = HO * HO, K = 9 * kC, ROW = K + 8;
  constexpr int TPC = CLS / 32;  // tiles per (image, parity class)
  static_assert(CLS % 32 == 0, "a parity class holds whole tiles");
  __shared__ __align__(16) bf16_t wt[kC * ROW];  // wt[ci][tap * 32 + co]
  for (int i = threadIdx.x; i < kC * K; i += blockDim.x) {
    const int co = i / K, r = i % K, tap = r / kC, ci = r % kC;
    wt[ci * ROW + tap * kC + co] = Wb[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n_tiles = n_img * 4 * TPC;
  const int kh = 8 * (lane >> 5), ci = lane & 31;
  // tiles grid-stride: the weights staged above serve every tile of the workgroup
  for (int tile = blockIdx.x * 4 + wave; tile < n_tiles; tile += gridDim.x * 4) {
    const int n = tile / (4 * TPC), cls = (tile / TPC) % 4, t = tile % TPC;
    const int py = cls >> 1, px = cls & 1;
    const int q = t * 32 + (lane & 31), a = q / HO, b = q % HO;
    f32x16 acc = {};
    for (int ky = py ? 0 : 1; ky <= (py ? 2 : 1); ky += 2) {
      const int oy = a + (py + 1 - ky) / 2;  // (iy + 1 - ky) / 2
      for (int kx = px ? 0 : 1; kx <= (px ? 2 : 1); kx += 2) {
        const int ox = b + (px + 1 - kx) / 2;
        const bool ok = oy < HO && ox < HO;  // both are >= 0
        const int tap = ky * 3 + kx;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int co0 = 16 * h + kh;
          uint4 av = make_uint4(0u, 0u, 0u, 0u);
          if (ok)
            av = *reinterpret_cast<const uint4*>(dpre + (((size_t)n * HO + oy) * HO + ox) * kC + co0);
          const uint4 bv = *reinterpret_cast<const uint4*>(wt + ci * ROW + tap * kC + co0);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(av), as_bf16x8(bv), acc, 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int qq = t * 32 + acc_row(e, lane);
      const size_t mm = ((size_t)n * HIN + 2 * (qq / HO) + py) * HIN + 2 * (qq % HO) + px;
      const bool on = bf2f(act_in[mm * kC + ci]) > 0.0f;  // ReLU of the previous layer
      din[mm * kC + ci] = f2bf(on ? acc[e] : 0.0f);
    }
  }
}

// ---------------------------------------------------------------------------
// convolution weight gradient: dW[co][k] += sum_m dpre[m][co] patch[m][k]
// ---------------------------------------------------------------------------

// Workgroup (kt, chunk): k columns [32 kt, 32 kt + 32), output pixels
// [chunk * 64 * pw, ...); each wave reduces pw groups of 16 pixels with MFMAs and
// adds its 32 x 32 partial to dW with atomics (pw is chosen so that the atomics
// stay few).  The kt = 0 workgroups also sum the pre-activation gradients they load
// into the bias gradient db[co] = sum_m dpre[m][co].
template <int CIN, int S, int HIN>
__global__ void __launch_bounds__(256)
    k_conv_wgrad(const bf16_t* __restrict__ dpre, const bf16_t* __restrict__ in,
                 float* __restrict__ dW, float* __restrict__ db, int n_img, int pw) {
  constexpr int HO = HIN / S, NPIX = HO * HO, K = 9 * CIN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int total = n_img * NPIX;
  const int kt = blockIdx.x;
  const int pbase = (blockIdx.y * 4 + wave) * 16 * pw;
  if (pbase >= total) return;
  const int co = lane & 31;
  const int kk = kt * 32 + (lane & 31);
  const int tap = kk / CIN, ci = kk % CIN;
  const int ky = tap / 3, kx = tap % 3;
  const int ph = 8 * (lane >> 5);
  f32x16 acc = {};
  float bsum = 0.0f;
  const int n_groups = min(pw, (total - pbase + 15) / 16);
  for (int g = 0; g < n_groups; ++g) {
    const int p0 = pbase + g * 16 + ph;
    unsigned short av[8], bv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int p = p0 + q;
      av[q] = 0;
      bv[q] = 0;
      if (p < total) {
        av[q] = dpre[(size_t)p * kC + co];
        if (kk < K) {
          const int n = p / NPIX, pix = p % NPIX, oy = pix / HO, ox = pix % HO;
          const int iy = oy * S + ky - 1, ix = ox * S + kx - 1;
          if (iy >= 0 && iy < HIN && ix >= 0 && ix < HIN)
            bv[q] = in[(((size_t)n * HIN + iy) * HIN + ix) * CIN + ci];
        }
      }
    }
    if (kt == 0)
#pragma unroll
      for (int q = 0; q < 8; ++q) bsum += bf2f(av[q]);
    uint4 a, b;
    a.x = av[0] | ((unsigned)av[1] << 16); a.y = av[2] | ((unsigned)av[3] << 16);
    a.z = av[4] | ((unsigned)av[5] << 16); a.w = av[6] | ((unsigned)av[7] << 16);
    b.x = bv[0] | ((unsigned)bv[1] << 16); b.y = bv[2] | ((unsigned)bv[3] << 16);
    b.z = bv[4] | ((unsigned)bv[5] << 16); b.w = bv[6] | ((unsigned)bv[7] << 16);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a), as_bf16x8(b), acc, 0, 0, 0);
  }
  if (kt == 0) {
    bsum += __shfl_xor(bsum, 32);  // the two pixel halves of channel co
    if (lane < 32) atomicAdd(&db[co], bsum);
  }
  // D[row = co][col = k]
  const int col = kt * 32 + (lane & 31);
  if (col < K) {
#pragma unroll
    for (int e = 0; e < 16; ++e) atomicAdd(&dW[acc_row(e, lane) * K + col], acc[e]);
  }
}

// ---------------------------------------------------------------------------
// pooling and head
// ---------------------------------------------------------------------------

// feat[n] = [mean over 8 x 8 of a4[n], mean over the centre 2 x 2 of a4[n]]
__global__ void k_pool_fwd(const bf16_t* a4, int n_img, float* feat) {
  const int n = blockIdx.x, c = threadIdx.x;
  if (n >= n_img || c >= kC) return;
  float s = 0.0f, sc = 0.0f;
  for (int p = 0; p < 64; ++p) {
    const float v = bf2f(a4[((size_t)n * 64 + p) * kC + c]);
    s += v;
    const int y = p / 8, x = p % 8;
    if (y >= 3 && y <= 4 && x >= 3 && x <= 4) sc += v;
  }
  feat[n * kFeat + c] = s / 64.0f;
  feat[n * kFeat + kC + c] = sc / 4.0f;
}

__global__ void k_pool_bwd(const float* dfeat, const bf16_t* a4, int n_img, bf16_t* dpre4) {
  const int n = blockIdx.x;
  if (n >= n_img) return;
  for (int t = threadIdx.x; t < 64 * kC; t += blockDim.x) {
    const int p = t / kC, c = t % kC, y = p / 8, x = p % 8;
    float g = dfeat[n * kFeat + c] / 64.0f;
    if (y >= 3 && y <= 4 && x >= 3 && x <= 4) g += dfeat[n * kFeat + kC + c] / 4.0f;
    const bool on = bf2f(a4[(size_t)n * 64 * kC + t]) > 0.0f;
    dpre4[(size_t)n * 64 * kC + t] = f2bf(on ? g : 0.0f);
  }
}

// head input of pair q: [feat (64), emb (16), cos, sin]
__device__ __forceinline__ void head_input(const float* feat, const float* emb, const Pair& pr,
                                           float* h) {
  for (int i = 0; i < kFeat; ++i) h[i] = feat[pr.crop * kFeat + i];
  for (int i = 0; i < kEmb; ++i) h[kFeat + i] = emb[pr.mesh * kEmb + i];
  h[kFeat + kEmb] = pr.cos_yaw;
  h[kFeat + kEmb + 1] = pr.sin_yaw;
}

// A pair is usable when its crop and mesh indices are in range.
__device__ __forceinline__ bool pair_ok(const Pair& pr, int n_crops, int n_mesh) {
  return pr.crop >= 0 && pr.crop < n_crops && pr.mesh >= 0 && pr.mesh < n_mesh;
}

// The first head layer splits into a per-crop term (features), a per-mesh term
// (embedding and bias; both computed by k_conv34_pool<true>) and the yaw terms, so
// inference evaluates the first two once per crop and per mesh and only adds them
// per pair.
// Inference head per pair, one per thread (NaN for an out-of-range pair).  The
// yaw weights and the output weights go to LDS first; each pair's per-crop and
// per-mesh rows (64 floats each, 256-byte aligned) are read as float4.
constexpr int kHeadPairThreads = 256;
__global__ void __launch_bounds__(kHeadPairThreads)
    k_head_pairs(const float* hid, const Params P, const Pair* pairs, int n_pairs, int n_crops,
                 int n_mesh, float* pred) {
  __shared__ float sw[3][kHid];  // cos-yaw weight, sin-yaw weight, output weight
  for (int r = threadIdx.x; r < kHid; r += blockDim.x) {
    const float* w = P.hW1 + r * kIn + kFeat + kEmb;
    sw[0][r] = w[0];
    sw[1][r] = w[1];
    sw[2][r] = P.hw2[r];
  }
  __syncthreads();
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_pairs) return;
  const Pair pr = pairs[q];
  if (!pair_ok(pr, n_crops, n_mesh)) {
    pred[q] = __uint_as_float(0x7fc00000u);
    return;
  }
  const float4* a = reinterpret_cast<const float4*>(hid + (size_t)pr.crop * kHid);
  const float4* bm = reinterpret_cast<const float4*>(hid + (size_t)(n_crops + pr.mesh) * kHid);
  float y = P.hb2[0];
#pragma unroll
  for (int r4 = 0; r4 < kHid / 4; ++r4) {
    const float4 u = a[r4], v = bm[r4];
    const float s4[4] = {u.x + v.x, u.y + v.y, u.z + v.z, u.w + v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 4 * r4 + j;
      const float z = fmaf(sw[1][r], pr.sin_yaw, fmaf(sw[0][r], pr.cos_yaw, s4[j]));
      y = fmaf(sw[2][r], fmaxf(z, 0.0f), y);
    }
  }
  pred[q] = y;
}

// Loss and head gradients for 64 pairs per workgroup: per-pair h and dz1 go to
// LDS, the weight gradients are reduced over the workgroup's pairs and added once.
__global__ void __launch_bounds__(64)
    k_head_bwd(const float* feat, const Params P, const Pair* pairs, const float* target,
               int n_pairs, int n_crops, int n_mesh, Params G, float* dfeat, float* loss_sum) {
  __shared__ float sh[64][kIn];    // head input per pair
  __shared__ float sdz[64][kHid];  // d loss / d z1 per pair
  __shared__ float sr1[64][kHid];  // relu(z1) per pair
  __shared__ float sdy[64];        // d loss / d y per pair
  const int t = threadIdx.x;
  const int q = blockIdx.x * 64 + t;
  const Pair pr = q < n_pairs ? pairs[q] : Pair{0, 0, 0.0f, 0.0f};
  const bool live = q < n_pairs && pair_ok(pr, n_crops, n_mesh);  // bad pairs contribute nothing
  float dy = 0.0f;
  if (live) {
    head_input(feat, P.emb, pr, sh[t]);
    float y = P.hb2[0];
    for (int r = 0; r < kHid; ++r) {
      float z = P.hb1[r];
      for (int i = 0; i < kIn; ++i) z = fmaf(P.hW1[r * kIn + i], sh[t][i], z);
      sr1[t][r] = fmaxf(z, 0.0f);
      sdz[t][r] = z;  // pre-activation for now
      y = fmaf(P.hw2[r], fmaxf(z, 0.0f), y);
    }
    const float diff = y - target[q];
    atomicAdd(loss_sum, diff * diff);
    dy = 2.0f * diff / (float)n_pairs;
    for (int r = 0; r < kHid; ++r) sdz[t][r] = sdz[t][r] > 0.0f ? dy * P.hw2[r] : 0.0f;
  } else {
    for (int i = 0; i < kIn; ++i) sh[t][i] = 0.0f;
    for (int r = 0; r < kHid; ++r) {
      sr1[t][r] = 0.0f;
      sdz[t][r] = 0.0f;
    }
  }
  sdy[t] = dy;
  __syncthreads();
  // dh = W1^T dz1 -> dfeat (per crop) and the embedding gradient (per mesh)
  if (live) {
    for (int i = 0; i < kFeat + kEmb; ++i) {
      float s = 0.0f;
      for (int r = 0; r < kHid; ++r) s = fmaf(P.hW1[r * kIn + i], sdz[t][r], s);
      if (i < kFeat)
        atomicAdd(&dfeat[pr.crop * kFeat + i], s);
      else
        atomicAdd(&G.emb[pr.mesh * kEmb + (i - kFeat)], s);
    }
  }
  // weight gradients reduced over the workgroup's pairs
  for (int e = t; e < kHid * kIn; e += 64) {
    const int r = e / kIn, i = e % kIn;
    float s = 0.0f;
    for (int u = 0; u < 64; ++u) s = fmaf(sdz[u][r], sh[u][i], s);
    atomicAdd(&G.hW1[e], s);
  }
  {
    const int r = t;  // kHid == blockDim.x
    float sb = 0.0f, sw = 0.0f;
    for (int u = 0; u < 64; ++u) {
      sb += sdz[u][r];
      sw = fmaf(sdy[u], sr1[u][r], sw);
    }
    atomicAdd(&G.hb1[r], sb);
    atomicAdd(&G.hw2[r], sw);
  }
  if (t == 0) {
    float s = 0.0f;
    for (int u = 0; u < 64; ++u) s += sdy[u];
    atomicAdd(&G.hb2[0], s);
  }
}

// ---------------------------------------------------------------------------
// optimiser and weight packing
// ---------------------------------------------------------------------------

__global__ void k_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bfloat16 MFMA copies of the conv weights: Wb[co][k] (k padded to KP with 0)
__global__ void k_pack(const float* master, int K, int KP, bf16_t* Wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kC * KP) return;
  const int co = i / KP, k = i % KP;
  Wb[i] = k < K ? f2bf(master[co * K + k]) : (bf16_t)0;
}

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------

void launch_crops(const float* obs, const unsigned* pdepth, int W, int H, const CropDesc* desc,
                  int n, bf16_t* out, hipStream_t s) {
  // 1,024 threads per crop: a few samples each, so that even a small batch keeps
  // enough loads in flight
  if (n > 0) hipLaunchKernelGGL(k_crops, dim3(n), dim3(1024), 0, s, obs, pdepth, W, H, desc, n, out);
}

// Input-gradient grid: one workgroup per four 32-pixel tiles up to 2,048 workgroups,
// which then take several tiles each (each workgroup stages the weights once).
static int dgrad_blocks(int n_img, int npix) {
  return std::max(1, std::min(2048, (n_img * npix + 127) / 128));
}

// Forward grid: about eight 32-pixel tiles per wave (the weight fragments a wave
// loads are reused across them), at least 512 workgroups while there are tiles.
static int conv_fwd_blocks(int n_img, int npix) {
  const int tiles = (n_img * npix + 31) / 32;
  const int full = (tiles + 3) / 4;  // one tile per wave
  return std::max(1, std::min(full, std::max(512, (tiles + 31) / 32)));
}

void launch_forward(const Net& net, int n_crops, hipStream_t s) {
  hipLaunchKernelGGL((k_conv_fwd<2, 1, 64>), dim3(conv_fwd_blocks(n_crops, 64 * 64)), dim3(256), 0, s,
                     net.crops, net.Wb[0], net.P.cb[0], net.a[1], n_crops);
  hipLaunchKernelGGL((k_conv_fwd<32, 2, 64>), dim3(conv_fwd_blocks(n_crops, 32 * 32)), dim3(256), 0,
                     s, net.a[1], net.Wb[1], net.P.cb[1], net.a[2], n_crops);
  hipLaunchKernelGGL((k_conv_fwd<32, 2, 32>), dim3(conv_fwd_blocks(n_crops, 16 * 16)), dim3(256), 0,
                     s, net.a[2], net.Wb[2], net.P.cb[2], net.a[3], n_crops);
  hipLaunchKernelGGL((k_conv_fwd<32, 2, 16>), dim3(conv_fwd_blocks(n_crops, 8 * 8)), dim3(256), 0, s,
                     net.a[3], net.Wb[3], net.P.cb[3], net.a[4], n_crops);
  hipLaunchKernelGGL(k_pool_fwd, dim3(n_crops), dim3(kC), 0, s, net.a[4], n_crops, net.feat);
}

// Grid of the fused first two layers: one workgroup per work item when they are
// few, else as many as are resident at once (three per CU, bound by the 45 KB band,
// on 256 CUs), each taking its share of the items.
static int conv12_blocks(int n_crops) { return std::max(1, std::min(n_crops * kConv12Items, 768)); }

static CropSource tensor_source(const bf16_t* crops) {
  CropSource c{};
  c.crops = crops;
  return c;
}

void launch_infer(const Net& net, int n_crops, hipStream_t s) {
  hipLaunchKernelGGL(k_conv12_fwd<false>, dim3(conv12_blocks(n_crops)), dim3(256), 0, s,
                     tensor_source(net.crops), net.Wb[0], net.P.cb[0], net.Wb[1], net.P.cb[1],
                     net.a[2], n_crops);
  hipLaunchKernelGGL(k_conv34_pool<false>, dim3(std::max(1, std::min(n_crops, 512))),
                     dim3(kConv34Threads), 0, s, net.a[2], net.Wb[2], net.P.cb[2], net.Wb[3],
                     net.P.cb[3], net.feat, n_crops, net.P, 0, nullptr);
}

void launch_infer_predict(const Net& net, int n_crops, int n_mesh, const Pair* pairs,
                          int n_pairs, float* pred, hipStream_t s, const ImageCrops* img) {
  if (img) {
    CropSource c{};
    c.obs = img->obs;
    c.pdepth = img->pdepth;
    c.W = img->W;
    c.H = img->H;
    c.desc = img->desc;
    hipLaunchKernelGGL(k_conv12_fwd<true>, dim3(conv12_blocks(n_crops)), dim3(256), 0, s, c,
                       net.Wb[0], net.P.cb[0], net.Wb[1], net.P.cb[1], net.a[2], n_crops);
  } else {
    hipLaunchKernelGGL(k_conv12_fwd<false>, dim3(conv12_blocks(n_crops)), dim3(256), 0, s,
                       tensor_source(net.crops), net.Wb[0], net.P.cb[0], net.Wb[1], net.P.cb[1],
                       net.a[2], n_crops);
  }
  hipLaunchKernelGGL(k_conv34_pool<true>,
                     dim3(std::max(n_mesh, std::max(1, std::min(n_crops, 512)))),
                     dim3(kConv34Threads), 0, s, net.a[2], net.Wb[2], net.P.cb[2], net.Wb[3],
                     net.P.cb[3], net.feat, n_crops, net.P, n_mesh, net.hid);
  if (n_pairs > 0)
    hipLaunchKernelGGL(k_head_pairs, dim3((n_pairs + kHeadPairThreads - 1) / kHeadPairThreads),
                       dim3(kHeadPairThreads), 0, s, net.hid,
                       net.P, pairs, n_pairs, n_crops, n_mesh, pred);
}

template <int CIN, int S, int HIN>
static void wgrad(const bf16_t* dpre, const bf16_t* in, float* dW, float* db, int n_img,
                  hipStream_t s) {
  constexpr int HO = HIN / S, K = 9 * CIN, KT = (K + 31) / 32;
  const int total = n_img * HO * HO;
  // about 2,048 workgroups over the k columns, at least 8 pixel groups per wave
  const int gy = std::max(1, 2048 / KT);
  const int pw = std::max(8, (total + 64 * gy - 1) / (64 * gy));
  const dim3 grid(KT, (total + 64 * pw - 1) / (64 * pw));
  hipLaunchKernelGGL((k_conv_wgrad<CIN, S, HIN>), grid, dim3(256), 0, s, dpre, in, dW, db, n_img,
                     pw);
}

void launch_backward(const Net& net, int n_crops, int n_mesh, const Pair* pairs,
                     const float* target, int n_pairs, hipStream_t s) {
  hipLaunchKernelGGL(k_head_bwd, dim3((n_pairs + 63) / 64), dim3(64), 0, s, net.feat, net.P,
                     pairs, target, n_pairs, n_crops, n_mesh, net.G, net.dfeat, net.loss);
  launch_trunk_backward(net, n_crops, s);
}

void launch_trunk_backward(const Net& net, int n_crops, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_bwd, dim3(n_crops), dim3(256), 0, s, net.dfeat, net.a[4], n_crops,
                     net.d[4]);
  wgrad<32, 2, 16>(net.d[4], net.a[3], net.G.cW[3], net.G.cb[3], n_crops, s);
  hipLaunchKernelGGL((k_conv_dgrad<2, 16>), dim3(dgrad_blocks(n_crops, 16 * 16)), dim3(256), 0, s,
                     net.d[4], net.Wb[3], net.a[3], net.d[3], n_crops);
  wgrad<32, 2, 32>(net.d[3], net.a[2], net.G.cW[2], net.G.cb[2], n_crops, s);
  hipLaunchKernelGGL((k_conv_dgrad<2, 32>), dim3(dgrad_blocks(n_crops, 32 * 32)), dim3(256), 0, s,
                     net.d[3], net.Wb[2], net.a[2], net.d[2], n_crops);
  wgrad<32, 2, 64>(net.d[2], net.a[1], net.G.cW[1], net.G.cb[1], n_crops, s);
  hipLaunchKernelGGL((k_conv_dgrad<2, 64>), dim3(dgrad_blocks(n_crops, 64 * 64)), dim3(256), 0, s,
                     net.d[2], net.Wb[1], net.a[1], net.d[1], n_crops);
  wgrad<2, 1, 64>(net.d[1], net.crops, net.G.cW[0], net.G.cb[0], n_crops, s);
}

void launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, int step,
                 hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2,
                     1e-8f, c1, c2);
}

void launch_pack(const Net& net, hipStream_t s) {
  const int Ks[4] = {18, 288, 288, 288}, KPs[4] = {32, 288, 288, 288};
  for (int l = 0; l < 4; ++l)
    hipLaunchKernelGGL(k_pack, dim3((kC * KPs[l] + 255) / 256), dim3(256), 0, s, net.P.cW[l],
                       Ks[l], KPs[l], net.Wb[l]);
}

}  // namespace cnn
}  // namespace perch
