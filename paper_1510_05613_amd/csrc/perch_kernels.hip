// perch_kernels.hip -- gfx950 kernels of PERCH successor evaluation
// (Narayanan & Likhachev, arXiv:1510.05613).
//
// One workgroup evaluates one successor s' = s + (mesh, pose) of a materialised
// parent s (Sec. IV-A): it transforms the candidate's vertices into LDS, rasterises
// its front faces into an LDS z-tile over the footprint, composites against the
// parent depth (the non-occlusion test of Eq. 3 and the new points dR), counts
// dR points unexplained by the observed cloud (dJ_r) by an exact pixel-window scan
// of the observed depth image (or, in radius mode 1, a uniform voxel hash of the
// cloud), counts observed points inside the candidate's volume unexplained by dR
// through an exact pixel window over the LDS tile (dJ_o), and at the goal level
// updates the parent's residual set U (Eq. 2, residual(K)).  Counts are wave
// ballot/popcount reductions.  The distance tests of Eq. 1 and the volume test are
// taken in float32 where a derived rounding margin proves the sign and in FP64
// otherwise, so every decision is that of exact arithmetic on the same inputs.
//
// Built with -ffp-contract=off: the float32 vertex stage is part of the
// rasterisation rule and must not have products fused into adds.
#include <algorithm>
#include <climits>

#include "perch_internal.h"

namespace perch {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

constexpr int kLdsPlanes = 64;   // V(O) planes staged in LDS per successor (more: read from HBM)

__device__ __forceinline__ int floor256(int x) { return x >> 8; }

// Product of two ints through the full-rate 24-bit multiplier: exact when both
// factors lie within +-2^23 and the product within +-2^31.  Image-space products
// qualify (images are at most 16,384 pixels wide and high), and so do the
// rasteriser's small-triangle edge terms (differences below 2^15 in 1/256 pixel).
__device__ __forceinline__ int imul(int a, int b) { return __mul24(a, b); }
__device__ __forceinline__ int ceil256(int x) { return -((-x) >> 8); }

__device__ __forceinline__ int wave_sum(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int ballot_count(bool p) { return __popcll(__ballot(p)); }

// Number of set bits of m below this lane.
__device__ __forceinline__ unsigned lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Orders this wave's LDS accesses: writes before the call are visible to every lane
// of the wave after it (a wave issues LDS operations in order; this stops the
// compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// vertex stage (float32, fixed operation order)
// ---------------------------------------------------------------------------

// Places model point m by pose (x, y, cos, sin) and maps it to the camera frame:
// w = (c m_x - s m_y + x, s m_x + c m_y + y, m_z); cam_k = ((M_k0 w_x + M_k1 w_y)
// + M_k2 w_z) + M_k3.
__device__ __forceinline__ void vcam(const Cam& c, const float4 pz, const float4 m, float& X,
                                     float& Y, float& Z) {
  const float wx = (pz.z * m.x - pz.w * m.y) + pz.x;
  const float wy = (pz.w * m.x + pz.z * m.y) + pz.y;
  const float wz = m.z;
  X = ((c.M[0] * wx + c.M[1] * wy) + c.M[2] * wz) + c.M[3];
  Y = ((c.M[4] * wx + c.M[5] * wy) + c.M[6] * wz) + c.M[7];
  Z = ((c.M[8] * wx + c.M[9] * wy) + c.M[10] * wz) + c.M[11];
}

// Projection and snap to 1/256 pixel: inv = 1/Z (IEEE division), u = fx (X inv) + cx,
// U = rint(256 u) (ties to even).  False when the vertex is within 1 cm of the
// camera plane or the snapped value leaves +-2^24.
__device__ __forceinline__ bool vsnap(const Cam& c, float X, float Y, float Z, int& U, int& V) {
  const float inv = 1.0f / Z;
  const float u = c.fx * (X * inv) + c.cx;
  const float v = c.fy * (Y * inv) + c.cy;
  const float su = rintf(256.0f * u), sv = rintf(256.0f * v);
  const bool ok = (Z > 0.01f) && (fabsf(su) <= 16777216.0f) && (fabsf(sv) <= 16777216.0f);
  U = ok ? (int)su : 0;
  V = ok ? (int)sv : 0;
  return ok;
}

// The snapped vertex of vcam + vsnap, out of line: the persistent batch kernel
// calls it only for footprints too wide for its packed vertex cache (inlined
// there, the rare path costs registers the whole kernel pays for).
__device__ __noinline__ int2 snapped_vertex(const Cam& c, const float4 pz, const float4 m) {
  float X, Y, Z;
  vcam(c, pz, m, X, Y, Z);
  int U, V;
  vsnap(c, X, Y, Z, U, V);
  return make_int2(U, V);
}

// ---------------------------------------------------------------------------
// depth: FP64 plane of the triangle's float32 camera-space vertices
// ---------------------------------------------------------------------------

// Camera Z where the ray through pixel centre (i, j) meets the triangle's plane:
// with n = (b - a) x (c - a), z = (n.a) / (n.r), r = ((i - cx)/fx, (j - cy)/fy, 1),
// written as z = N / (A i + B j + C).
struct Plane64 {
  double A, B, C, N;
};

__device__ __forceinline__ Plane64 make_plane(const Cam& c, float ax, float ay, float az,
                                              float bx, float by, float bz, float cx_,
                                              float cy_, float cz) {
  const double e1x = (double)bx - ax, e1y = (double)by - ay, e1z = (double)bz - az;
  const double e2x = (double)cx_ - ax, e2y = (double)cy_ - ay, e2z = (double)cz - az;
  const double nx = e1y * e2z - e1z * e2y;
  const double ny = e1z * e2x - e1x * e2z;
  const double nz = e1x * e2y - e1y * e2x;
  Plane64 p;
  p.N = nx * ax + ny * ay + nz * az;
  p.A = nx * c.dinv_fx;
  p.B = ny * c.dinv_fy;
  p.C = nz - p.A * c.dcx - p.B * c.dcy;
  return p;
}

// FP64 reciprocal estimate refined by one Newton step: the step squares the
// estimate's relative error, leaving the quotient far more accurate than the
// final rounding to float32 needs (depth ties closer than 1e-6 m are flagged by
// the parity rule anyway).
__device__ __forceinline__ float plane_depth(const Plane64& p, int i, int j) {
  const double den = fma(p.A, (double)i, fma(p.B, (double)j, p.C));
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);
  return (float)(p.N * r);
}

// Camera-space vertex for the depth plane only: the placement and camera
// rotation folded into one 3x3 map plus offset (FMA).  Coverage never uses it;
// it differs from the snapped vertex stage by float rounding only.
struct PoseMap {
  float a[9], b[3];
};

__device__ __forceinline__ PoseMap make_pose_map(const Cam& c, const float4 pz) {
  PoseMap m;
  for (int r = 0; r < 3; ++r) {
    m.a[3 * r + 0] = fmaf(c.M[4 * r], pz.z, c.M[4 * r + 1] * pz.w);
    m.a[3 * r + 1] = fmaf(c.M[4 * r + 1], pz.z, -(c.M[4 * r] * pz.w));
    m.a[3 * r + 2] = c.M[4 * r + 2];
    m.b[r] = fmaf(c.M[4 * r], pz.x, fmaf(c.M[4 * r + 1], pz.y, c.M[4 * r + 3]));
  }
  return m;
}

__device__ __forceinline__ void map_vertex(const PoseMap& m, const float4 v, float& X, float& Y,
                                           float& Z) {
  X = fmaf(m.a[0], v.x, fmaf(m.a[1], v.y, fmaf(m.a[2], v.z, m.b[0])));
  Y = fmaf(m.a[3], v.x, fmaf(m.a[4], v.y, fmaf(m.a[5], v.z, m.b[1])));
  Z = fmaf(m.a[6], v.x, fmaf(m.a[7], v.y, fmaf(m.a[8], v.z, m.b[2])));
}

// ---------------------------------------------------------------------------
// triangle coverage: integer edge functions, top-left rule, front faces only
// ---------------------------------------------------------------------------

// floor(e / a) for |e| < 2^29 and 1 <= a < 2^22 with |e / a| < 2^23, given
// ra = rcp(a): the float estimate is off by at most one (|e| rounds by <= 16, the
// product by a few ulps of a quotient below 2^21), and the exact 24-bit products
// fix it.  Quotients outside that range come out wrong and must go unused.
__device__ __forceinline__ int floor_div(int e, int a, float ra) {
  int q = (int)floorf((float)e * ra);
  q += (__mul24(q + 1, a) <= e) ? 1 : 0;
  q -= (__mul24(q, a) > e) ? 1 : 0;
  return q;
}

// One edge of raster_tri's int32 path, as a bound on a row's covered columns.
// The edge value at column offset k of row j is e_j - s k with e_{j+1} = e_j + t
// (s = 256 dy, t = 256 dx).  For s != 0 it holds for k <= q (s > 0) or k >= -q
// (s < 0) with q = floor(e_j / |s|), kept with its remainder and stepped per row
// by floor(t / |s|) and a carry.  For s = 0 it holds on whole rows: those are
// clipped once (rows rlo..rhi) and the bound is neutral.
struct EdgeDDA {
  int q, rem, dq, dr, a;
  bool pos;
  __device__ __forceinline__ void bound(int& lo, int& hi) const {
    hi = pos ? min(hi, q) : hi;
    lo = pos ? lo : max(lo, -q);
  }
  __device__ __forceinline__ void step() {
    rem += dr;
    q += dq;
    const bool c = rem >= a;
    rem -= c ? a : 0;
    q += c ? 1 : 0;
  }
};

__device__ __forceinline__ void edge_dda(int e, int dy, int dx, int ja, int& rlo, int& rhi,
                                         EdgeDDA& g) {
  const int s = 256 * dy, t = 256 * dx;
  const int a = abs(s);
  const bool flat = a == 0;
  // one divisor per edge: |s| for a sloped edge, |t| for a horizontal one (t != 0
  // for an edge of non-zero length, and both are multiples of 256)
  const int d = max(1, flat ? abs(t) : a);
  const float rd = __builtin_amdgcn_rcpf((float)d);
  const int q = floor_div(e, d, rd), dq = floor_div(t, d, rd);
  g.q = flat ? (1 << 20) : q;
  g.rem = flat ? 0 : e - imul(q, d);
  g.dq = flat ? 0 : dq;
  g.dr = flat ? 0 : t - imul(dq, d);
  g.a = d;
  g.pos = flat || s > 0;
  // horizontal edge: e + (j - ja) t >= 0 on rows j >= ja - floor(e / t) (t > 0) or
  // j <= ja + floor(e / -t) (t < 0), with q = floor(e / |t|) here
  rlo = (flat && t > 0) ? max(rlo, ja - q) : rlo;
  rhi = (flat && t < 0) ? min(rhi, ja + q) : rhi;
}

// Calls emit(i, j) for every pixel centre (256 i, 256 j) covered by the triangle
// with snapped vertices (x_k, y_k), restricted to columns [c0, c1] and rows
// [r0, r1].  Outward-CCW faces seen from the front have negative signed area in
// these y-down coordinates; others (back faces, zero area) are skipped.  A centre
// on an edge is covered iff the edge is a top edge (horizontal, interior below) or
// a left edge (interior to its right) of the positively oriented triangle.
template <class Emit>
__device__ __forceinline__ void raster_tri(int x0, int y0, int x1, int y1, int x2, int y2,
                                           int c0, int c1, int r0, int r1, Emit&& emit) {
  const int xmin = min(x0, min(x1, x2)), xmax = max(x0, max(x1, x2));
  const int ymin = min(y0, min(y1, y2)), ymax = max(y0, max(y1, y2));
  const int ia = max(c0, ceil256(xmin)), ib = min(c1, floor256(xmax));
  const int ja = max(r0, ceil256(ymin)), jb = min(r1, floor256(ymax));
  if (ia > ib || ja > jb) return;
  if (xmax - xmin < 16384 && ymax - ymin < 16384) {
    // all products below 2^28: int32 is exact
    int bx = x1 - x0, by = y1 - y0, cx = x2 - x0, cy = y2 - y0;
    const int area = imul(bx, cy) - imul(by, cx);
    if (area >= 0) return;
    int t = bx; bx = cx; cx = t;
    t = by; by = cy; cy = t;
    // edges a->b, b->c, c->a (a at the origin)
    const int d0x = bx, d0y = by, d1x = cx - bx, d1y = cy - by, d2x = -cx, d2y = -cy;
    const int b0 = (d0y < 0 || (d0y == 0 && d0x > 0)) ? 0 : -1;
    const int b1 = (d1y < 0 || (d1y == 0 && d1x > 0)) ? 0 : -1;
    const int b2 = (d2y < 0 || (d2y == 0 && d2x > 0)) ? 0 : -1;
    // Per row the covered centres form one interval; each sloped edge bounds it
    // from one side at floor(e / |s|) pixels from the box start, a quotient that
    // is stepped from row to row by exact integer DDA (quotient and remainder), so
    // thin triangles, whose boxes are mostly empty, cost a few adds per row.  A
    // horizontal edge (at most one) instead limits the rows.
    const int py = 256 * ja - y0, px0 = 256 * ia - x0;
    const int w = ib - ia + 1;
    int rlo = ja, rhi = jb;
    EdgeDDA g0, g1, g2;
    edge_dda(imul(d0x, py) - imul(d0y, px0) + b0, d0y, d0x, ja, rlo, rhi, g0);
    edge_dda(imul(d1x, py - by) - imul(d1y, px0 - bx) + b1, d1y, d1x, ja, rlo, rhi, g1);
    edge_dda(imul(d2x, py - cy) - imul(d2y, px0 - cx) + b2, d2y, d2x, ja, rlo, rhi, g2);
    for (int j = ja; j <= jb; ++j) {
      int lo = 0, hi = (j >= rlo && j <= rhi) ? w - 1 : -1;
      g0.bound(lo, hi);
      g1.bound(lo, hi);
      g2.bound(lo, hi);
      for (int i = lo; i <= hi; ++i) emit(ia + i, j);
      g0.step();
      g1.step();
      g2.step();
    }
  } else {
    long long bx = (long long)x1 - x0, by = (long long)y1 - y0;
    long long cx = (long long)x2 - x0, cy = (long long)y2 - y0;
    const long long area = bx * cy - by * cx;
    if (area >= 0) return;
    long long t = bx; bx = cx; cx = t;
    t = by; by = cy; cy = t;
    const long long d0x = bx, d0y = by, d1x = cx - bx, d1y = cy - by, d2x = -cx, d2y = -cy;
    const long long b0 = (d0y < 0 || (d0y == 0 && d0x > 0)) ? 0 : -1;
    const long long b1 = (d1y < 0 || (d1y == 0 && d1x > 0)) ? 0 : -1;
    const long long b2 = (d2y < 0 || (d2y == 0 && d2x > 0)) ? 0 : -1;
    for (int j = ja; j <= jb; ++j) {
      const long long py = 256LL * j - y0;
      const long long px0 = 256LL * ia - x0;
      long long e0 = d0x * py - d0y * px0 + b0;
      long long e1 = d1x * (py - by) - d1y * (px0 - bx) + b1;
      long long e2 = d2x * (py - cy) - d2y * (px0 - cx) + b2;
      for (int i = ia; i <= ib; ++i) {
        if ((e0 | e1 | e2) >= 0) emit(i, j);
        e0 -= 256 * d0y;
        e1 -= 256 * d1y;
        e2 -= 256 * d2y;
      }
    }
  }
}

// raster_tri by rows: calls row(j, i0, i1) for each row j of the triangle with its
// covered columns i0..i1 (non-empty), restricted as raster_tri is.  Same coverage.
template <class Row>
__device__ __forceinline__ void raster_tri_rows(int x0, int y0, int x1, int y1, int x2, int y2,
                                                int c0, int c1, int r0, int r1, Row&& row) {
  const int xmin = min(x0, min(x1, x2)), xmax = max(x0, max(x1, x2));
  const int ymin = min(y0, min(y1, y2)), ymax = max(y0, max(y1, y2));
  const int ia = max(c0, ceil256(xmin)), ib = min(c1, floor256(xmax));
  const int ja = max(r0, ceil256(ymin)), jb = min(r1, floor256(ymax));
  if (ia > ib || ja > jb) return;
  if (xmax - xmin < 16384 && ymax - ymin < 16384) {
    int bx = x1 - x0, by = y1 - y0, cx = x2 - x0, cy = y2 - y0;
    const int area = imul(bx, cy) - imul(by, cx);
    if (area >= 0) return;
    int t = bx; bx = cx; cx = t;
    t = by; by = cy; cy = t;
    const int d0x = bx, d0y = by, d1x = cx - bx, d1y = cy - by, d2x = -cx, d2y = -cy;
    const int b0 = (d0y < 0 || (d0y == 0 && d0x > 0)) ? 0 : -1;
    const int b1 = (d1y < 0 || (d1y == 0 && d1x > 0)) ? 0 : -1;
    const int b2 = (d2y < 0 || (d2y == 0 && d2x > 0)) ? 0 : -1;
    const int py = 256 * ja - y0, px0 = 256 * ia - x0;
    const int w = ib - ia + 1;
    int rlo = ja, rhi = jb;
    EdgeDDA g0, g1, g2;
    edge_dda(imul(d0x, py) - imul(d0y, px0) + b0, d0y, d0x, ja, rlo, rhi, g0);
    edge_dda(imul(d1x, py - by) - imul(d1y, px0 - bx) + b1, d1y, d1x, ja, rlo, rhi, g1);
    edge_dda(imul(d2x, py - cy) - imul(d2y, px0 - cx) + b2, d2y, d2x, ja, rlo, rhi, g2);
    for (int j = ja; j <= jb; ++j) {
      int lo = 0, hi = (j >= rlo && j <= rhi) ? w - 1 : -1;
      g0.bound(lo, hi);
      g1.bound(lo, hi);
      g2.bound(lo, hi);
      if (lo <= hi) row(j, ia + lo, ia + hi);
      g0.step();
      g1.step();
      g2.step();
    }
  } else {
    // large boxes: per-pixel 64-bit edge functions, as raster_tri
    raster_tri(x0, y0, x1, y1, x2, y2, c0, c1, r0, r1, [&](int i, int j) { row(j, i, i); });
  }
}

// True when the triangle is front-facing (negative snapped area) and its box
// holds at least one pixel centre inside columns [c0, c1] and rows [r0, r1]: the
// triangles raster_tri can emit for.
__device__ __forceinline__ bool tri_candidate(int x0, int y0, int x1, int y1, int x2, int y2,
                                              int c0, int c1, int r0, int r1) {
  // evaluated without early exits: the scan runs it for every triangle
  const int xmin = min(x0, min(x1, x2)), xmax = max(x0, max(x1, x2));
  const int ymin = min(y0, min(y1, y2)), ymax = max(y0, max(y1, y2));
  const bool inb = (max(c0, ceil256(xmin)) <= min(c1, floor256(xmax))) &
                   (max(r0, ceil256(ymin)) <= min(r1, floor256(ymax)));
  const bool small = (xmax - xmin < 16384) & (ymax - ymin < 16384);
  // 24-bit products: exact when small (factors below 2^14, products below 2^28);
  // larger triangles are decided in 64 bits below
  const int a32 = imul(x1 - x0, y2 - y0) - imul(y1 - y0, x2 - x0);
  bool front = a32 < 0;
  if (!small) {
    const long long area = (long long)(x1 - x0) * (y2 - y0) - (long long)(y1 - y0) * (x2 - x0);
    front = area < 0;
  }
  return inb & front;
}

// ---------------------------------------------------------------------------
// observed cloud helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ float3 backproject(const Cam& c, int i, int j, float z) {
  return make_float3(((float)i - c.cx) * z * c.inv_fx, ((float)j - c.cy) * z * c.inv_fy, z);
}

// ---------------------------------------------------------------------------
// decisions at a threshold: float32 outside a proven error margin, FP64 inside it
// ---------------------------------------------------------------------------

// Margin of the float32 distance test for a point seen at depth z: when the float32
// |q - p|^2 - delta^2 exceeds it in magnitude, its sign is the sign of the exact
// value for the same pixels and float32 depths (derivation with the host's
// constants t_lin, t_0, t_a, t_s).
__device__ __forceinline__ float delta_margin(const Cam& c, float z) {
  const float a = fmaf(c.t_a, z, c.t_s);
  return fmaf(c.t_lin, z, c.t_0) + 4.0f * a * a;
}

// Eq. (1)'s test |q - p| <= delta for q = pixel (iq, jq) at depth zq and p = pixel
// (ip, jp) at depth zp, back-projected through the pixel centres in FP64.
__device__ __forceinline__ bool within_delta64(const Cam& c, int iq, int jq, float zq, int ip,
                                            int jp, float zp) {
  const double dq = zq, dp = zp;
  const double ex = (((double)iq - c.dcx) * dq - ((double)ip - c.dcx) * dp) * c.dinv_fx;
  const double ey = (((double)jq - c.dcy) * dq - ((double)jp - c.dcy) * dp) * c.dinv_fy;
  const double ez = dq - dp;
  return ex * ex + ey * ey + ez * ez <= c.ddelta2;
}

// The same test from the float32 squared distance d2 of the float32 back-projections
// and the margin tau of the point held fixed: decided by d2 outside the margin, in
// FP64 inside it.
__device__ __forceinline__ bool within_delta(const Cam& c, float d2, float tau, int iq, int jq,
                                             float zq, int ip, int jp, float zp) {
  const float t = d2 - c.delta2;
  if (__builtin_expect(fabsf(t) > tau, 1)) return t <= 0.0f;
  return within_delta64(c, iq, jq, zq, ip, jp, zp);
}

__device__ __forceinline__ unsigned long long cell_key(int x, int y, int z) {
  return (unsigned long long)((unsigned)(x + (1 << 20)) & 0x1FFFFFu) |
         ((unsigned long long)((unsigned)(y + (1 << 20)) & 0x1FFFFFu) << 21) |
         ((unsigned long long)((unsigned)(z + (1 << 20)) & 0x1FFFFFu) << 42);
}

__device__ __forceinline__ unsigned hash_key(unsigned long long k) {
  k ^= k >> 31;
  k *= 0x7fb5d329728ea185ull;
  k ^= k >> 27;
  k *= 0x81dadef4bc2dd44dull;
  k ^= k >> 33;
  return (unsigned)k;
}

// Eq. (1) against the whole observed cloud: true iff some observed point lies
// within delta of q (camera frame; pixel (iq, jq) at depth zq, distance margin tau).
// Scans every voxel cell overlapping the cube q +- qpad (qpad slightly above delta,
// so float rounding of the cell index cannot drop a neighbour) and stops at the
// first hit.  Each point carries its pixel index (as float bits in w) for the FP64
// decision near delta.
__device__ __forceinline__ bool explained_by_cloud(const Cam& cam, const Hash& hs, float qx,
                                                   float qy, float qz, int iq, int jq, float tau) {
  const int x0 = (int)floorf((qx - hs.qpad) * hs.inv_cell);
  const int x1 = (int)floorf((qx + hs.qpad) * hs.inv_cell);
  const int y0 = (int)floorf((qy - hs.qpad) * hs.inv_cell);
  const int y1 = (int)floorf((qy + hs.qpad) * hs.inv_cell);
  const int z0 = (int)floorf((qz - hs.qpad) * hs.inv_cell);
  const int z1 = (int)floorf((qz + hs.qpad) * hs.inv_cell);
  for (int cz = z0; cz <= z1; ++cz)
    for (int cy = y0; cy <= y1; ++cy)
      for (int cx = x0; cx <= x1; ++cx) {
        const unsigned long long key = cell_key(cx, cy, cz);
        unsigned slot = hash_key(key) & (unsigned)hs.mask;
        for (;;) {
          const unsigned long long k = hs.keys[slot];
          if (k == key) {
            const int2 se = hs.cells[slot];
            for (int t = se.x; t < se.x + se.y; ++t) {
              const float4 p = hs.pts[t];
              const float dx = p.x - qx, dy = p.y - qy, dz = p.z - qz;
              const float e = dx * dx + dy * dy + dz * dz - cam.delta2;
              if (__builtin_expect(fabsf(e) > tau, 1)) {
                if (e <= 0.0f) return true;
              } else {
                const int pix = __float_as_int(p.w);
                if (within_delta64(cam, iq, jq, qz, pix % cam.W, pix / cam.W, p.z)) return true;
              }
            }
            break;
          }
          if (k == kEmptyKey) break;
          slot = (slot + 1) & (unsigned)hs.mask;
        }
      }
  return false;
}

// Camera frame -> object frame of one pose, folded into a 3x4 map:
// o = Rz(theta)^-1 (Winv p - (x, y, 0)) with the exact inverse of the placement.
struct ObjMap {
  float a[9], b[3];
};

__device__ __forceinline__ ObjMap make_obj_map(const Cam& c, const float4 pz) {
  const float inv_n2 = 1.0f / (pz.z * pz.z + pz.w * pz.w);
  const float cs = pz.z * inv_n2, sn = pz.w * inv_n2;
  ObjMap m;
  for (int k = 0; k < 3; ++k) {
    m.a[k] = fmaf(cs, c.Winv[k], sn * c.Winv[4 + k]);
    m.a[3 + k] = fmaf(cs, c.Winv[4 + k], -(sn * c.Winv[k]));
    m.a[6 + k] = c.Winv[8 + k];
  }
  const float tx = c.Winv[3] - pz.x, ty = c.Winv[7] - pz.y;
  m.b[0] = fmaf(cs, tx, sn * ty);
  m.b[1] = fmaf(cs, ty, -(sn * tx));
  m.b[2] = c.Winv[11];
  return m;
}

__device__ __forceinline__ float3 apply_obj_map(const ObjMap& m, float3 p) {
  return make_float3(fmaf(m.a[0], p.x, fmaf(m.a[1], p.y, fmaf(m.a[2], p.z, m.b[0]))),
                     fmaf(m.a[3], p.x, fmaf(m.a[4], p.y, fmaf(m.a[5], p.z, m.b[1]))),
                     fmaf(m.a[6], p.x, fmaf(m.a[7], p.y, fmaf(m.a[8], p.z, m.b[2]))));
}

// The same map in FP64 from the FP64 world_from_cam and the pose's float32 values:
// o = (c dx + s dy, -s dx + c dy) / (c^2 + s^2), o_z = w_z, with (dx, dy) = w - (x, y)
// and w = Winv p.
struct ObjMap64 {
  double a[9], b[3];
};

__device__ __forceinline__ ObjMap64 make_obj_map64(const Cam& c, const float4 pz) {
  const double cs = pz.z, sn = pz.w;
  const double n2 = cs * cs + sn * sn;
  const double ca = cs / n2, sa = sn / n2;
  const double* W = c.dWinv;
  ObjMap64 m;
  for (int k = 0; k < 3; ++k) {
    m.a[k] = ca * W[k] + sa * W[4 + k];
    m.a[3 + k] = ca * W[4 + k] - sa * W[k];
    m.a[6 + k] = W[8 + k];
  }
  const double tx = W[3] - (double)pz.x, ty = W[7] - (double)pz.y;
  m.b[0] = ca * tx + sa * ty;
  m.b[1] = ca * ty - sa * tx;
  m.b[2] = W[11];
  return m;
}

// Face-plane value n.o - w of a float32 object-frame point, in fused products.
__device__ __forceinline__ float plane_val(const float4 pl, float3 o) {
  return fmaf(pl.x, o.x, fmaf(pl.y, o.y, fmaf(pl.z, o.z, -pl.w)));
}

__device__ __forceinline__ float max8(float a, float b, float c, float d, float e, float f,
                                      float g, float h) {
  return fmaxf(fmaxf(fmaxf(a, b), fmaxf(c, d)), fmaxf(fmaxf(e, f), fmaxf(g, h)));
}

// max_f (n_f . o - w_f) <= 0 in FP64.
__device__ __forceinline__ bool inside_planes64(const float4* planes, int n_planes, double ox,
                                             double oy, double oz) {
  double m = -INFINITY;
  for (int f = 0; f < n_planes; ++f) {
    const float4 pl = planes[f];
    m = fmax(m, (double)pl.x * ox + (double)pl.y * oy + (double)pl.z * oz - (double)pl.w);
  }
  return m <= 0.0;
}

// The mesh's boxes about its vertex-box centre ctr for the volume test, widened
// (outer) and narrowed (inner) by the float32 object point's error bound vbox.
struct VolBoxes {
  float3 outer;  // vertex-box half-extents + vbox
  float3 inner;  // inner-box half-extents - vbox (negative: no inner box)
};

__device__ __forceinline__ VolBoxes vol_boxes(const EvalParams& ep, const float4 hout,
                                              const float4 hin) {
  const float mb = ep.vbox;
  VolBoxes b;
  b.outer = make_float3(hout.x + mb, hout.y + mb, hout.z + mb);
  b.inner = make_float3(hin.x - mb, hin.y - mb, hin.z - mb);
  return b;
}

// Sign of max_f (n_f . o - w_f) for a float32 point whose plane values are within
// tau of the exact ones: -1 all below -tau (inside), +1 one above +tau (outside), 0
// undecided.
__device__ __forceinline__ int plane_side(const float4* planes, int n_planes, float3 o,
                                          float tau) {
  float mx = -INFINITY;
  int f = 0;
  for (; f + 8 <= n_planes; f += 8) {  // eight planes per branch
    mx = fmaxf(mx, max8(plane_val(planes[f], o), plane_val(planes[f + 1], o),
                        plane_val(planes[f + 2], o), plane_val(planes[f + 3], o),
                        plane_val(planes[f + 4], o), plane_val(planes[f + 5], o),
                        plane_val(planes[f + 6], o), plane_val(planes[f + 7], o)));
    if (mx > tau) return 1;
  }
  for (; f + 4 <= n_planes; f += 4) {
    mx = fmaxf(mx, fmaxf(fmaxf(plane_val(planes[f], o), plane_val(planes[f + 1], o)),
                         fmaxf(plane_val(planes[f + 2], o), plane_val(planes[f + 3], o))));
    if (mx > tau) return 1;
  }
  for (; f < n_planes; ++f) mx = fmaxf(mx, plane_val(planes[f], o));
  if (mx > tau) return 1;
  return __builtin_expect(mx < -tau, 1) ? -1 : 0;
}

// Observed point p in V(O) = {o : n_f . o <= w_f for every face plane}, the decision
// of exact arithmetic on the same inputs (pixel (i, j), float32 depth z) outside an
// FP64 rounding band.  o32 (the float32 map of the float32 back-projection, within
// vbox of the exact object-frame point in every coordinate, the 1e-6 m slack in vbox
// covering the rounding of o32 - ctr) rules out points more than vbox outside the
// mesh's vertex box and rules in points more than vbox inside its inner box
// (strictly inside every face plane).  The rest take the face-plane values of o32:
// all below -vtau32 is inside, one above +vtau32 is outside; what stays undecided
// takes the FP64 object-frame point rounded to float32 with the tighter vtau, and
// anything still undecided is decided in FP64.
__device__ __forceinline__ bool in_volume_at(const Cam& c, const EvalParams& ep,
                                             const ObjMap64& dm, const float4 ctr,
                                             const VolBoxes& bx, const float4* planes,
                                             int n_planes, float3 o32, int i, int j, float z) {
  const float ax = fabsf(o32.x - ctr.x), ay = fabsf(o32.y - ctr.y), az = fabsf(o32.z - ctr.z);
  if (ax > bx.outer.x || ay > bx.outer.y || az > bx.outer.z) return false;
  if (ax <= bx.inner.x && ay <= bx.inner.y && az <= bx.inner.z) return true;
  const int s32 = plane_side(planes, n_planes, o32, ep.vtau32);
  if (__builtin_expect(s32 != 0, 1)) return s32 < 0;
  const double dz = z;
  const double px = ((double)i - c.dcx) * dz * c.dinv_fx;
  const double py = ((double)j - c.dcy) * dz * c.dinv_fy;
  const double ox = fma(dm.a[0], px, fma(dm.a[1], py, fma(dm.a[2], dz, dm.b[0])));
  const double oy = fma(dm.a[3], px, fma(dm.a[4], py, fma(dm.a[5], dz, dm.b[1])));
  const double oz = fma(dm.a[6], px, fma(dm.a[7], py, fma(dm.a[8], dz, dm.b[2])));
  const int s = plane_side(planes, n_planes, make_float3((float)ox, (float)oy, (float)oz), ep.vtau);
  if (s != 0) return s < 0;
  return inside_planes64(planes, n_planes, ox, oy, oz);
}

// p in V(O) of mesh `mesh` at the pose of maps om / dm.
__device__ __forceinline__ bool in_volume(const Cam& c, const EvalParams& ep, const Meshes& M,
                                          int mesh, const ObjMap& om, const ObjMap64& dm,
                                          float3 p, int i, int j, float z) {
  const VolBoxes bx = vol_boxes(ep, M.aabb[4 * mesh + 1], M.aabb[4 * mesh + 2]);
  const int2 fr = M.frange[mesh];
  return in_volume_at(c, ep, dm, M.aabb[4 * mesh], bx, M.planes + fr.x, fr.y,
                      apply_obj_map(om, p), i, j, z);
}

// Pixel window radii (columns, rows) that hold every point within dwin of the
// point p seen at depth p.z: |du| <= fx dwin sqrt(1 + (X/Z)^2) / (Z - dwin), +1 for
// rounding, capped by the scene-wide halo.
__device__ __forceinline__ void window_radius(const Cam& c, const EvalParams& ep, float3 p,
                                              int& ru, int& rv) {
  const float den = p.z - ep.dwin;
  if (!(den > 0.0f)) {
    ru = rv = ep.halo;
    return;
  }
  // hardware reciprocal and square root: the largest integer offset needed is
  // floor(x) for the exact bound x, and floor(x~) + 1 >= floor(x) whenever the
  // estimate x~ > x - 1, which a relative error of a few ulps guarantees
  const float iz = __builtin_amdgcn_rcpf(p.z), iden = __builtin_amdgcn_rcpf(den);
  const float a = p.x * iz, b = p.y * iz;
  ru = min(ep.halo, (int)(c.fx * ep.dwin * __builtin_amdgcn_sqrtf(1.0f + a * a) * iden) + 1);
  rv = min(ep.halo, (int)(c.fy * ep.dwin * __builtin_amdgcn_sqrtf(1.0f + b * b) * iden) + 1);
}

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------

__global__ void k_fill_u32(unsigned* p, unsigned v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_i32(int* p, int v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Per pixel: the least and greatest observed depth within the (2R+1)^2 window
// around it ((+inf, -inf) when the window holds no return).  Every observed point
// within delta of a point q seen at that pixel lies in its pixel window (radius
// <= R), so |z_p - z_q| <= delta fails for all of them when z_q is outside
// [min - delta, max + delta].
__global__ void k_obs_range(Cam cam, const float* obs, float2* out, int R) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cam.W * cam.H) return;
  const int i = k % cam.W, j = k / cam.W;
  float lo = INFINITY, hi = -INFINITY;
  for (int jj = max(0, j - R); jj <= min(cam.H - 1, j + R); ++jj)
    for (int ii = max(0, i - R); ii <= min(cam.W - 1, i + R); ++ii) {
      const float z = obs[jj * cam.W + ii];
      if (z > 0.0f) {
        lo = fminf(lo, z);
        hi = fmaxf(hi, z);
      }
    }
  out[k] = make_float2(lo, hi);
}

// ---------------------------------------------------------------------------
// voxel hash of the observed cloud
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long point_cell(float3 p, float inv_cell) {
  return cell_key((int)floorf(p.x * inv_cell), (int)floorf(p.y * inv_cell),
                  (int)floorf(p.z * inv_cell));
}

__device__ __forceinline__ unsigned find_slot(const unsigned long long* keys, int mask,
                                              unsigned long long key) {
  unsigned slot = hash_key(key) & (unsigned)mask;
  while (keys[slot] != key) slot = (slot + 1) & (unsigned)mask;
  return slot;
}

__global__ void k_hash_insert(Cam cam, const float* depth, unsigned long long* keys, int* counts,
                              int mask, float inv_cell, int* n_points) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cam.W * cam.H) return;
  const float z = depth[k];
  if (!(z > 0.0f)) return;
  const float3 p = backproject(cam, k % cam.W, k / cam.W, z);
  const unsigned long long key = point_cell(p, inv_cell);
  unsigned slot = hash_key(key) & (unsigned)mask;
  for (;;) {
    const unsigned long long prev = atomicCAS(&keys[slot], kEmptyKey, key);
    if (prev == kEmptyKey || prev == key) break;
    slot = (slot + 1) & (unsigned)mask;
  }
  atomicAdd(&counts[slot], 1);
  atomicAdd(n_points, 1);
}

// exclusive scan of the per-slot counts (one workgroup of 1024 threads)
__global__ void __launch_bounds__(1024) k_scan_cells(const int* counts, int2* cells, int n) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int a = min(n, t * chunk), b = min(n, a + chunk);
  int s = 0;
  for (int i = a; i < b; ++i) s += counts[i];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int i = a; i < b; ++i) {
    cells[i] = make_int2(run, counts[i]);
    run += counts[i];
  }
}

__global__ void k_hash_scatter(Cam cam, const float* depth, const unsigned long long* keys,
                               const int2* cells, int* fill, float4* pts, int mask,
                               float inv_cell) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cam.W * cam.H) return;
  const float z = depth[k];
  if (!(z > 0.0f)) return;
  const float3 p = backproject(cam, k % cam.W, k / cam.W, z);
  const unsigned slot = find_slot(keys, mask, point_cell(p, inv_cell));
  const int pos = cells[slot].x + atomicAdd(&fill[slot], 1);
  pts[pos] = make_float4(p.x, p.y, p.z, __int_as_float(k));  // w: the pixel index
}

// ---------------------------------------------------------------------------
// full-frame render of one object (parent composites, perch_render)
// ---------------------------------------------------------------------------

struct ParentObjs {
  int2 o[kMaxObjects];
};

// One triangle of one object per thread, into a full-frame depth image.
__device__ __forceinline__ void render_triangle(const Cam& cam, const Meshes& M,
                                                const float4* poses, int mesh, int pose, int t,
                                                unsigned* depth) {
  const int4 rg = M.range[mesh];
  if (t >= rg.w) return;
  const float4 pz = poses[pose];
  const int4 tr = M.tris[rg.z + t];
  float X[3], Y[3], Z[3];
  int U[3], V[3];
  const int idx[3] = {tr.x, tr.y, tr.z};
  bool ok = true;
  for (int k = 0; k < 3; ++k) {
    vcam(cam, pz, M.verts[rg.x + idx[k]], X[k], Y[k], Z[k]);
    ok &= vsnap(cam, X[k], Y[k], Z[k], U[k], V[k]);
  }
  if (!ok) return;
  const Plane64 pl = make_plane(cam, X[0], Y[0], Z[0], X[1], Y[1], Z[1], X[2], Y[2], Z[2]);
  const int W = cam.W;
  raster_tri(U[0], V[0], U[1], V[1], U[2], V[2], 0, cam.W - 1, 0, cam.H - 1,
             [&](int i, int j) {
               const float z = plane_depth(pl, i, j);
               atomicMin(&depth[j * W + i], __float_as_uint(z));
             });
}

__global__ void k_render_object(Cam cam, Meshes M, const float4* poses, int mesh, int pose,
                                unsigned* depth) {
  render_triangle(cam, M, poses, mesh, pose, blockIdx.x * blockDim.x + threadIdx.x, depth);
}

// All j objects of a parent in one launch (blockIdx.y = object): the composite is
// the same minimum as j single-object launches, without their launch latency.
__global__ void k_render_objects(Cam cam, Meshes M, const float4* poses, ParentObjs po, int j,
                                 unsigned* depth) {
  const int k = blockIdx.y;
  if (k >= j) return;
  render_triangle(cam, M, poses, po.o[k].x, po.o[k].y, blockIdx.x * blockDim.x + threadIdx.x,
                  depth);
}

// ---------------------------------------------------------------------------
// goal-level parent set U: observed points outside every parent volume and
// unexplained by the parent composite R_{K-1}
// ---------------------------------------------------------------------------



__global__ void k_parent_u(Cam cam, Meshes M, const float4* poses, const float* obs,
                           ParentObjs po, int j, const unsigned* pdepth, unsigned* ubits,
                           int* ucount, EvalParams ep) {
  // the parent objects' camera-to-object maps, once per workgroup (j <= 16 threads)
  __shared__ ObjMap s_om[kMaxObjects];
  __shared__ ObjMap64 s_dm[kMaxObjects];
  if ((int)threadIdx.x < j) {
    const float4 pz = poses[po.o[threadIdx.x].y];
    s_om[threadIdx.x] = make_obj_map(cam, pz);
    s_dm[threadIdx.x] = make_obj_map64(cam, pz);
  }
  __syncthreads();
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int W = cam.W, H = cam.H;
  bool inU = false;
  if (k < W * H) {
    const float z = obs[k];
    if (z > 0.0f) {
      const int i = k % W, jj = k / W;
      const float3 p = backproject(cam, i, jj, z);
      bool inV = false;
      for (int a = 0; a < j && !inV; ++a)
        inV = in_volume(cam, ep, M, po.o[a].x, s_om[a], s_dm[a], p, i, jj, z);
      if (!inV) {
        int ru, rv;
        window_radius(cam, ep, p, ru, rv);
        const float tau = delta_margin(cam, z);
        bool expl = false;
        for (int jq = max(0, jj - rv); jq <= min(H - 1, jj + rv) && !expl; ++jq)
          for (int iq = max(0, i - ru); iq <= min(W - 1, i + ru); ++iq) {
            const unsigned kq = pdepth[jq * W + iq];
            if (kq == kInfBits) continue;
            const float zq = __uint_as_float(kq);
            const float3 q = backproject(cam, iq, jq, zq);
            const float dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
            if (within_delta(cam, dx * dx + dy * dy + dz * dz, tau, iq, jq, zq, i, jj, z)) {
              expl = true;
              break;
            }
          }
        inU = !expl;
      }
    }
  }
  const unsigned long long b = __ballot(inU);
  if (inU) atomicOr(&ubits[k >> 5], 1u << (k & 31));
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(ucount, __popcll(b));
}

// ---------------------------------------------------------------------------
// overlap heuristic: observed pixels inside the union V_j of the parent volumes
// ---------------------------------------------------------------------------

__global__ void k_parent_v(Cam cam, Meshes M, const float4* poses, const float* obs,
                           ParentObjs po, int j, unsigned* vbits, EvalParams ep) {
  __shared__ ObjMap s_om[kMaxObjects];  // as in k_parent_u
  __shared__ ObjMap64 s_dm[kMaxObjects];
  if ((int)threadIdx.x < j) {
    const float4 pz = poses[po.o[threadIdx.x].y];
    s_om[threadIdx.x] = make_obj_map(cam, pz);
    s_dm[threadIdx.x] = make_obj_map64(cam, pz);
  }
  __syncthreads();
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int W = cam.W;
  bool inV = false;
  if (k < W * cam.H) {
    const float z = obs[k];
    if (z > 0.0f) {
      const int i = k % W, jj = k / W;
      const float3 p = backproject(cam, i, jj, z);
      for (int a = 0; a < j && !inV; ++a)
        inV = in_volume(cam, ep, M, po.o[a].x, s_om[a], s_dm[a], p, i, jj, z);
    }
  }
  if (inV) atomicOr(&vbits[k >> 5], 1u << (k & 31));
}

// ---------------------------------------------------------------------------
// successor evaluation: one workgroup per successor
// ---------------------------------------------------------------------------

// Evaluates successor s' = parent + (cd.x = mesh, cd.y = pose) of scene S and
// writes output slot s.  Every thread of the workgroup calls it with the same
// arguments; it synchronises the workgroup internally.
// GAIN: also write the overlap gain (points of V(O) outside the parent's V_j) to
// out_gain, which must then be non-null.
// HQ: the scene may answer dJ_r by the voxel hash (radius mode 1).  G: the parent
// may be at the goal level (the set U and the residual).  P: there may be a parent
// (below the root); without one dR is the silhouette, so the composite pass is
// skipped and the dJ pass counts the covered pixels.  Instantiations without the
// hash, the goal-level or the parent code measurably shorten the kernel's critical
// loops; G false requires a parent below the goal level, P false the root.
template <int NT, bool OUTLINE, bool VP, bool GAIN, bool HQ, bool G, bool P>
__device__ __forceinline__ void eval_successor(const SceneDev& S, const Parent& par, const int2 cd,
                                               const int s, int* __restrict__ out_cost,
                                               int* __restrict__ out_status,
                                               int* __restrict__ out_comps,
                                               int* __restrict__ out_gain, unsigned char* smem,
                                               int* s_bb, int* s_acc, float4* s_pl,
                                               ObjMap64* s_dm) {
  const Cam& cam = S.cam;
  const Meshes& M = S.M;
  const float4* __restrict__ poses = S.poses;
  const float* __restrict__ obs = S.obs;
  const float2* __restrict__ obs_range = S.obs_range;
  const Hash& hs = S.hs;
  const EvalParams& ep = S.ep;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int W = cam.W, H = cam.H;
  if (cd.x < 0 || cd.x >= ep.n_mesh || cd.y < 0 || cd.y >= ep.n_poses) {
    if (tid == 0) {
      out_status[s] = -4;
      out_cost[s] = -1;
      if (GAIN) out_gain[s] = -1;
      if (out_comps)
        for (int c = 0; c < 5; ++c) out_comps[5 * s + c] = -1;
    }
    return;
  }
  const int mesh = cd.x;
  const float4 pz = poses[cd.y];
  const ObjMap om = make_obj_map(cam, pz);
  // the FP64 map waits in LDS: only points inside the vertex box read it
  if (tid == 0) *s_dm = make_obj_map64(cam, pz);
  const ObjMap64& dm = *s_dm;
  const int4 rg = M.range[mesh];
  // snapped vertices: int2 (ep.vpack = 0) or relative to the footprint's corner in
  // 16 + 16 bits (ep.vpack = 1, meshes too large for int2)
  constexpr bool vpack = VP;  // the host picks the instantiation from ep.vpack
  int2* suv2 = reinterpret_cast<int2*>(smem);
  unsigned* suv = reinterpret_cast<unsigned*>(smem);
  unsigned* tile = reinterpret_cast<unsigned*>(
      smem + (size_t)ep.max_nv * (vpack ? sizeof(unsigned) : sizeof(int2)));
  unsigned* ring = tile + ep.tile_px + (tid >> 6) * 128;  // this wave's triangle queue
  if (tid < 4) s_bb[tid] = tid < 2 ? INT_MAX : INT_MIN;
  if (tid < 8) s_acc[tid] = 0;
  // V(O): box corners in registers, planes in LDS when they fit
  const int2 fr = M.frange[mesh];
  const float4 vctr = M.aabb[4 * mesh];
  const VolBoxes vbx = vol_boxes(ep, M.aabb[4 * mesh + 1], M.aabb[4 * mesh + 2]);
  const bool pl_lds = fr.y <= kLdsPlanes;
  if (pl_lds)
    for (int f = tid; f < fr.y; f += NT) s_pl[f] = M.planes[fr.x + f];
  __syncthreads();

  // ---- vertex stage: footprint bounding box, then the vertex cache ----
  // int2 cache: written directly.  Packed cache: the snapped vertices wait in the
  // z-tile's LDS (free until the first band) when they fit there, so packing them
  // needs no second vertex stage.
  int2* stage = vpack ? reinterpret_cast<int2*>(tile) : suv2;
  const bool staged =
      !vpack || (size_t)rg.y * sizeof(int2) <= (size_t)ep.tile_px * sizeof(unsigned);
  {
    int xmn = INT_MAX, ymn = INT_MAX, xmx = INT_MIN, ymx = INT_MIN;
    bool bad = false;
    for (int v = tid; v < rg.y; v += NT) {
      float X, Y, Z;
      vcam(cam, pz, M.verts[rg.x + v], X, Y, Z);
      int U, V;
      bad |= !vsnap(cam, X, Y, Z, U, V);
      if (staged) stage[v] = make_int2(U, V);
      xmn = min(xmn, U);
      ymn = min(ymn, V);
      xmx = max(xmx, U);
      ymx = max(ymx, V);
    }
    xmn = wave_min(xmn);
    ymn = wave_min(ymn);
    xmx = wave_max(xmx);
    ymx = wave_max(ymx);
    const bool any_bad = __ballot(bad) != 0;
    if (lane == 0) {
      atomicMin(&s_bb[0], xmn);
      atomicMin(&s_bb[1], ymn);
      atomicMax(&s_bb[2], xmx);
      atomicMax(&s_bb[3], ymx);
      if (any_bad) s_acc[6] = 1;
    }
  }
  __syncthreads();
  if (s_acc[6]) {
    if (tid == 0) {
      out_status[s] = -2;
      out_cost[s] = -1;
      if (GAIN) out_gain[s] = -1;
      if (out_comps)
        for (int c = 0; c < 5; ++c) out_comps[5 * s + c] = -1;
    }
    return;
  }
  // Packed cache: a footprint under 256 x 256 pixels packs its snapped vertices
  // into 32 bits each (from the staged copy, or from the same vertex stage again,
  // so the values are identical); a larger one is rasterised from vertices
  // recomputed where they are needed.
  // the footprint box is workgroup-uniform: scalar registers
  const int bb0 = __builtin_amdgcn_readfirstlane(s_bb[0]);
  const int bb1 = __builtin_amdgcn_readfirstlane(s_bb[1]);
  const int bb2 = __builtin_amdgcn_readfirstlane(s_bb[2]);
  const int bb3 = __builtin_amdgcn_readfirstlane(s_bb[3]);
  const int ox = bb0, oy = bb1;
  const bool packed = vpack && bb2 - ox < 65536 && bb3 - oy < 65536;
  if (packed) {
    for (int v = tid; v < rg.y; v += NT) {
      int2 uv;
      if (staged) {
        uv = stage[v];
      } else {
        float X, Y, Z;
        vcam(cam, pz, M.verts[rg.x + v], X, Y, Z);
        vsnap(cam, X, Y, Z, uv.x, uv.y);
      }
      suv[v] = (unsigned)(uv.x - ox) | ((unsigned)(uv.y - oy) << 16);
    }
    __syncthreads();  // the staged copy is read before the first band clears the tile
  }
  auto vert_uv = [&](int idx) -> int2 {
    if (!vpack) return suv2[idx];
    if (packed) {
      const unsigned w = suv[idx];
      return make_int2(ox + (int)(w & 0xFFFFu), oy + (int)(w >> 16));
    }
    if (OUTLINE) return snapped_vertex(cam, pz, M.verts[rg.x + idx]);
    float X, Y, Z;
    vcam(cam, pz, M.verts[rg.x + idx], X, Y, Z);
    int U, V;
    vsnap(cam, X, Y, Z, U, V);
    return make_int2(U, V);
  };

  // observed region: the vertex box (+1 px: every point of V(O) projects inside it),
  // grown by the window halo at the goal level (points of U explained by dR)
  const bool goal = G && par.goal;
  const int ext = goal ? max(1, ep.halo) : 1;
  const int ca = max(0, floor256(bb0) - ext), cb = min(W - 1, ceil256(bb2) + ext);
  const int ra = max(0, floor256(bb1) - ext), rb = min(H - 1, ceil256(bb3) + ext);
  const int tw = cb - ca + 1;
  const int nrows = rb - ra + 1;
  int core = nrows;
  if (tw > 0 && nrows > 0 && tw * nrows > ep.tile_px) core = ep.tile_px / tw - 2 * ep.halo;
  if (tw > 0 && nrows > 0 && core < 1) {
    if (tid == 0) {
      out_status[s] = -3;
      out_cost[s] = -1;
      if (GAIN) out_gain[s] = -1;
      if (out_comps)
        for (int c = 0; c < 5; ++c) out_comps[5 * s + c] = -1;
    }
    return;
  }
  int n_dJr = 0, n_dJo = 0, n_rem = 0, n_gain = 0;  // wave-uniform ballot counts
  int n_cov = 0;  // covered core pixels (the silhouette), counted in the dJ pass when !P

  for (int b0 = ra; b0 <= rb && tw > 0; b0 += core) {
    const int b1 = min(rb, b0 + core - 1);
    const int t0 = max(ra, b0 - ep.halo), t1 = min(rb, b1 + ep.halo);
    const int tn = (t1 - t0 + 1) * tw;
    for (int k = tid; k < tn; k += NT) tile[k] = kInfBits;
    __syncthreads();

    // ---- rasterise the candidate into the z-tile (rows t0..t1) ----
    // Each wave scans 64 triangles at a time, queues the front-facing ones whose
    // box holds a pixel centre of the tile (ballot compaction into an LDS ring),
    // and rasterises 64 queued triangles at once, so lanes stay busy although most
    // triangles are back-facing or fall between pixel centres.
    {
      auto raster_one = [&](unsigned t) {
        // queued triangles are front-facing with a pixel centre in their box, so
        // the depth plane is set up for every lane at once, outside the pixel walk;
        // its vertices are the vertex stage's float32 camera-space vertices
        const int4 tr = M.tris[rg.z + t];
        const float4 v0 = M.verts[rg.x + tr.x], v1 = M.verts[rg.x + tr.y];
        const float4 v2 = M.verts[rg.x + tr.z];
        const int2 a = vert_uv(tr.x), b = vert_uv(tr.y), c = vert_uv(tr.z);
        float X0, Y0, Z0, X1, Y1, Z1, X2, Y2, Z2;
        vcam(cam, pz, v0, X0, Y0, Z0);
        vcam(cam, pz, v1, X1, Y1, Z1);
        vcam(cam, pz, v2, X2, Y2, Z2);
        const Plane64 pl = make_plane(cam, X0, Y0, Z0, X1, Y1, Z1, X2, Y2, Z2);
        // the plane's denominator A i + B j + C steps by A along a row (FP64: the
        // accumulated rounding stays near 1e-14 of it, far below float32's)
        raster_tri_rows(a.x, a.y, b.x, b.y, c.x, c.y, ca, cb, t0, t1, [&](int j, int i0, int i1) {
          double den = fma(pl.A, (double)i0, fma(pl.B, (double)j, pl.C));
          unsigned* t = tile + imul(j - t0, tw) + (i0 - ca);
          for (int i = i0; i <= i1; ++i, ++t, den += pl.A) {
            double r = __builtin_amdgcn_rcp(den);
            r = fma(r, fma(-den, r, 1.0), r);
            atomicMin(t, __float_as_uint((float)(pl.N * r)));
          }
        });
      };
      unsigned head = 0, tail = 0;  // wave-uniform ring positions
      for (int base = (tid >> 6) * 64; base < rg.w; base += NT) {
        const int t = base + lane;
        bool keep = false;
        if (t < rg.w) {
          const int4 tr = M.tris[rg.z + t];
          const int2 a = vert_uv(tr.x), b = vert_uv(tr.y), c = vert_uv(tr.z);
          keep = tri_candidate(a.x, a.y, b.x, b.y, c.x, c.y, ca, cb, t0, t1);
        }
        const unsigned long long m = __ballot(keep);
        if (keep) ring[(tail + lanes_below(m)) & 127u] = (unsigned)t;
        tail += (unsigned)__popcll(m);
        wave_sync();
        if (tail - head >= 64u) {
          raster_one(ring[(head + lane) & 127u]);
          head += 64u;
          wave_sync();
        }
      }
      if ((unsigned)lane < tail - head) raster_one(ring[(head + lane) & 127u]);
    }
    __syncthreads();

    // ---- composite against the parent: validity (Eq. 3) and dR ----
    if (P) {
      int sl = 0, dr = 0;
      bool occ = false;
      const float inv_tw = __builtin_amdgcn_rcpf((float)tw);
      for (int k = tid; k < tn; k += NT) {
        const int r = (int)(((float)k + 0.5f) * inv_tw);  // k / tw, exact for k < 2^21
        const int jj = t0 + r, ii = ca + (k - imul(r, tw));
        const unsigned key = tile[k];
        const bool cov = key != kInfBits;
        // only a covered pixel needs the parent, and only one the parent also
        // covers changes (it leaves dR)
        const unsigned pk = (cov && par.has_parent) ? par.depth[imul(jj, W) + ii] : kInfBits;
        const bool pfin = pk != kInfBits;
        occ |= cov && pfin && key < pk;  // positive floats order like their bits
        const bool core_row = jj >= b0 && jj <= b1;
        sl += (cov && core_row);
        dr += (cov && !pfin && core_row);
        if (pfin) tile[k] = kInfBits;
      }
      sl = wave_sum(sl);
      dr = wave_sum(dr);
      const bool any_occ = __ballot(occ) != 0;
      if (lane == 0) {
        atomicAdd(&s_acc[0], sl);
        atomicAdd(&s_acc[1], dr);
        if (any_occ) atomicOr(&s_acc[5], 1);
      }
      __syncthreads();
      if (s_acc[5]) break;
    }

    // ---- dJ_r, dJ_o and U: one pass over the core rows ----
    // Per pixel: the new point q (dR, from the tile) and the observed point p; the
    // same-pixel test settles most points either way.  dJ_r: an unsettled q is
    // unexplained when the dilated observed depth range rules every window pixel
    // out, otherwise the whole wave scans its exact window, two points at a time.
    // dJ_o / U: p needs the dR window when it lies in V(O) or in U; each lane walks
    // its own window of the LDS tile with a depth pre-test (walks come in bunches:
    // measured slower walked by the whole wave).  Hash mode: dJ_r by a range query
    // of the voxel hash.
    {
      const int nk = (b1 - b0 + 1) * tw;
      const int kt = (b0 - t0) * tw;  // tile index of the first core pixel
      const float inv_tw = __builtin_amdgcn_rcpf((float)tw);
      for (int base = 0; base < nk; base += NT) {
        const int k = base + tid;
        int state = 0;  // dJ_r: 1 explained, 2 unexplained, 3 undecided
        bool inV = false, inU = false, expl = false;
        float zq = 0.0f;
        int ii = 0, jj = 0;
        bool hqv = false;
        if (k < nk) {
          // k / tw for k < 2^21: (k + 1/2) / tw is at least 1 / (2 tw) from an integer
          const int r = (int)(((float)k + 0.5f) * inv_tw);
          ii = ca + (k - imul(r, tw));
          jj = b0 + r;
          const unsigned key = tile[kt + k];
          const int pix = imul(jj, W) + ii;
          const float zo = obs[pix];
          const bool hq = key != kInfBits, hp = zo > 0.0f;
          hqv = hq;
          zq = __uint_as_float(key);
          // the same arithmetic as the window scans and the voxel hash, so that
          // every radius mode takes identical decisions
          const float3 q = backproject(cam, ii, jj, zq);
          const float3 p = backproject(cam, ii, jj, zo);
          const float ex = q.x - p.x, ey = q.y - p.y, ez = q.z - p.z;
          const float tq = hq ? delta_margin(cam, zq) : 0.0f;
          const bool same = hq && hp &&
                            within_delta(cam, ex * ex + ey * ey + ez * ez, tq, ii, jj, zq, ii, jj, zo);
          if (hq) {
            if (HQ && ep.radius_mode == 1) {
              state = explained_by_cloud(cam, hs, q.x, q.y, q.z, ii, jj, tq) ? 1 : 2;
            } else if (same) {
              state = 1;
            } else {
              const float2 zr = obs_range[pix];
              state = (zq + ep.dwin < zr.x || zq - ep.dwin > zr.y) ? 2 : 3;
            }
          }
          if (hp) {
            // separate calls, so that the staged copy is read as LDS (not flat)
            const float3 o = apply_obj_map(om, p);
            inV = pl_lds ? in_volume_at(cam, ep, dm, vctr, vbx, s_pl, fr.y, o, ii, jj, zo)
                         : in_volume_at(cam, ep, dm, vctr, vbx, M.planes + fr.x, fr.y, o, ii, jj,
                                        zo);
            inU = goal && ((par.ubits[pix >> 5] >> (pix & 31)) & 1u);
            expl = same;
            if ((inV || inU) && !expl) {
              int ru, rv;
              window_radius(cam, ep, p, ru, rv);
              const float tp = delta_margin(cam, zo);
              const int wja = max(t0, jj - rv), wjb = min(t1, jj + rv);
              const int wia = max(ca, ii - ru), wib = min(cb, ii + ru);
              const float zlo = zo - ep.dwin, zhi = zo + ep.dwin;
              // one flat walk over the clipped window, two pixels per step, stopping
              // after the first hit; the depth pre-test also skips +inf (no point)
              const int n = imul(wib - wia + 1, wjb - wja + 1);
              int iq = wia, jq = wja;
              int row = imul(wja - t0, tw) - ca;  // tile index of (0, jq)
              for (int w = 0; w < n && !expl; w += 2) {
                const bool wrap = iq == wib;  // (ib, jb): the pixel after (iq, jq)
                const int rowb = row + (wrap ? tw : 0), jb = jq + (wrap ? 1 : 0);
                const int ib = wrap ? wia : iq + 1;
                const bool two = w + 1 < n;
                const float za = __uint_as_float(tile[row + iq]);
                const float zb = two ? __uint_as_float(tile[rowb + ib]) : __builtin_inff();
                const bool ina = za >= zlo && za <= zhi, inb = zb >= zlo && zb <= zhi;
                if (ina | inb) {
                  bool h = false;
                  if (ina) {
                    const float3 q = backproject(cam, iq, jq, za);
                    const float ex = q.x - p.x, ey = q.y - p.y, ez = q.z - p.z;
                    h = within_delta(cam, ex * ex + ey * ey + ez * ez, tp, iq, jq, za, ii, jj, zo);
                  }
                  if (inb) {
                    const float3 q = backproject(cam, ib, jb, zb);
                    const float ex = q.x - p.x, ey = q.y - p.y, ez = q.z - p.z;
                    h = h ||
                        within_delta(cam, ex * ex + ey * ey + ez * ez, tp, ib, jb, zb, ii, jj, zo);
                  }
                  expl = h;
                }
                const bool wrap2 = ib == wib;
                row = rowb + (wrap2 ? tw : 0);
                jq = jb + (wrap2 ? 1 : 0);
                iq = wrap2 ? wia : ib + 1;
              }
            }
          }
        }
        if (!P) n_cov += ballot_count(hqv);
        n_dJr += ballot_count(state == 2);
        n_dJo += ballot_count(inV && !expl);
        n_rem += ballot_count(inU && (inV || expl));
        if (GAIN) {  // overlap heuristic: points V(O) adds to V_j
          const int pix = imul(jj, W) + ii;
          const bool inVj = par.vbits && ((par.vbits[pix >> 5] >> (pix & 31)) & 1u);
          n_gain += ballot_count(inV && !inVj);
        }
        unsigned long long und = __ballot(state == 3);
        // wave-uniform: two undecided points at a time, each lane testing one pixel
        // of either window per step, so two observed-depth loads are in flight
        while (und) {
          const int sa = __ffsll((long long)und) - 1;
          und &= und - 1;
          const bool two = und != 0ull;
          const int sb = two ? __ffsll((long long)und) - 1 : sa;
          if (two) und &= und - 1;
          const int ai = __shfl(ii, sa, 64), aj = __shfl(jj, sa, 64);
          const int bi = __shfl(ii, sb, 64), bj = __shfl(jj, sb, 64);
          const float azq = __shfl(zq, sa, 64), bzq = __shfl(zq, sb, 64);
          const float3 aq = backproject(cam, ai, aj, azq);
          const float3 bq = backproject(cam, bi, bj, bzq);
          const float ta = delta_margin(cam, azq), tb = delta_margin(cam, bzq);
          int aru, arv, bru, brv;
          window_radius(cam, ep, aq, aru, arv);
          window_radius(cam, ep, bq, bru, brv);
          const int awu = 2 * aru + 1, anw = imul(awu, 2 * arv + 1);
          const int bwu = 2 * bru + 1, bnw = two ? imul(bwu, 2 * brv + 1) : 0;
          // w / wu for w < 2^21: (w + 1/2) / wu is at least 1 / (2 wu) from an integer
          const float ainv = __builtin_amdgcn_rcpf((float)awu);
          const float binv = __builtin_amdgcn_rcpf((float)bwu);
          bool ahit = false, bhit = !two;
          for (int w0 = 0; w0 < max(anw, bnw) && !(ahit && bhit); w0 += 64) {
            const int w = w0 + lane;
            float za = 0.0f, zb = 0.0f;
            int aii = 0, ajj = 0, bii = 0, bjj = 0;
            if (!ahit && w < anw) {
              const int r = (int)(((float)w + 0.5f) * ainv);
              aii = ai - aru + (w - imul(r, awu));
              ajj = aj - arv + r;
              if (aii >= 0 && aii < W && ajj >= 0 && ajj < H) za = obs[imul(ajj, W) + aii];
            }
            if (!bhit && w < bnw) {
              const int r = (int)(((float)w + 0.5f) * binv);
              bii = bi - bru + (w - imul(r, bwu));
              bjj = bj - brv + r;
              if (bii >= 0 && bii < W && bjj >= 0 && bjj < H) zb = obs[imul(bjj, W) + bii];
            }
            bool ha = false, hb = false;
            if (za > 0.0f) {
              const float3 p = backproject(cam, aii, ajj, za);
              const float dx = p.x - aq.x, dy = p.y - aq.y, dz = p.z - aq.z;
              ha = within_delta(cam, dx * dx + dy * dy + dz * dz, ta, ai, aj, azq, aii, ajj, za);
            }
            if (zb > 0.0f) {
              const float3 p = backproject(cam, bii, bjj, zb);
              const float dx = p.x - bq.x, dy = p.y - bq.y, dz = p.z - bq.z;
              hb = within_delta(cam, dx * dx + dy * dy + dz * dz, tb, bi, bj, bzq, bii, bjj, zb);
            }
            ahit = ahit || __ballot(ha) != 0ull;
            bhit = bhit || __ballot(hb) != 0ull;
          }
          n_dJr += (ahit ? 0 : 1) + (bhit ? 0 : 1);
        }
      }
    }
    __syncthreads();  // the next band overwrites the tile
  }

  if (lane == 0) {
    if (!P) {
      atomicAdd(&s_acc[0], n_cov);
      atomicAdd(&s_acc[1], n_cov);
    }
    atomicAdd(&s_acc[2], n_dJr);
    atomicAdd(&s_acc[3], n_dJo);
    atomicAdd(&s_acc[4], n_rem);
    if (GAIN) atomicAdd(&s_acc[7], n_gain);
  }
  __syncthreads();
  if (tid == 0) {
    const bool valid = s_acc[5] == 0;
    const int res = goal ? (*par.ucount - s_acc[4]) : 0;
    out_status[s] = valid ? 1 : 0;
    out_cost[s] = valid ? s_acc[2] + s_acc[3] + res : -1;
    if (GAIN) out_gain[s] = valid ? s_acc[7] : -1;
    if (out_comps) {  // an invalid successor stops at its first occluding band
      out_comps[5 * s + 0] = valid ? s_acc[0] : -1;
      out_comps[5 * s + 1] = valid ? s_acc[1] : -1;
      out_comps[5 * s + 2] = valid ? s_acc[2] : -1;
      out_comps[5 * s + 3] = valid ? s_acc[3] : -1;
      out_comps[5 * s + 4] = valid ? res : -1;
    }
  }
}

// One workgroup per successor of one parent.
template <int NT, bool VP, bool GAIN, bool HQ, bool G, bool P>
__global__ void __launch_bounds__(NT)
    k_eval(SceneDev S, Parent par, const int2* __restrict__ cands, int n,
           int* __restrict__ out_cost, int* __restrict__ out_status, int* __restrict__ out_comps,
           int* __restrict__ out_gain) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_bb[4];
  __shared__ int s_acc[8];  // S, |dR|, dJ_r, dJ_o, removed-from-U, invalid, near-plane, gain
  __shared__ float4 s_pl[kLdsPlanes];
  __shared__ ObjMap64 s_dm;
  const int s = blockIdx.x;
  if (s >= n) return;
  eval_successor<NT, false, VP, GAIN, HQ, G, P>(S, par, cands[s], s, out_cost, out_status,
                                                out_comps, out_gain, smem, s_bb, s_acc, s_pl,
                                                &s_dm);
}

// Persistent workgroups over a work queue of (parent slot, mesh, pose) items that
// may belong to different scenes: each workgroup takes the next item from an
// atomic counter until the queue is empty, so uneven meshes balance across CUs.
template <int NT, bool VP, bool HQ, bool G, bool P>
__global__ void __launch_bounds__(NT, 4)  // at least 4 waves per SIMD: <= 128 VGPRs
    k_eval_batch(const SceneDev* __restrict__ scenes, const ParentDev* __restrict__ parents,
                 int n_parents, const int4* __restrict__ items, int n, int* counter,
                 int* __restrict__ out_cost, int* __restrict__ out_status,
                 int* __restrict__ out_comps) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_bb[4];
  __shared__ int s_acc[8];
  __shared__ float4 s_pl[kLdsPlanes];
  __shared__ ObjMap64 s_dm;
  __shared__ int s_item;
  for (;;) {
    __syncthreads();  // the previous item is done with LDS
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= n) break;
    const int4 w = items[it];
    const int pslot = __builtin_amdgcn_readfirstlane(w.x);
    if (pslot < 0 || pslot >= n_parents) {
      if (threadIdx.x == 0) {
        out_status[it] = -4;
        out_cost[it] = -1;
        if (out_comps)
          for (int c = 0; c < 5; ++c) out_comps[5 * it + c] = -1;
      }
      continue;
    }
    const ParentDev& pd = parents[pslot];
    Parent par;
    par.depth = pd.depth;
    par.ubits = pd.ubits;
    par.ucount = pd.ucount;
    par.vbits = nullptr;
    par.has_parent = pd.has_parent;
    par.goal = pd.goal;
    const int scene = __builtin_amdgcn_readfirstlane(pd.scene);
    eval_successor<NT, true, VP, false, HQ, G, P>(scenes[scene], par, make_int2(w.y, w.z),
                                                        it,
                                            out_cost, out_status, out_comps, nullptr, smem, s_bb,
                                            s_acc, s_pl, &s_dm);
  }
}

// ---------------------------------------------------------------------------
// local ICP (Sec. IV-E): compensating for the pose discretization
// ---------------------------------------------------------------------------

// Per observed pixel, in FP64: the world point p = Rinv (q - t) of its
// back-projection q (w = 1 when it has a surface normal, else 0; 0 everywhere for
// pixels without a return) and its unit normal facing the camera, from the cross
// product of the central differences of its four pixel neighbours, all observed
// and within `radius` of it.  FP64 keeps the association of the ICP rounds the
// same decisions as exact arithmetic, up to FP64 rounding.
__device__ __forceinline__ double3 world_point64(const Cam& cam, int i, int j, float z) {
  const double dz = z;
  const double q0 = ((double)i - cam.dcx) * dz * cam.dinv_fx - cam.dM[3];
  const double q1 = ((double)j - cam.dcy) * dz * cam.dinv_fy - cam.dM[7];
  const double q2 = dz - cam.dM[11];
  const double* R = cam.dWinv;
  return make_double3(R[0] * q0 + R[1] * q1 + R[2] * q2, R[4] * q0 + R[5] * q1 + R[6] * q2,
                      R[8] * q0 + R[9] * q1 + R[10] * q2);
}

__global__ void k_obs_normals(Cam cam, const float* __restrict__ obs, float radius,
                              double4* __restrict__ pn) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cam.W * cam.H) return;
  const int u = k % cam.W, v = k / cam.W;
  const float z = obs[k];
  double4 P = make_double4(0.0, 0.0, 0.0, 0.0), N = make_double4(0.0, 0.0, 0.0, 0.0);
  if (z > 0.0f) {
    const double3 c = world_point64(cam, u, v, z);
    P = make_double4(c.x, c.y, c.z, 0.0);
    if (u >= 1 && v >= 1 && u <= cam.W - 2 && v <= cam.H - 2) {
      const float z1 = obs[k + 1], z0 = obs[k - 1], z3 = obs[k + cam.W], z2 = obs[k - cam.W];
      if (z0 > 0.0f && z1 > 0.0f && z2 > 0.0f && z3 > 0.0f) {
        const double3 a1 = world_point64(cam, u + 1, v, z1), a0 = world_point64(cam, u - 1, v, z0);
        const double3 b1 = world_point64(cam, u, v + 1, z3), b0 = world_point64(cam, u, v - 1, z2);
        const double r = radius;
        auto dist = [&](double3 p) {
          const double dx = c.x - p.x, dy = c.y - p.y, dz = c.z - p.z;
          return sqrt(dx * dx + dy * dy + dz * dz);
        };
        if (dist(a1) <= r && dist(a0) <= r && dist(b1) <= r && dist(b0) <= r) {
          const double ex = a1.x - a0.x, ey = a1.y - a0.y, ez = a1.z - a0.z;
          const double fx = b1.x - b0.x, fy = b1.y - b0.y, fz = b1.z - b0.z;
          const double nx = ey * fz - ez * fy, ny = ez * fx - ex * fz, nz = ex * fy - ey * fx;
          const double len = sqrt(nx * nx + ny * ny + nz * nz);
          if (len > 0.0) {
            // towards the camera centre (world_from_cam's translation)
            const double tw = nx * (cam.dWinv[3] - c.x) + ny * (cam.dWinv[7] - c.y) +
                              nz * (cam.dWinv[11] - c.z);
            const double sg = tw < 0.0 ? -1.0 : 1.0;
            N = make_double4(sg * nx / len, sg * ny / len, sg * nz / len, 0.0);
            P.w = 1.0;
          }
        }
      }
    }
  }
  pn[2 * (size_t)k] = P;
  pn[2 * (size_t)k + 1] = N;
}

// cos and sin of x in FP64 without a library call: x is halved until |x| <= 1/4,
// the Taylor series of both (to x^17, truncation below 1e-20) is summed, and the
// double-angle formulas undo the halvings (each at most doubles the relative
// rounding error: a few 1e-15 for ICP's steps).
__device__ __forceinline__ void cos_sin64(double x, double& c, double& s) {
  int h = 0;
  while (fabs(x) > 0.25 && h < 64) {
    x *= 0.5;
    ++h;
  }
  const double x2 = x * x;
  double cs = 1.0, sn = 1.0, tc = 1.0, ts = 1.0;
  for (int k = 1; k <= 8; ++k) {  // terms x^(2k) / (2k)! and x^(2k+1) / (2k+1)!
    tc *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
    ts *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
    cs += tc;
    sn += ts;
  }
  sn *= x;
  for (int k = 0; k < h; ++k) {
    const double c2 = cs * cs - sn * sn, s2 = 2.0 * sn * cs;
    cs = c2;
    sn = s2;
  }
  c = cs;
  s = sn;
}

// Raw sums of one association round, reduced over the workgroup: matches, the
// moved model points (x, y, relative to the grid position), and the products of
// g = n_y a_x - n_x a_y, n_x, n_y and the residual r = n.(a - p).
constexpr int kIcpSums = 12;

// One workgroup per candidate: render it into the LDS tile, composite against the
// parent (an occluding candidate is not aligned), then `iters` rounds over the
// non-occluded pixels dR: move each model point by the motion so far, associate it
// with the observed point at the nearest pixel of its projection when that point
// has a normal and lies within `radius`, and take one point-to-plane step (a
// rotation about the vertical axis through the matched points' centroid and a
// translation, from the damped 3 x 3 normal equations).  Writes the adjusted pose
// to arena[s] and (mesh, base + s) to out_obj[s].  CACHE: snapped vertices kept in
// LDS (meshes of at most 5,120 vertices), else recomputed where they are needed.
template <int NT, bool CACHE>
__global__ void __launch_bounds__(NT, 4)  // at least 4 waves per SIMD: two workgroups per CU
    k_icp(SceneDev S, Parent par, const int2* __restrict__ cands, int n, IcpArgs ia,
          int2* __restrict__ out_obj, int* __restrict__ out_match, int* __restrict__ out_status) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_bb[4];
  __shared__ int s_flag[3];  // vertex stage failed, occludes the parent, stop
  __shared__ double s_red[NT / 64][kIcpSums];
  __shared__ double s_T[4];  // cos phi, sin phi, tx, ty of the motion so far
  __shared__ int s_nm;
  const int s = blockIdx.x;
  if (s >= n) return;
  if (ia.retry && out_status[s] != -3) return;  // settled by the pass with the smaller tile
  const Cam& cam = S.cam;
  const Meshes& M = S.M;
  const EvalParams& ep = S.ep;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int W = cam.W, H = cam.H;
  const int2 cd = cands[s];
  if (cd.x < 0 || cd.x >= ep.n_mesh || cd.y < 0 || cd.y >= ep.n_poses) {
    if (tid == 0) {
      out_status[s] = -4;
      out_match[s] = 0;
      out_obj[s] = cd;
      ia.arena[s] = make_float4(0.0f, 0.0f, 1.0f, 0.0f);
    }
    return;
  }
  const float4 pz = S.poses[cd.y];
  const int4 rg = M.range[cd.x];
  int2* suv = reinterpret_cast<int2*>(smem);
  unsigned* tile =
      reinterpret_cast<unsigned*>(smem + (CACHE ? (size_t)ep.max_nv * sizeof(int2) : 0));
  unsigned* ring = tile + ep.tile_px + (tid >> 6) * 128;
  if (tid < 4) s_bb[tid] = tid < 2 ? INT_MAX : INT_MIN;
  if (tid < 3) s_flag[tid] = 0;
  if (tid == 0) {
    s_T[0] = 1.0;
    s_T[1] = s_T[2] = s_T[3] = 0.0;
    s_nm = 0;
  }
  __syncthreads();
  {
    int xmn = INT_MAX, ymn = INT_MAX, xmx = INT_MIN, ymx = INT_MIN;
    bool bad = false;
    for (int v = tid; v < rg.y; v += NT) {
      float X, Y, Z;
      vcam(cam, pz, M.verts[rg.x + v], X, Y, Z);
      int U, V;
      bad |= !vsnap(cam, X, Y, Z, U, V);
      if (CACHE) suv[v] = make_int2(U, V);
      xmn = min(xmn, U);
      ymn = min(ymn, V);
      xmx = max(xmx, U);
      ymx = max(ymx, V);
    }
    xmn = wave_min(xmn);
    ymn = wave_min(ymn);
    xmx = wave_max(xmx);
    ymx = wave_max(ymx);
    const bool any_bad = __ballot(bad) != 0;
    if (lane == 0) {
      atomicMin(&s_bb[0], xmn);
      atomicMin(&s_bb[1], ymn);
      atomicMax(&s_bb[2], xmx);
      atomicMax(&s_bb[3], ymx);
      if (any_bad) s_flag[0] = 1;
    }
  }
  __syncthreads();
  auto vert_uv = [&](int idx) -> int2 {
    if (CACHE) return suv[idx];
    float X, Y, Z;
    vcam(cam, pz, M.verts[rg.x + idx], X, Y, Z);
    int U, V;
    vsnap(cam, X, Y, Z, U, V);
    return make_int2(U, V);
  };
  auto finish = [&](int status, int nm, float4 pose) {
    if (tid == 0) {
      out_status[s] = status;
      out_match[s] = nm;
      out_obj[s] = make_int2(cd.x, ia.base + s);
      ia.arena[s] = pose;
    }
  };
  if (s_flag[0]) {
    finish(-2, 0, pz);
    return;
  }
  const int ca = max(0, floor256(s_bb[0]) - 1), cb = min(W - 1, ceil256(s_bb[2]) + 1);
  const int ra = max(0, floor256(s_bb[1]) - 1), rb = min(H - 1, ceil256(s_bb[3]) + 1);
  const int tw = cb - ca + 1, nrows = rb - ra + 1;
  if (tw <= 0 || nrows <= 0) {  // nothing in view: nothing to align
    finish(1, 0, pz);
    return;
  }
  if (tw * nrows > ep.tile_px) {
    finish(-3, 0, pz);
    return;
  }
  const int tn = tw * nrows;
  for (int k = tid; k < tn; k += NT) tile[k] = kInfBits;
  __syncthreads();
  // rasterise (front faces queued per wave as in the successor kernel)
  {
    auto raster_one = [&](unsigned t) {
      const int4 tr = M.tris[rg.z + t];
      const float4 v0 = M.verts[rg.x + tr.x], v1 = M.verts[rg.x + tr.y];
      const float4 v2 = M.verts[rg.x + tr.z];
      const int2 a = vert_uv(tr.x), b = vert_uv(tr.y), c = vert_uv(tr.z);
      float X0, Y0, Z0, X1, Y1, Z1, X2, Y2, Z2;
      vcam(cam, pz, v0, X0, Y0, Z0);
      vcam(cam, pz, v1, X1, Y1, Z1);
      vcam(cam, pz, v2, X2, Y2, Z2);
      const Plane64 pl = make_plane(cam, X0, Y0, Z0, X1, Y1, Z1, X2, Y2, Z2);
      raster_tri(a.x, a.y, b.x, b.y, c.x, c.y, ca, cb, ra, rb, [&](int i, int j) {
        atomicMin(&tile[(j - ra) * tw + (i - ca)], __float_as_uint(plane_depth(pl, i, j)));
      });
    };
    unsigned head = 0, tail = 0;
    for (int base = (tid >> 6) * 64; base < rg.w; base += NT) {
      const int t = base + lane;
      bool keep = false;
      if (t < rg.w) {
        const int4 tr = M.tris[rg.z + t];
        const int2 a = vert_uv(tr.x), b = vert_uv(tr.y), c = vert_uv(tr.z);
        keep = tri_candidate(a.x, a.y, b.x, b.y, c.x, c.y, ca, cb, ra, rb);
      }
      const unsigned long long m = __ballot(keep);
      if (keep) ring[(tail + lanes_below(m)) & 127u] = (unsigned)t;
      tail += (unsigned)__popcll(m);
      wave_sync();
      if (tail - head >= 64u) {
        raster_one(ring[(head + lane) & 127u]);
        head += 64u;
        wave_sync();
      }
    }
    if ((unsigned)lane < tail - head) raster_one(ring[(head + lane) & 127u]);
  }
  __syncthreads();
  // k / tw for k < 2^21: (k + 1/2) / tw is at least 1 / (2 tw) from an integer
  const float inv_tw = __builtin_amdgcn_rcpf((float)tw);
  // composite: validity (Eq. 3) and the non-occluded part dR
  {
    bool occ = false;
    for (int k = tid; k < tn; k += NT) {
      const int r = (int)(((float)k + 0.5f) * inv_tw);
      const int jj = ra + r, ii = ca + (k - r * tw);
      const unsigned key = tile[k];
      const bool cov = key != kInfBits;
      const unsigned pk = par.has_parent ? par.depth[jj * W + ii] : kInfBits;
      const bool pfin = pk != kInfBits;
      occ |= cov && pfin && key < pk;
      tile[k] = (cov && !pfin) ? key : kInfBits;
    }
    if (__ballot(occ) != 0ull && lane == 0) s_flag[1] = 1;
  }
  __syncthreads();
  if (s_flag[1]) {
    finish(0, 0, pz);
    return;
  }
  // ICP rounds in FP64, as exact arithmetic up to FP64 rounding: each model point
  // (the back-projection of its float32 depth, world frame) is moved by the
  // motion so far, projected, and paired with the observed point at the nearest
  // pixel; thread 0 solves for the step
  double cphi = 1.0, sphi = 0.0, mtx = 0.0, mty = 0.0;  // the motion so far
  const double r2 = (double)ia.radius * (double)ia.radius;
  const double ox = pz.x, oy = pz.y;  // local origin of the sums
  for (int it = 0; it < ia.iters; ++it) {
    const double cT = s_T[0], sT = s_T[1], txT = s_T[2], tyT = s_T[3];
    double acc[kIcpSums];
    for (int q = 0; q < kIcpSums; ++q) acc[q] = 0.0;
#pragma unroll 1
    for (int k = tid; k < tn; k += NT) {
      const unsigned key = tile[k];
      if (key == kInfBits) continue;
      const int r = (int)(((float)k + 0.5f) * inv_tw);
      const int jj = ra + r, ii = ca + (k - r * tw);
      const double3 w = world_point64(cam, ii, jj, __uint_as_float(key));
      const double ax = cT * w.x - sT * w.y + txT, ay = sT * w.x + cT * w.y + tyT, az = w.z;
      const double* Md = cam.dM;
      const double cx = Md[0] * ax + Md[1] * ay + Md[2] * az + Md[3];
      const double cy = Md[4] * ax + Md[5] * ay + Md[6] * az + Md[7];
      const double cz = Md[8] * ax + Md[9] * ay + Md[10] * az + Md[11];
      if (!(cz > 0.0)) continue;
      const double iz = 1.0 / cz;
      const double uf = cam.dfx * cx * iz + cam.dcx, vf = cam.dfy * cy * iz + cam.dcy;
      const double fu = floor(uf + 0.5), fv = floor(vf + 0.5);
      if (!(fu >= 0.0 && fu <= (double)(W - 1) && fv >= 0.0 && fv <= (double)(H - 1))) continue;
      const size_t pix = (size_t)fv * W + (size_t)fu;
      const double4 P = ia.pn[2 * pix];
      if (!(P.w > 0.0)) continue;
      const double dx = ax - P.x, dy = ay - P.y, dz = az - P.z;
      if (dx * dx + dy * dy + dz * dz > r2) continue;
      const double4 N = ia.pn[2 * pix + 1];
      const double lx = ax - ox, ly = ay - oy;
      const double g = N.y * lx - N.x * ly;
      const double res = N.x * dx + N.y * dy + N.z * dz;
      acc[0] += 1.0;
      acc[1] += lx;
      acc[2] += ly;
      acc[3] += g * g;
      acc[4] += g * N.x;
      acc[5] += g * N.y;
      acc[6] += N.x * N.x;
      acc[7] += N.x * N.y;
      acc[8] += N.y * N.y;
      acc[9] += g * res;
      acc[10] += N.x * res;
      acc[11] += N.y * res;
    }
    for (int q = 0; q < kIcpSums; ++q) {
      double v = acc[q];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) s_red[wv][q] = v;
    }
    __syncthreads();
    if (tid == 0) {
      double t[kIcpSums];
      for (int q = 0; q < kIcpSums; ++q) {
        t[q] = 0.0;
        for (int w = 0; w < NT / 64; ++w) t[q] += s_red[w][q];
      }
      const int nm = (int)t[0];
      s_nm = nm;
      if (nm < 3) {
        s_flag[2] = 1;
      } else {
        const double cx = t[1] / nm, cy = t[2] / nm;  // centroid, local frame
        // normal equations of J = (g - (c_x n_y - c_y n_x), n_x, n_y), b = -J r
        double A[3][3], b[3];
        A[0][0] = t[3] - 2.0 * (cx * t[5] - cy * t[4]) + cx * cx * t[8] - 2.0 * cx * cy * t[7] +
                  cy * cy * t[6];
        A[0][1] = A[1][0] = t[4] - cx * t[7] + cy * t[6];
        A[0][2] = A[2][0] = t[5] - cx * t[8] + cy * t[7];
        A[1][1] = t[6];
        A[1][2] = A[2][1] = t[7];
        A[2][2] = t[8];
        b[0] = -(t[9] - cx * t[11] + cy * t[10]);
        b[1] = -t[10];
        b[2] = -t[11];
        for (int u = 0; u < 3; ++u) A[u][u] += 1e-6 * A[u][u] + 1e-12;
        auto det3 = [](const double (&m)[3][3]) {
          return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
                 m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
                 m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
        };
        const double det = det3(A);
        double x[3];
        for (int c = 0; c < 3; ++c) {
          double Mc[3][3];
          for (int u = 0; u < 3; ++u)
            for (int v = 0; v < 3; ++v) Mc[u][v] = v == c ? b[u] : A[u][v];
          x[c] = det3(Mc) / det;
        }
        // the step about the world z axis: t' = c_w + t - R c_w; composed after the
        // motion so far (rotations compose by the angle-sum formulas)
        double co, si;
        cos_sin64(x[0], co, si);
        const double cwx = cx + ox, cwy = cy + oy;
        const double stx = cwx + x[1] - (co * cwx - si * cwy);
        const double sty = cwy + x[2] - (si * cwx + co * cwy);
        const double nx = co * mtx - si * mty + stx, ny = si * mtx + co * mty + sty;
        const double nc = co * cphi - si * sphi, ns = si * cphi + co * sphi;
        cphi = nc;
        sphi = ns;
        mtx = nx;
        mty = ny;
        s_T[0] = cphi;
        s_T[1] = sphi;
        s_T[2] = mtx;
        s_T[3] = mty;
      }
    }
    __syncthreads();
    if (s_flag[2]) break;
  }
  if (tid == 0) {
    const double co = cphi, si = sphi;
    const double x = pz.x, y = pz.y, pc = pz.z, ps = pz.w;
    finish(1, s_nm,
           make_float4((float)(co * x - si * y + mtx), (float)(si * x + co * y + mty),
                       (float)(pc * co - ps * si), (float)(ps * co + pc * si)));
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static int blocks_for(size_t n, int t) { return (int)std::min<size_t>((n + t - 1) / t, 65535); }

void launch_fill_u32(unsigned* p, unsigned v, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, v, n);
}
void launch_fill_i32(int* p, int v, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, v, n);
}

void launch_hash_insert(const Cam& cam, const float* depth, unsigned long long* keys, int* counts,
                        int mask, float inv_cell, int* n_points, hipStream_t s) {
  const int n = cam.W * cam.H;
  hipLaunchKernelGGL(k_hash_insert, dim3((n + 255) / 256), dim3(256), 0, s, cam, depth, keys,
                     counts, mask, inv_cell, n_points);
}
void launch_scan_cells(const int* counts, int2* cells, int n_slots, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_cells, dim3(1), dim3(1024), 0, s, counts, cells, n_slots);
}
void launch_hash_scatter(const Cam& cam, const float* depth, const unsigned long long* keys,
                         const int2* cells, int* fill, float4* pts, int mask, float inv_cell,
                         hipStream_t s) {
  const int n = cam.W * cam.H;
  hipLaunchKernelGGL(k_hash_scatter, dim3((n + 255) / 256), dim3(256), 0, s, cam, depth, keys,
                     cells, fill, pts, mask, inv_cell);
}

void launch_obs_range(const Cam& cam, const float* obs, float2* out, int R, hipStream_t s) {
  const int n = cam.W * cam.H;
  hipLaunchKernelGGL(k_obs_range, dim3((n + 255) / 256), dim3(256), 0, s, cam, obs, out, R);
}

void launch_render_object(const Cam& cam, const Meshes& M, const float4* poses, int mesh,
                          int pose, int n_tris, unsigned* depth_bits, hipStream_t s) {
  if (n_tris <= 0) return;
  hipLaunchKernelGGL(k_render_object, dim3((n_tris + 127) / 128), dim3(128), 0, s, cam, M,
                     poses, mesh, pose, depth_bits);
}

void launch_render_objects(const Cam& cam, const Meshes& M, const float4* poses,
                           const int* mesh_pose, int j, int max_tris, unsigned* depth_bits,
                           hipStream_t s) {
  if (j <= 0 || max_tris <= 0) return;
  ParentObjs po;
  for (int a = 0; a < kMaxObjects; ++a)
    po.o[a] = a < j ? make_int2(mesh_pose[2 * a], mesh_pose[2 * a + 1]) : make_int2(0, 0);
  hipLaunchKernelGGL(k_render_objects, dim3((max_tris + 127) / 128, j), dim3(128), 0, s, cam, M,
                     poses, po, j, depth_bits);
}

void launch_parent_u(const Cam& cam, const Meshes& M, const float4* poses, const float* obs,
                     const int* par_mesh_pose, int j, const unsigned* depth_bits, unsigned* ubits,
                     int* ucount, const EvalParams& ep, hipStream_t s) {
  ParentObjs po;
  for (int a = 0; a < kMaxObjects; ++a)
    po.o[a] = a < j ? make_int2(par_mesh_pose[2 * a], par_mesh_pose[2 * a + 1]) : make_int2(0, 0);
  const int n = cam.W * cam.H;
  hipLaunchKernelGGL(k_parent_u, dim3((n + 255) / 256), dim3(256), 0, s, cam, M, poses, obs, po,
                     j, depth_bits, ubits, ucount, ep);
}

void launch_parent_v(const Cam& cam, const Meshes& M, const float4* poses, const float* obs,
                     const int* par_mesh_pose, int j, unsigned* vbits, const EvalParams& ep,
                     hipStream_t s) {
  ParentObjs po;
  for (int a = 0; a < kMaxObjects; ++a)
    po.o[a] = a < j ? make_int2(par_mesh_pose[2 * a], par_mesh_pose[2 * a + 1]) : make_int2(0, 0);
  const int n = cam.W * cam.H;
  launch_fill_u32(vbits, 0u, (size_t)(n + 31) / 32, s);
  if (j > 0)
    hipLaunchKernelGGL(k_parent_v, dim3((n + 255) / 256), dim3(256), 0, s, cam, M, poses, obs, po,
                       j, vbits, ep);
}

template <class K>
static hipError_t allow_lds(K kernel, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int NT, bool VP, bool GAIN, bool HQ, bool G, bool P>
static hipError_t launch_eval_g(const SceneDev& S, const Parent& par, const int2* cands, int n,
                                int* cost, int* status, int* comps, int* gain, size_t lds,
                                hipStream_t s) {
  hipError_t e = allow_lds(&k_eval<NT, VP, GAIN, HQ, G, P>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_eval<NT, VP, GAIN, HQ, G, P>), dim3(n), dim3(NT), lds, s, S, par, cands,
                     n, cost, status, comps, gain);
  return hipGetLastError();
}

template <int NT, bool VP, bool HQ, bool G, bool P>
static hipError_t launch_eval_t(const SceneDev& S, const Parent& par, const int2* cands, int n,
                                int* cost, int* status, int* comps, int* gain, size_t lds,
                                hipStream_t s) {
  return gain ? launch_eval_g<NT, VP, true, HQ, G, P>(S, par, cands, n, cost, status, comps, gain,
                                                      lds, s)
              : launch_eval_g<NT, VP, false, HQ, G, P>(S, par, cands, n, cost, status, comps,
                                                       gain, lds, s);
}

template <bool VP, bool HQ, bool G, bool P>
static hipError_t launch_eval_vp(int threads, const SceneDev& S, const Parent& par,
                                 const int2* cands, int n, int* cost, int* status, int* comps,
                                 int* gain, size_t lds, hipStream_t s) {
  switch (threads) {
    case 64:
      return launch_eval_t<64, VP, HQ, G, P>(S, par, cands, n, cost, status, comps, gain, lds, s);
    case 128:
      return launch_eval_t<128, VP, HQ, G, P>(S, par, cands, n, cost, status, comps, gain, lds,
                                              s);
    case 512:
      return launch_eval_t<512, VP, HQ, G, P>(S, par, cands, n, cost, status, comps, gain, lds,
                                              s);
    case 1024:
      return launch_eval_t<1024, VP, HQ, G, P>(S, par, cands, n, cost, status, comps, gain, lds,
                                               s);
    default:
      return launch_eval_t<256, VP, HQ, G, P>(S, par, cands, n, cost, status, comps, gain, lds,
                                              s);
  }
}

// Hash-mode scenes and goal-level parents take instantiations with the goal-level
// and parent code; below the goal, the root takes the one without a parent.
template <bool VP>
static hipError_t launch_eval_hq(int threads, const SceneDev& S, const Parent& par,
                                 const int2* cands, int n, int* cost, int* status, int* comps,
                                 int* gain, size_t lds, hipStream_t s) {
  if (S.ep.radius_mode == 1)
    return launch_eval_vp<VP, true, true, true>(threads, S, par, cands, n, cost, status, comps,
                                                gain, lds, s);
  if (par.goal)
    return launch_eval_vp<VP, false, true, true>(threads, S, par, cands, n, cost, status, comps,
                                                 gain, lds, s);
  return par.has_parent ? launch_eval_vp<VP, false, false, true>(threads, S, par, cands, n, cost,
                                                                 status, comps, gain, lds, s)
                        : launch_eval_vp<VP, false, false, false>(threads, S, par, cands, n,
                                                                  cost, status, comps, gain,
                                                                  lds, s);
}

hipError_t launch_eval(int threads, const SceneDev& S, const Parent& par, const int2* cands,
                       int n, int* cost, int* status, int* comps, int* gain, size_t lds_bytes,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  return S.ep.vpack ? launch_eval_hq<true>(threads, S, par, cands, n, cost, status, comps, gain,
                                           lds_bytes, s)
                    : launch_eval_hq<false>(threads, S, par, cands, n, cost, status, comps,
                                            gain, lds_bytes, s);
}

template <int NT, bool VP, bool HQ, bool G, bool P>
static hipError_t prepare_eval_batch_t(size_t lds, int* per_cu) {
  hipError_t e = allow_lds(&k_eval_batch<NT, VP, HQ, G, P>, lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_eval_batch<NT, VP, HQ, G, P>, NT,
                                                      lds);
}

template <bool VP, bool HQ, bool G, bool P>
static hipError_t prepare_eval_batch_vp(int threads, size_t lds, int* per_cu) {
  switch (threads) {
    case 64:
      return prepare_eval_batch_t<64, VP, HQ, G, P>(lds, per_cu);
    case 128:
      return prepare_eval_batch_t<128, VP, HQ, G, P>(lds, per_cu);
    case 512:
      return prepare_eval_batch_t<512, VP, HQ, G, P>(lds, per_cu);
    default:
      return prepare_eval_batch_t<256, VP, HQ, G, P>(lds, per_cu);
  }
}

template <bool VP>
static hipError_t prepare_eval_batch_f(int threads, int flags, size_t lds, int* per_cu) {
  if (flags & kBatchHash) return prepare_eval_batch_vp<VP, true, true, true>(threads, lds, per_cu);
  if (flags & kBatchGoal) return prepare_eval_batch_vp<VP, false, true, true>(threads, lds, per_cu);
  if (flags & kBatchParent)
    return prepare_eval_batch_vp<VP, false, false, true>(threads, lds, per_cu);
  return prepare_eval_batch_vp<VP, false, false, false>(threads, lds, per_cu);
}

hipError_t prepare_eval_batch(int threads, int vpack, int flags, size_t lds_bytes,
                              int* blocks_per_cu) {
  return vpack ? prepare_eval_batch_f<true>(threads, flags, lds_bytes, blocks_per_cu)
               : prepare_eval_batch_f<false>(threads, flags, lds_bytes, blocks_per_cu);
}

template <int NT, bool VP, bool HQ, bool G, bool P>
static hipError_t launch_eval_batch_t(const SceneDev* scenes, const ParentDev* parents,
                                      int n_parents, const int4* items, int n, int* counter,
                                      int* cost, int* status, int* comps, size_t lds, int grid,
                                      hipStream_t s) {
  grid = std::max(1, std::min(grid, n));
  hipLaunchKernelGGL((k_eval_batch<NT, VP, HQ, G, P>), dim3(grid), dim3(NT), lds, s, scenes,
                     parents, n_parents, items, n, counter, cost, status, comps);
  return hipGetLastError();
}

template <bool VP, bool HQ, bool G, bool P>
static hipError_t launch_eval_batch_vp(int threads, const SceneDev* scenes,
                                       const ParentDev* parents, int n_parents, const int4* items,
                                       int n, int* counter, int* cost, int* status, int* comps,
                                       size_t lds, int grid, hipStream_t s) {
  switch (threads) {
    case 64:
      return launch_eval_batch_t<64, VP, HQ, G, P>(scenes, parents, n_parents, items, n, counter,
                                                   cost, status, comps, lds, grid, s);
    case 128:
      return launch_eval_batch_t<128, VP, HQ, G, P>(scenes, parents, n_parents, items, n,
                                                    counter, cost, status, comps, lds, grid, s);
    case 512:
      return launch_eval_batch_t<512, VP, HQ, G, P>(scenes, parents, n_parents, items, n,
                                                    counter, cost, status, comps, lds, grid, s);
    default:
      return launch_eval_batch_t<256, VP, HQ, G, P>(scenes, parents, n_parents, items, n,
                                                    counter, cost, status, comps, lds, grid, s);
  }
}

// The batch's flags (over its whole parent table) pick the leanest instantiation
// that covers every item, as for single-parent launches.
template <bool VP>
static hipError_t launch_eval_batch_f(int threads, int flags, const SceneDev* scenes,
                                      const ParentDev* parents, int n_parents, const int4* items,
                                      int n, int* counter, int* cost, int* status, int* comps,
                                      size_t lds, int grid, hipStream_t s) {
  if (flags & kBatchHash)
    return launch_eval_batch_vp<VP, true, true, true>(threads, scenes, parents, n_parents, items,
                                                      n, counter, cost, status, comps, lds, grid,
                                                      s);
  if (flags & kBatchGoal)
    return launch_eval_batch_vp<VP, false, true, true>(threads, scenes, parents, n_parents, items,
                                                       n, counter, cost, status, comps, lds,
                                                       grid, s);
  if (flags & kBatchParent)
    return launch_eval_batch_vp<VP, false, false, true>(threads, scenes, parents, n_parents,
                                                        items, n, counter, cost, status, comps,
                                                        lds, grid, s);
  return launch_eval_batch_vp<VP, false, false, false>(threads, scenes, parents, n_parents, items,
                                                       n, counter, cost, status, comps, lds, grid,
                                                       s);
}

hipError_t launch_eval_batch(int threads, int vpack, int flags, const SceneDev* scenes,
                             const ParentDev* parents, int n_parents, const int4* items, int n,
                             int* counter, int* cost, int* status, int* comps, size_t lds_bytes,
                             int grid, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  launch_fill_i32(counter, 0, 1, s);  // a fill kernel (not a memset): safe in captured graphs
  return vpack ? launch_eval_batch_f<true>(threads, flags, scenes, parents, n_parents, items, n,
                                           counter, cost, status, comps, lds_bytes, grid, s)
               : launch_eval_batch_f<false>(threads, flags, scenes, parents, n_parents, items, n,
                                            counter, cost, status, comps, lds_bytes, grid, s);
}

void launch_obs_normals(const Cam& cam, const float* obs, float radius, double4* pn,
                        hipStream_t s) {
  const int n = cam.W * cam.H;
  hipLaunchKernelGGL(k_obs_normals, dim3((n + 255) / 256), dim3(256), 0, s, cam, obs, radius, pn);
}

template <bool CACHE>
static hipError_t launch_icp_t(const SceneDev& S, const Parent& par, const int2* cands, int n,
                               const IcpArgs& ia, int2* out_obj, int* out_match,
                               int* out_status, size_t lds, hipStream_t s) {
  hipError_t e = allow_lds(&k_icp<kIcpThreads, CACHE>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_icp<kIcpThreads, CACHE>), dim3(n), dim3(kIcpThreads), lds, s, S, par,
                     cands, n, ia, out_obj, out_match, out_status);
  return hipGetLastError();
}

hipError_t launch_icp(const SceneDev& S, const Parent& par, const int2* cands, int n,
                      const IcpArgs& ia, int2* out_obj, int* out_match, int* out_status,
                      bool vertex_cache, size_t lds, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  return vertex_cache
             ? launch_icp_t<true>(S, par, cands, n, ia, out_obj, out_match, out_status, lds, s)
             : launch_icp_t<false>(S, par, cands, n, ia, out_obj, out_match, out_status, lds, s);
}

}  // namespace perch
