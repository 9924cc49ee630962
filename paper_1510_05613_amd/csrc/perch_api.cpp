// perch_api.cpp -- the C ABI of libperch.so (declared in include/perch.h).
//
// Host side of PERCH successor evaluation (arXiv:1510.05613): owns the scene's
// device buffers (observed depth, voxel hash of I, mesh library, pose table,
// parent buffers), materialises a parent state R_j before its successors are
// evaluated (Sec. IV-A), and launches the gfx950 kernels on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "perch_ctx.h"

using namespace perch;
static_assert(kMaxObjects == PERCH_MAX_OBJECTS, "device and ABI object limits differ");

namespace perch {

namespace {
thread_local std::string g_err;
}

namespace {
std::atomic<long long> g_dev_bytes{0};
}

bool dev_mem_admit(size_t n) {
  const char* cap = std::getenv("PERCH_DEVICE_MEM_CAP");
  if (!cap || !*cap) return true;
  char* end = nullptr;
  const unsigned long long c = std::strtoull(cap, &end, 10);
  if (end == cap) return true;  // not a number: no cap
  return (unsigned long long)g_dev_bytes.load() + n <= c;
}

void dev_mem_account(long long delta) { g_dev_bytes += delta; }

perch_status fail(perch_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

// Float32 error of the observed-point volume test.  u = 2^-24 is float32's unit
// roundoff.
//  - Vertex-box pre-test on o = A p + b (float32 back-projection p, float32 map A, b
//    of the camera-to-object transform): each coordinate of p carries <= 4u of its
//    size, the entries of A (products of the rounded world_from_cam and the pose's
//    cos / sin divided by cos^2 + sin^2) <= 12u, b (camera position relative to the
//    pose, |b| <= Tm) <= 16u |b|, and the fused chain three more roundings of its
//    partial sums; together well below 64u (|p|_1 + Tm) with |p|_1 <= zmax (1 +
//    amax + bmax) over the observed points.  vbox = 64u (Pm + Tm) + 1e-6 m, so a
//    point the float32 test puts more than vbox outside the vertex box is outside.
//  - Plane test: o in FP64 (within 1e-15 m of the exact map of the same float32
//    inputs), rounded to float32 (u |o| per coordinate), then s = n.o - d by three
//    fused roundings (<= 3.01u (|o| + |d|) for unit n).  Inside the box widened by
//    vbox, |o| <= Rm + 2 vbox, so vtau = 8u (Rm + 2 vbox + Wm) + 1e-12 m bounds the
//    float32 error of every plane value; a plane value beyond +-vtau has the sign of
//    the exact one, and the rest are decided in FP64.
//  - Plane test on the float32 point o32 itself: each coordinate within vbox of the
//    exact point, so a unit normal moves the plane value by at most sqrt(3) vbox,
//    and the fused chain rounds as above: vtau32 = sqrt(3) vbox + vtau (inflated by
//    1e-3) bounds its error, and only values within it need the FP64 point.
void vol_margins(const Cam& cam, float obs_zmax, float pose_xy_max, float mesh_rmax,
                 float mesh_wmax, float& vbox, float& vtau, float& vtau32) {
  const double u = std::ldexp(1.0, -24);
  const double amax = std::max(std::fabs((double)cam.cx), std::fabs(cam.W - 1.0 - cam.cx)) / cam.fx;
  const double bmax = std::max(std::fabs((double)cam.cy), std::fabs(cam.H - 1.0 - cam.cy)) / cam.fy;
  const double Pm = (double)obs_zmax * (1.0 + amax + bmax);
  const double Tm = std::fabs(cam.dWinv[3]) + std::fabs(cam.dWinv[7]) +
                    std::fabs(cam.dWinv[11]) + pose_xy_max + 0.1;  // + local ICP moves
  const double vb = 64.0 * u * (Pm + Tm) + 1e-6;
  vbox = (float)vb;
  const double vt = 8.0 * u * (mesh_rmax + 2.0 * vb + mesh_wmax) + 1e-12;
  vtau = (float)vt;
  vtau32 = (float)((std::sqrt(3.0) * vb + vt) * (1.0 + 1e-3));
}

// Margin of the float32 test |q - p|^2 <= delta^2 for pixel points q = (i_q, j_q,
// z_q) and p (both inside the image), each back-projected in float32 as ((i - cx) z)
// (1/fx): every coordinate within 4u of its size, z exact.  With K = amax + bmax (the
// largest |i - cx| / fx and |j - cy| / fy) and the fixed point at depth z, the other
// within d of it, the error vector of the float32 difference has length <= A + B d,
// A = 8u K z, B = 4u K + 2u, and the rounded d^2 and delta^2 add 3u d^2 and u delta^2.
// So |t - (d^2 - delta^2)| <= 2 delta A + delta^2 (2B + 4u) + 2 (A + B delta)^2 for t =
// the float32 d^2 - delta^2 whenever its sign could be wrong; tau is twice that:
// tau(z) = t_lin z + t_0 + 4 (t_a z + t_s)^2.  |t| > tau decides by its sign; the
// rest is decided in FP64 (needs delta much larger than A, i.e. delta >= 1e-4 m).
static void delta_margins(Cam& cam) {
  const double u = std::ldexp(1.0, -24);
  const double amax = std::max(std::fabs((double)cam.cx), std::fabs(cam.W - 1.0 - cam.cx)) / cam.fx;
  const double bmax = std::max(std::fabs((double)cam.cy), std::fabs(cam.H - 1.0 - cam.cy)) / cam.fy;
  const double K = amax + bmax, d = cam.delta;
  const double ta = 8.0 * u * K, B = 4.0 * u * K + 2.0 * u;
  cam.t_lin = (float)(4.0 * d * ta * (1.0 + 1e-3));
  cam.t_0 = (float)(d * d * (4.0 * B + 8.0 * u) * (1.0 + 1e-3));
  cam.t_a = (float)(ta * (1.0 + 1e-3));
  cam.t_s = (float)(B * d * (1.0 + 1e-3));
}

}  // namespace perch

// A box inside the volume V(O) = {o : n_f . o <= w_f for every face f}: the vertex
// box's z range (less a margin) with its x/y half-extents scaled about the centre as
// far as every plane allows, or, when that leaves less than a quarter, the whole
// vertex box scaled uniformly.  Computed in FP64 on the planes' float32 values with
// its corners rounded inward to float32, and checked corner by corner: every point
// of it lies at least 1e-9 m inside every plane.  Empty (min > max) when there is no
// such box (a mesh whose planes do not enclose its vertex-box centre).
static void inner_box(const std::vector<float>& planes, const float lo[3], const float hi[3],
                      float a[3], float b[3]) {
  const double m = 1e-9;
  const int nf = (int)planes.size() / 4;
  double c[3], h[3];
  for (int k = 0; k < 3; ++k) {
    c[k] = 0.5 * ((double)lo[k] + (double)hi[k]);
    h[k] = 0.5 * ((double)hi[k] - (double)lo[k]);
  }
  for (int k = 0; k < 3; ++k) {  // empty
    a[k] = 1.0f;
    b[k] = -1.0f;
  }
  if (nf == 0) return;
  auto slack = [&](int f) {  // w - m - n . c
    const float* p = &planes[4 * (size_t)f];
    return (double)p[3] - m - ((double)p[0] * c[0] + (double)p[1] * c[1] + (double)p[2] * c[2]);
  };
  // (a) x/y scaled by la, z half-extent shrunk by 2 m
  const double hz = std::max(0.0, h[2] - 2.0 * m);
  double la = 1.0;
  for (int f = 0; f < nf && la >= 0.0; ++f) {
    const float* p = &planes[4 * (size_t)f];
    const double rest = slack(f) - std::fabs((double)p[2]) * hz;
    const double den = std::fabs((double)p[0]) * h[0] + std::fabs((double)p[1]) * h[1];
    if (den > 0.0) la = std::min(la, rest / den);
    else if (rest < 0.0) la = -1.0;
  }
  double e[3] = {la * h[0], la * h[1], hz};
  if (!(la >= 0.25)) {  // (b) uniform scaling
    double lb = 1.0;
    for (int f = 0; f < nf; ++f) {
      const float* p = &planes[4 * (size_t)f];
      const double den = std::fabs((double)p[0]) * h[0] + std::fabs((double)p[1]) * h[1] +
                         std::fabs((double)p[2]) * h[2];
      if (den > 0.0) lb = std::min(lb, slack(f) / den);
      else if (slack(f) < 0.0) lb = -1.0;
    }
    if (!(lb > 0.0)) return;
    for (int k = 0; k < 3; ++k) e[k] = lb * h[k];
  }
  float ra[3], rb[3];
  for (int k = 0; k < 3; ++k) {
    ra[k] = (float)(c[k] - e[k]);
    if ((double)ra[k] < c[k] - e[k]) ra[k] = std::nextafter(ra[k], INFINITY);
    rb[k] = (float)(c[k] + e[k]);
    if ((double)rb[k] > c[k] + e[k]) rb[k] = std::nextafter(rb[k], -INFINITY);
    if (!(ra[k] <= rb[k])) return;
  }
  for (int f = 0; f < nf; ++f) {  // the rounded corners, checked
    const float* p = &planes[4 * (size_t)f];
    double v = -(double)p[3];
    for (int k = 0; k < 3; ++k) v += (double)p[k] * (p[k] > 0.0f ? (double)rb[k] : (double)ra[k]);
    if (!(v <= -0.5 * m)) return;
  }
  for (int k = 0; k < 3; ++k) {
    a[k] = ra[k];
    b[k] = rb[k];
  }
}

// The volume test's boxes of one mesh (the layout of Meshes::aabb): the vertex box's
// centre (float32), its half-extents rounded up so that centre +- them holds
// [lo, hi], and the inner box's half-extents about that centre rounded down (-1 when
// the inner box is empty).
static void volume_boxes(const std::vector<float>& planes, const float lo[3], const float hi[3],
                         std::vector<float4>& out) {
  float a[3], b[3];
  inner_box(planes, lo, hi, a, b);
  float ctr[3], ho[3], hi_[3];
  for (int k = 0; k < 3; ++k) {
    ctr[k] = (float)(0.5 * ((double)lo[k] + (double)hi[k]));
    const double o = std::max((double)hi[k] - ctr[k], (double)ctr[k] - lo[k]);
    ho[k] = (float)o;
    if ((double)ho[k] < o) ho[k] = std::nextafter(ho[k], INFINITY);
    const double in = std::min((double)b[k] - ctr[k], (double)ctr[k] - a[k]);
    hi_[k] = (float)in;
    if ((double)hi_[k] > in) hi_[k] = std::nextafter(hi_[k], -INFINITY);
  }
  const bool empty = !(hi_[0] > 0.0f && hi_[1] > 0.0f && hi_[2] > 0.0f);
  out.push_back(make_float4(ctr[0], ctr[1], ctr[2], 0.0f));
  out.push_back(make_float4(ho[0], ho[1], ho[2], 0.0f));
  out.push_back(empty ? make_float4(-1.0f, -1.0f, -1.0f, 0.0f)
                      : make_float4(hi_[0], hi_[1], hi_[2], 0.0f));
  out.push_back(make_float4(0.0f, 0.0f, 0.0f, 0.0f));
}

perch_status upload_meshes(perch_ctx* c) {
  if (!c->meshes_dirty) return PERCH_OK;
  const int nm = (int)c->meshes.size();
  if (nm == 0) return fail(PERCH_E_STATE, "no meshes added");
  std::vector<float4> v;
  std::vector<int4> t, rg;
  std::vector<float4> pl, bb;
  std::vector<int2> fr;
  int max_nv = 0;
  float rmax = 0.0f, wmax = 0.0f;
  for (int m = 0; m < nm; ++m) {
    const HostMesh& h = c->meshes[m];
    if (!h.set) return fail(PERCH_E_STATE, "mesh id %d was never added (ids must be dense)", m);
    const int nv = (int)h.verts.size() / 3, nt = (int)h.tris.size() / 3,
              nf = (int)h.planes.size() / 4;
    rg.push_back(make_int4((int)v.size(), nv, (int)t.size(), nt));
    fr.push_back(make_int2((int)pl.size(), nf));
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < nv; ++k) {
      float x = h.verts[3 * k], y = h.verts[3 * k + 1], z = h.verts[3 * k + 2];
      v.push_back(make_float4(x, y, z, 0.0f));
      lo[0] = std::min(lo[0], x); lo[1] = std::min(lo[1], y); lo[2] = std::min(lo[2], z);
      hi[0] = std::max(hi[0], x); hi[1] = std::max(hi[1], y); hi[2] = std::max(hi[2], z);
    }
    for (int k = 0; k < nt; ++k)
      t.push_back(make_int4(h.tris[3 * k], h.tris[3 * k + 1], h.tris[3 * k + 2], 0));
    for (int k = 0; k < nf; ++k)
      pl.push_back(make_float4(h.planes[4 * k], h.planes[4 * k + 1], h.planes[4 * k + 2],
                               h.planes[4 * k + 3]));
    volume_boxes(h.planes, lo, hi, bb);
    max_nv = std::max(max_nv, nv);
    if (nv > 0) {
      const float cx = std::max(std::fabs(lo[0]), std::fabs(hi[0]));
      const float cy = std::max(std::fabs(lo[1]), std::fabs(hi[1]));
      const float cz = std::max(std::fabs(lo[2]), std::fabs(hi[2]));
      rmax = std::max(rmax, std::sqrt(cx * cx + cy * cy + cz * cz));
    }
    for (int k = 0; k < nf; ++k) wmax = std::max(wmax, std::fabs(h.planes[4 * k + 3]));
  }
  HIP_TRY(c->verts.ensure(v.size() * sizeof(float4)));
  HIP_TRY(c->tris.ensure(std::max<size_t>(1, t.size()) * sizeof(int4)));
  HIP_TRY(c->planes.ensure(std::max<size_t>(1, pl.size()) * sizeof(float4)));
  HIP_TRY(c->range.ensure(rg.size() * sizeof(int4)));
  HIP_TRY(c->frange.ensure(fr.size() * sizeof(int2)));
  HIP_TRY(c->aabb.ensure(bb.size() * sizeof(float4)));
  HIP_TRY(hipMemcpy(c->verts.p, v.data(), v.size() * sizeof(float4), hipMemcpyHostToDevice));
  if (!t.empty())
    HIP_TRY(hipMemcpy(c->tris.p, t.data(), t.size() * sizeof(int4), hipMemcpyHostToDevice));
  if (!pl.empty())
    HIP_TRY(hipMemcpy(c->planes.p, pl.data(), pl.size() * sizeof(float4), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->range.p, rg.data(), rg.size() * sizeof(int4), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->frange.p, fr.data(), fr.size() * sizeof(int2), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->aabb.p, bb.data(), bb.size() * sizeof(float4), hipMemcpyHostToDevice));
  c->max_nv = max_nv;
  c->mesh_rmax = rmax * (1.0f + 1e-6f);
  c->mesh_wmax = wmax * (1.0f + 1e-6f);
  c->meshes_dirty = false;
  return PERCH_OK;
}

// vertex cache + z-tile + one 128-entry triangle ring per wave

static bool objects_ok(const perch_ctx* c, const perch_object* o, int n) {
  for (int k = 0; k < n; ++k)
    if (o[k].mesh_id < 0 || o[k].mesh_id >= (int)c->meshes.size() || o[k].pose_idx < 0 ||
        o[k].pose_idx >= c->n_poses())
      return false;
  return true;
}

// Composite R_j of parent[0..j) into depth (float bits, +inf = empty); at the goal
// level also the set U (bitmap + count) of observed points outside every parent
// volume and unexplained by R_j.
perch_status materialise_into(perch_ctx* c, const perch_object* parent, int j, bool goal,
                              unsigned* depth, unsigned* ubits, int* ucount, hipStream_t st) {
  const size_t npx = (size_t)c->cam.W * c->cam.H;
  const Meshes M = c->dev_meshes();
  const float4* poses = c->poses.as<float4>();
  launch_fill_u32(depth, kInfBits, npx, st);
  int mp[2 * kMaxObjects];
  int max_tris = 0;
  for (int k = 0; k < j; ++k) {
    mp[2 * k] = parent[k].mesh_id;
    mp[2 * k + 1] = parent[k].pose_idx;
    max_tris = std::max(max_tris, (int)c->meshes[parent[k].mesh_id].tris.size() / 3);
  }
  launch_render_objects(c->cam, M, poses, mp, j, max_tris, depth, st);
  if (goal) {
    launch_fill_u32(ubits, 0u, (npx + 31) / 32, st);
    launch_fill_i32(ucount, 0, 1, st);
    launch_parent_u(c->cam, M, poses, c->obs.as<float>(), mp, j, depth, ubits, ucount,
                    c->eval_params(), st);
  }
  HIP_TRY(hipGetLastError());
  return PERCH_OK;
}

static perch_status materialise_parent(perch_ctx* c, const perch_object* parent, int j,
                                       bool goal) {
  const size_t npx = (size_t)c->cam.W * c->cam.H;
  HIP_TRY(c->par_depth.ensure(npx * sizeof(unsigned)));
  HIP_TRY(c->par_ubits.ensure(((npx + 31) / 32) * sizeof(unsigned)));
  HIP_TRY(c->par_ucount.ensure(sizeof(int)));
  return materialise_into(c, parent, j, goal, c->par_depth.as<unsigned>(),
                          c->par_ubits.as<unsigned>(), c->par_ucount.as<int>(), c->stream);
}

extern "C" {

const char* perch_last_error(void) { return perch::g_err.c_str(); }

perch_status perch_create(const perch_sensor* s, void* hip_stream, perch_ctx** out) {
  if (!s || !out) return fail(PERCH_E_ARG, "null argument");
  *out = nullptr;
  if (s->width <= 0 || s->height <= 0 || s->width > 16384 || s->height > 16384)
    return fail(PERCH_E_ARG, "bad image size %dx%d", s->width, s->height);
  if (!(s->fx > 0) || !(s->fy > 0) || !(s->delta >= 0))
    return fail(PERCH_E_ARG, "bad intrinsics or delta");
  double R[9], t[3];
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) R[3 * r + k] = s->cam_from_world[4 * r + k];
    t[r] = s->cam_from_world[4 * r + 3];
  }
  const double A = R[4] * R[8] - R[5] * R[7], B = -(R[3] * R[8] - R[5] * R[6]),
               C = R[3] * R[7] - R[4] * R[6];
  const double det = R[0] * A + R[1] * B + R[2] * C;
  if (!(std::fabs(det) > 1e-12)) return fail(PERCH_E_ARG, "singular camera rotation");
  double Ri[9] = {A / det,
                  -(R[1] * R[8] - R[2] * R[7]) / det,
                  (R[1] * R[5] - R[2] * R[4]) / det,
                  B / det,
                  (R[0] * R[8] - R[2] * R[6]) / det,
                  -(R[0] * R[5] - R[2] * R[3]) / det,
                  C / det,
                  -(R[0] * R[7] - R[1] * R[6]) / det,
                  (R[0] * R[4] - R[1] * R[3]) / det};
  perch_ctx* c = new perch_ctx();
  Cam& cam = c->cam;
  cam.W = s->width;
  cam.H = s->height;
  cam.fx = s->fx;
  cam.fy = s->fy;
  cam.cx = s->cx;
  cam.cy = s->cy;
  for (int k = 0; k < 12; ++k) {
    cam.M[k] = s->cam_from_world[k];
    cam.dM[k] = s->cam_from_world[k];
  }
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) cam.Winv[4 * r + k] = (float)Ri[3 * r + k];
    cam.Winv[4 * r + 3] = (float)(-(Ri[3 * r] * t[0] + Ri[3 * r + 1] * t[1] + Ri[3 * r + 2] * t[2]));
  }
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) cam.dWinv[4 * r + k] = Ri[3 * r + k];
    cam.dWinv[4 * r + 3] = -(Ri[3 * r] * t[0] + Ri[3 * r + 1] * t[1] + Ri[3 * r + 2] * t[2]);
  }
  cam.delta = s->delta;
  cam.delta2 = s->delta * s->delta;
  cam.ddelta2 = (double)s->delta * (double)s->delta;
  cam.inv_fx = 1.0f / s->fx;
  cam.inv_fy = 1.0f / s->fy;
  cam.dfx = s->fx;
  cam.dfy = s->fy;
  cam.dcx = s->cx;
  cam.dcy = s->cy;
  cam.dinv_fx = 1.0 / (double)s->fx;
  cam.dinv_fy = 1.0 / (double)s->fy;
  delta_margins(cam);
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(PERCH_E_HIP, "hipGetDevice failed");
  }
  *out = c;
  return PERCH_OK;
}

void perch_destroy(perch_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (DevBuf* b : {&c->verts, &c->tris, &c->planes, &c->range, &c->frange, &c->aabb, &c->poses,
                    &c->obs, &c->obs_range, &c->h_keys, &c->h_cells, &c->h_pts, &c->h_counts, &c->par_depth,
                    &c->par_ubits, &c->par_ucount, &c->par_vbits, &c->s_cands, &c->s_out,
                    &c->s_adj, &c->icp_pn, &c->cnn_desc})
    b->release();
  for (DevBuf& b : c->learned_bufs) b.release();
  if (c->s_batch) perch_batch_destroy(c->s_batch);
  for (DevBuf* b : {&c->s_items, &c->s_bout, &c->s_bcrops, &c->s_bpairs, &c->s_bpred,
                    &c->s_bcands})
    b->release();
  c->s_hitems.release();
  c->s_hbout.release();
  c->s_hcands.release();
  c->s_hout.release();
  c->s_hposes.release();
  delete c;
}

// Back-projects the observation, derives the pixel-window halo and builds the
// voxel hash of I from c->obs (synchronous).
static perch_status build_observation(perch_ctx* c) {
  const Cam& cam = c->cam;
  const size_t npx = (size_t)cam.W * cam.H;
  std::vector<float> host(npx);
  HIP_TRY(hipMemcpyAsync(host.data(), c->obs.p, npx * sizeof(float), hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  int n = 0;
  float zmin = INFINITY, zmax = 0.0f;
  for (size_t k = 0; k < npx; ++k)
    if (host[k] > 0.0f) {
      ++n;
      zmin = std::min(zmin, host[k]);
      zmax = std::max(zmax, host[k]);
    }
  if (!(zmax < INFINITY)) return fail(PERCH_E_ARG, "observed depth is not finite");
  c->obs_zmax = zmax;
  // Pixel halo: the largest window radius fx dwin sqrt(1 + a^2) / (Z - dwin) + 1
  // over the observed points (a = |u - cx| / fx at the image border, Z >= zmin).
  const double dwin = (double)cam.delta * 1.001 + 1e-6;
  int halo = 1;
  if (n > 0) {
    if (!(zmin > dwin)) return fail(PERCH_E_UNSUPPORTED, "observed depth within delta of camera");
    const double amax = std::max(std::fabs(0.0 - cam.cx), std::fabs(cam.W - 1.0 - cam.cx)) / cam.fx;
    const double bmax = std::max(std::fabs(0.0 - cam.cy), std::fabs(cam.H - 1.0 - cam.cy)) / cam.fy;
    const double ru = cam.fx * dwin * std::sqrt(1 + amax * amax) / (zmin - dwin);
    const double rv = cam.fy * dwin * std::sqrt(1 + bmax * bmax) / (zmin - dwin);
    halo = (int)std::floor(std::max(ru, rv)) + 2;
  }
  c->ep.halo = halo;
  c->ep.dwin = (float)dwin;
  c->n_points = n;
  HIP_TRY(c->obs_range.ensure(npx * sizeof(float2)));
  launch_obs_range(cam, c->obs.as<float>(), c->obs_range.as<float2>(), halo, c->stream);
  // voxel hash of I
  const int slots = next_pow2(std::max(64, 2 * n));
  c->h_mask = slots - 1;
  HIP_TRY(c->h_keys.ensure((size_t)slots * sizeof(unsigned long long)));
  HIP_TRY(c->h_cells.ensure((size_t)slots * sizeof(int2)));
  HIP_TRY(c->h_counts.ensure((size_t)(2 * slots + 1) * sizeof(int)));
  HIP_TRY(c->h_pts.ensure((size_t)std::max(1, n) * sizeof(float4)));
  int* counts = c->h_counts.as<int>();
  int* fill = counts + slots;
  int* npts = counts + 2 * slots;
  launch_fill_u32(reinterpret_cast<unsigned*>(c->h_keys.p), 0xffffffffu, 2 * (size_t)slots,
                  c->stream);
  launch_fill_i32(counts, 0, 2 * (size_t)slots + 1, c->stream);
  const Hash h = c->dev_hash();
  launch_hash_insert(cam, c->obs.as<float>(), c->h_keys.as<unsigned long long>(), counts, c->h_mask,
                     h.inv_cell, npts, c->stream);
  launch_scan_cells(counts, c->h_cells.as<int2>(), slots, c->stream);
  launch_hash_scatter(cam, c->obs.as<float>(), c->h_keys.as<unsigned long long>(),
                      c->h_cells.as<int2>(), fill, c->h_pts.as<float4>(), c->h_mask, h.inv_cell,
                      c->stream);
  HIP_TRY(hipGetLastError());
  int dev_n = 0;
  HIP_TRY(hipMemcpyAsync(&dev_n, npts, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (dev_n != n) return fail(PERCH_E_HIP, "hash build counted %d points, expected %d", dev_n, n);
  c->has_obs = true;
  ++c->obs_serial;
  return PERCH_OK;
}

perch_status perch_set_observation(perch_ctx* c, const float* depth_dev) {
  if (!c || !depth_dev) return fail(PERCH_E_ARG, "null argument");
  const size_t npx = (size_t)c->cam.W * c->cam.H;
  c->has_obs = false;
  c->parent_j = -1;
  HIP_TRY(c->obs.ensure(npx * sizeof(float)));
  HIP_TRY(hipMemcpyAsync(c->obs.p, depth_dev, npx * sizeof(float), hipMemcpyDeviceToDevice,
                         c->stream));
  return build_observation(c);
}

perch_status perch_add_mesh(perch_ctx* c, int32_t mesh_id, const float* verts, int32_t nv,
                            const int32_t* tris, int32_t nt, const float* planes, int32_t nf) {
  if (!c || !verts || !tris || (!planes && nf > 0)) return fail(PERCH_E_ARG, "null argument");
  if (mesh_id < 0 || mesh_id > 4096 || nv < 3 || nt < 1 || nf < 0)
    return fail(PERCH_E_ARG, "bad mesh sizes");
  for (int k = 0; k < 3 * nt; ++k)
    if (tris[k] < 0 || tris[k] >= nv) return fail(PERCH_E_ARG, "triangle index out of range");
  if ((int)c->meshes.size() <= mesh_id) c->meshes.resize(mesh_id + 1);
  HostMesh& h = c->meshes[mesh_id];
  h.verts.assign(verts, verts + 3 * (size_t)nv);
  h.tris.assign(tris, tris + 3 * (size_t)nt);
  h.planes.assign(planes, planes + 4 * (size_t)nf);
  h.set = true;
  c->meshes_dirty = true;
  return PERCH_OK;
}

perch_status perch_set_symmetric(perch_ctx* c, int32_t mesh_id, int32_t symmetric) {
  if (!c) return fail(PERCH_E_ARG, "null context");
  if (mesh_id < 0 || mesh_id >= (int)c->meshes.size() || !c->meshes[mesh_id].set)
    return fail(PERCH_E_ARG, "mesh %d not added", mesh_id);
  if ((int)c->symmetric.size() <= mesh_id) c->symmetric.resize(mesh_id + 1, 0);
  c->symmetric[mesh_id] = symmetric ? 1 : 0;
  return PERCH_OK;
}

perch_status perch_set_poses(perch_ctx* c, const float* poses, int32_t P) {
  if (!c || !poses || P <= 0) return fail(PERCH_E_ARG, "bad pose table");
  float xy = 0.0f;
  for (int k = 0; k < P; ++k) {
    const float e = std::fabs(poses[4 * k]) + std::fabs(poses[4 * k + 1]);
    if (!(e < 1e4f)) return fail(PERCH_E_ARG, "pose %d is not finite or beyond 1e4 m", k);
    xy = std::max(xy, e);
  }
  HIP_TRY(c->poses.ensure(((size_t)P + c->arena_cap) * sizeof(float4)));
  HIP_TRY(hipMemcpy(c->poses.p, poses, (size_t)P * sizeof(float4), hipMemcpyHostToDevice));
  c->pose_xy_max = xy;
  c->P = P;
  c->arena_used = 0;
  c->h_poses.assign(poses, poses + 4 * (size_t)P);
  c->parent_j = -1;
  return PERCH_OK;
}

perch_status perch_set_pose_arena(perch_ctx* c, int32_t capacity) {
  if (!c || capacity < 0) return fail(PERCH_E_ARG, "bad arena capacity");
  if (c->P <= 0) return fail(PERCH_E_STATE, "perch_set_poses not called");
  if ((int64_t)c->P + capacity > INT32_MAX) return fail(PERCH_E_ARG, "arena too large");
  HIP_TRY(hipStreamSynchronize(c->stream));
  const size_t need = ((size_t)c->P + capacity) * sizeof(float4);
  if (need > c->poses.bytes) {
    HIP_TRY(c->poses.ensure(need));
    HIP_TRY(hipMemcpy(c->poses.p, c->h_poses.data(), (size_t)c->P * sizeof(float4),
                      hipMemcpyHostToDevice));
  }
  c->arena_cap = capacity;
  c->arena_used = 0;
  c->parent_j = -1;  // a materialised parent may use arena poses
  return PERCH_OK;
}

perch_status perch_get_poses(perch_ctx* c, int32_t first, int32_t n, float* poses_host) {
  if (!c || first < 0 || n < 0 || (n > 0 && !poses_host)) return fail(PERCH_E_ARG, "bad range");
  if ((int64_t)first + n > c->n_poses()) return fail(PERCH_E_ARG, "poses out of range");
  if (n == 0) return PERCH_OK;
  HIP_TRY(hipMemcpyAsync(poses_host, c->poses.as<float4>() + first, (size_t)n * sizeof(float4),
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return PERCH_OK;
}

perch_status perch_set_objects(perch_ctx* c, const int32_t* mesh_ids, int32_t K) {
  if (!c || (!mesh_ids && K > 0) || K < 1 || K > PERCH_MAX_OBJECTS)
    return fail(PERCH_E_ARG, "bad object list");
  c->objects.assign(mesh_ids, mesh_ids + K);
  c->parent_j = -1;
  return PERCH_OK;
}

perch_status perch_set_tuning(perch_ctx* c, int32_t threads, int32_t tile_px,
                              float cell_over_delta, int32_t radius_mode) {
  if (!c) return fail(PERCH_E_ARG, "null context");
  if (radius_mode < -1 || radius_mode > 1) return fail(PERCH_E_ARG, "radius_mode must be -1, 0 or 1");
  if (threads && threads != 64 && threads != 128 && threads != 256 && threads != 512 &&
      threads != 1024)
    return fail(PERCH_E_ARG, "threads must be 64, 128, 256, 512 or 1024");
  if (tile_px && tile_px != -1 && (tile_px < 256 || tile_px > 36864))
    return fail(PERCH_E_ARG, "bad tile_px");
  if (cell_over_delta != 0.0f && !(cell_over_delta >= 1.0f && cell_over_delta <= 8.0f))
    return fail(PERCH_E_ARG, "cell_over_delta must be in [1, 8]");
  // every argument is checked before any is applied
  if (radius_mode >= 0) c->radius_mode = radius_mode;
  if (threads) {
    c->threads = threads;
    c->threads_auto = false;
  }
  if (tile_px) c->tile_px = tile_px < 0 ? 0 : tile_px;
  if (cell_over_delta != 0.0f && cell_over_delta != c->cell_over_delta) {
    c->cell_over_delta = cell_over_delta;
    if (c->has_obs) {
      perch_status st = build_observation(c);  // rebuild the hash with the new cell size
      if (st) return st;
    }
  }
  return PERCH_OK;
}

perch_status perch_get_info(perch_ctx* c, int32_t* n_points, int32_t* halo) {
  if (!c) return fail(PERCH_E_ARG, "null context");
  if (n_points) *n_points = c->n_points;
  if (halo) *halo = c->ep.halo;
  return PERCH_OK;
}

perch_status perch_set_parent(perch_ctx* c, const perch_object* parent, int32_t j) {
  if (!c) return fail(PERCH_E_ARG, "null context");
  c->parent_j = -1;
  if (!c->has_obs) return fail(PERCH_E_STATE, "perch_set_observation not called");
  if (c->P <= 0) return fail(PERCH_E_STATE, "perch_set_poses not called");
  const int K = (int)c->objects.size();
  if (K < 1) return fail(PERCH_E_STATE, "perch_set_objects not called");
  if (j < 0 || j >= K || (j > 0 && !parent)) return fail(PERCH_E_ARG, "bad parent (j=%d, K=%d)", j, K);
  perch_status st = upload_meshes(c);
  if (st) return st;
  if (!objects_ok(c, parent, j)) return fail(PERCH_E_ARG, "parent object out of range");
  roctxRangePushA("perch_set_parent");
  st = materialise_parent(c, parent, j, j + 1 == K);
  roctxRangePop();
  if (st) return st;
  c->parent_objs.assign(parent, parent + j);
  ++c->parent_serial;
  c->parent_j = j;
  return PERCH_OK;
}

// Successor launch over the materialised parent; gain_dev != null also counts, per
// successor, the observed points its volume adds to V_j.
static perch_status eval_children_impl(perch_ctx* c, const perch_object* cands_dev, int32_t n,
                                       int32_t* cost_dev, int32_t* status_dev,
                                       int32_t* comps_dev, int32_t* gain_dev) {
  if (!c) return fail(PERCH_E_ARG, "null context");
  if (n < 0 || (n > 0 && (!cands_dev || !cost_dev || !status_dev)))
    return fail(PERCH_E_ARG, "bad successor arrays");
  if (c->parent_j < 0) return fail(PERCH_E_STATE, "perch_set_parent not called");
  if (c->meshes_dirty) return fail(PERCH_E_STATE, "meshes changed since perch_set_parent");
  if (c->n_cus == 0) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&c->n_cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  const int nt = c->launch_threads(n);
  const int tile = c->tile_for(nt);
  const size_t lds = eval_lds_bytes(c->max_nv, tile, nt);
  if (lds > 160 * 1024 - 256)
    return fail(PERCH_E_UNSUPPORTED, "LDS need %zu B exceeds the CU (max_nv=%d, tile=%d)", lds,
                c->max_nv, tile);
  if (n == 0) return PERCH_OK;
  const int K = (int)c->objects.size();
  Parent par;
  par.depth = c->par_depth.as<unsigned>();
  par.ubits = c->par_ubits.as<unsigned>();
  par.ucount = c->par_ucount.as<int>();
  par.vbits = nullptr;
  par.has_parent = c->parent_j > 0;
  par.goal = (c->parent_j + 1 == K);
  if (gain_dev) {
    if (c->vbits_for != c->parent_serial) {
      const size_t npx = (size_t)c->cam.W * c->cam.H;
      HIP_TRY(c->par_vbits.ensure(((npx + 31) / 32) * sizeof(unsigned)));
      int mp[2 * kMaxObjects];
      const int j = c->parent_j;
      for (int k = 0; k < j; ++k) {
        mp[2 * k] = c->parent_objs[k].mesh_id;
        mp[2 * k + 1] = c->parent_objs[k].pose_idx;
      }
      launch_parent_v(c->cam, c->dev_meshes(), c->poses.as<float4>(), c->obs.as<float>(), mp, j,
                      c->par_vbits.as<unsigned>(), c->eval_params(), c->stream);
      HIP_TRY(hipGetLastError());
      c->vbits_for = c->parent_serial;
    }
    par.vbits = c->par_vbits.as<unsigned>();
  }
  perch::SceneDev S = c->scene_dev();
  S.ep.tile_px = tile;
  HIP_TRY(launch_eval(nt, S, par, reinterpret_cast<const int2*>(cands_dev), n, cost_dev,
                      status_dev, comps_dev, gain_dev, lds, c->stream));
  return PERCH_OK;
}

perch_status perch_eval_children(perch_ctx* c, const perch_object* cands_dev, int32_t n,
                                 int32_t* cost_dev, int32_t* status_dev, int32_t* comps_dev) {
  roctxRangePushA("perch_eval_children");
  const perch_status st = eval_children_impl(c, cands_dev, n, cost_dev, status_dev, comps_dev,
                                             nullptr);
  roctxRangePop();
  return st;
}

perch_status perch_overlap_gain(perch_ctx* c, const perch_object* cands_dev, int32_t n,
                                int32_t* cost_dev, int32_t* status_dev, int32_t* gain_dev) {
  if (n > 0 && !gain_dev) return fail(PERCH_E_ARG, "null gain array");
  return eval_children_impl(c, cands_dev, n, cost_dev, status_dev, nullptr, gain_dev);
}

perch_status perch_icp_children(perch_ctx* c, const perch_object* cands_dev, int32_t n,
                                int32_t iters, float radius, perch_object* adjusted_dev,
                                int32_t* n_match_dev, int32_t* status_dev) {
  if (!c) return fail(PERCH_E_ARG, "null context");
  if (n < 0 || (n > 0 && (!cands_dev || !adjusted_dev || !n_match_dev || !status_dev)))
    return fail(PERCH_E_ARG, "bad candidate arrays");
  if (iters < 0 || iters > 1000 || !(radius > 0.0f) || !(radius < 1.0f))
    return fail(PERCH_E_ARG, "bad ICP iterations or radius");
  if (c->parent_j < 0) return fail(PERCH_E_STATE, "perch_set_parent not called");
  if (c->meshes_dirty) return fail(PERCH_E_STATE, "meshes changed since perch_set_parent");
  const int tile = icp_tile_px(c->max_nv);
  if (tile <= 0) return fail(PERCH_E_UNSUPPORTED, "no LDS left for the ICP tile");
  if ((int64_t)c->arena_used + n > c->arena_cap)
    return fail(PERCH_E_ARG, "pose arena full (%d of %d used, %d more asked)", c->arena_used,
                c->arena_cap, n);
  if (n == 0) return PERCH_OK;
  const size_t npx = (size_t)c->cam.W * c->cam.H;
  if (c->icp_pn_obs != c->obs_serial || c->icp_pn_radius != radius) {
    HIP_TRY(c->icp_pn.ensure(2 * npx * sizeof(double4)));
    launch_obs_normals(c->cam, c->obs.as<float>(), radius, c->icp_pn.as<double4>(), c->stream);
    HIP_TRY(hipGetLastError());
    c->icp_pn_obs = c->obs_serial;
    c->icp_pn_radius = radius;
  }
  const int K = (int)c->objects.size();
  Parent par;
  par.depth = c->par_depth.as<unsigned>();
  par.ubits = c->par_ubits.as<unsigned>();
  par.ucount = c->par_ucount.as<int>();
  par.vbits = nullptr;
  par.has_parent = c->parent_j > 0;
  par.goal = (c->parent_j + 1 == K);
  perch::SceneDev S = c->scene_dev();
  IcpArgs ia;
  ia.iters = iters;
  ia.radius = radius;
  ia.pn = c->icp_pn.as<double4>();
  ia.base = c->P + c->arena_used;
  ia.arena = c->poses.as<float4>() + ia.base;
  ia.retry = 0;
  const bool vc = icp_vertex_cache(c->max_nv);
  // a first pass whose tile lets two workgroups share a CU; the footprints it cannot
  // hold (status -3) go through a second pass with the largest tile
  const int tile2 = icp_tile_px(c->max_nv, 2);
  const bool two_pass = tile2 >= 4096 && tile2 < tile;
  S.ep.tile_px = two_pass ? tile2 : tile;
  HIP_TRY(launch_icp(S, par, reinterpret_cast<const int2*>(cands_dev), n, ia,
                     reinterpret_cast<int2*>(adjusted_dev), n_match_dev, status_dev, vc,
                     icp_fixed_lds(c->max_nv) + (size_t)S.ep.tile_px * sizeof(unsigned),
                     c->stream));
  if (two_pass) {
    ia.retry = 1;
    S.ep.tile_px = tile;
    HIP_TRY(launch_icp(S, par, reinterpret_cast<const int2*>(cands_dev), n, ia,
                       reinterpret_cast<int2*>(adjusted_dev), n_match_dev, status_dev, vc,
                       icp_fixed_lds(c->max_nv) + (size_t)tile * sizeof(unsigned), c->stream));
  }
  c->arena_used += n;
  return PERCH_OK;
}

perch_status perch_eval_successors(perch_ctx* c, const perch_object* parent, int32_t j,
                                   const perch_object* cands_dev, int32_t n, int32_t* cost_dev,
                                   int32_t* status_dev, int32_t* comps_dev) {
  if (!c) return fail(PERCH_E_ARG, "null context");
  if (n < 0 || (n > 0 && (!cands_dev || !cost_dev || !status_dev)))
    return fail(PERCH_E_ARG, "bad successor arrays");
  perch_status st = perch_set_parent(c, parent, j);
  if (st) return st;
  return perch_eval_children(c, cands_dev, n, cost_dev, status_dev, comps_dev);
}

perch_status perch_render(perch_ctx* c, const perch_object* objs, int32_t n, int32_t composite,
                          float* depth_dev) {
  if (!c || (n > 0 && (!objs || !depth_dev)) || n < 0) return fail(PERCH_E_ARG, "bad arguments");
  if (c->P <= 0) return fail(PERCH_E_STATE, "perch_set_poses not called");
  perch_status st = upload_meshes(c);
  if (st) return st;
  if (!objects_ok(c, objs, n)) return fail(PERCH_E_ARG, "object out of range");
  const size_t npx = (size_t)c->cam.W * c->cam.H;
  unsigned* out = reinterpret_cast<unsigned*>(depth_dev);
  const Meshes M = c->dev_meshes();
  if (composite) {
    launch_fill_u32(out, kInfBits, npx, c->stream);
    for (int k0 = 0; k0 < n; k0 += kMaxObjects) {  // up to kMaxObjects objects per launch
      const int m = std::min(kMaxObjects, n - k0);
      int mp[2 * kMaxObjects];
      int max_tris = 0;
      for (int k = 0; k < m; ++k) {
        mp[2 * k] = objs[k0 + k].mesh_id;
        mp[2 * k + 1] = objs[k0 + k].pose_idx;
        max_tris = std::max(max_tris, (int)c->meshes[objs[k0 + k].mesh_id].tris.size() / 3);
      }
      launch_render_objects(c->cam, M, c->poses.as<float4>(), mp, m, max_tris, out, c->stream);
    }
  } else {
    launch_fill_u32(out, kInfBits, npx * (size_t)n, c->stream);
    for (int k = 0; k < n; ++k)
      launch_render_object(c->cam, M, c->poses.as<float4>(), objs[k].mesh_id, objs[k].pose_idx,
                           (int)c->meshes[objs[k].mesh_id].tris.size() / 3, out + npx * k,
                           c->stream);
  }
  HIP_TRY(hipGetLastError());
  return PERCH_OK;
}

}  // extern "C"
