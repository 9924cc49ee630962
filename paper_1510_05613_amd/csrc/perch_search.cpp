// perch_search.cpp -- tree search over the Monotone Scene Generation Tree
// (arXiv:1510.05613 Sec. IV-A/B, Alg. 1 ComputePath) on GPU-evaluated successors.
//
// A state is a set of placed objects (Eq. 3); its children add any not-yet-placed
// object of the known multiset at any pose of the grid, and each child costs
// c(s, s') (Eq. 4).  Every expansion materialises the parent on the GPU and
// evaluates all of its children in one launch; the host keeps the open list.
//   - exhaustive: depth-first enumeration of the whole tree; argmin (cost, key)
//     over goals (the literal optimum of Theorem 2 with w = 1);
//   - uniform-cost: best-first on (g, -|s|, key), states deduplicated by their
//     canonical key (the paper keeps one insertion order per configuration,
//     Sec. IV-A); the first goal popped is optimal because edge costs are >= 0;
//   - focal: anchor queue ordered by g (admissible h = 0, Sec. IV-C) and an
//     inadmissible queue preferring deeper states (h_depth = K - |s|, Sec. IV-C)
//     restricted to FOCAL = {g <= w * min g}; a goal chosen from FOCAL costs at
//     most w * OPT (Theorem 2).  With anytime = 1 the search continues, keeping the
//     best goal, until the incumbent is no worse than the anchor's min g;
//   - multi-heuristic (Focal-MHA*, Sec. IV-C): the anchor and two inadmissible
//     queues restricted to FOCAL, h_depth and h_overlap = |I| - #{p in I : p in V_j}
//     (kept per state from the per-child decrease the successor kernel counts),
//     expanded round robin; same bound and anytime rule as focal;
//   - learned: the focal scheme with a learned network ranking the children of an
//     expanded state: only the top-k predicted children are evaluated exactly and
//     enter the inadmissible queue; the remaining children wait as one lazy block
//     keyed at g(parent) (a lower bound, edge costs being >= 0) in the anchor queue
//     and are evaluated when the anchor reaches them, so completeness and the
//     w-bound are those of the focal search; the learned multi-heuristic variant
//     adds h_overlap as a second inadmissible queue over the evaluated children.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <queue>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <unordered_map>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "perch_cnn.h"
#include "perch_ctx.h"

using namespace perch;

namespace {

using Clock = std::chrono::steady_clock;

struct Node {
  int64_t g;
  int32_t j;
  int32_t parent;  // node index, -1 for the root
  int32_t edge;    // cost of the edge from the parent
  int32_t lazy;    // learned search: a block of unevaluated children of `parent`
  uint64_t h;      // hash of the canonical key (key_hash)
  int64_t hov;     // overlap heuristic: observed points outside V_j (MHA search)
  double hpr;      // pose-prior heuristic: sum of distances to the estimates
  perch_object last;  // the object this state added to its parent's (not for the root)
  int64_t key[PERCH_MAX_OBJECTS];  // canonical: sorted (mesh << 32 | pose) (first j)
};

// Room for n more elements, growing geometrically (reserve alone would allocate the
// exact size and copy the whole vector on every call).
template <class T>
void grow_for(std::vector<T>& v, size_t n) {
  if (v.size() + n > v.capacity()) v.reserve(std::max(2 * v.capacity(), v.size() + n));
}

// The state's objects in canonical order (materialising a state depends on the set
// only: the composite is a per-pixel minimum).
void objs_of(const Node& n, perch_object* out) {
  for (int k = 0; k < n.j; ++k)
    out[k] = perch_object{(int32_t)(n.key[k] >> 32), (int32_t)(uint32_t)n.key[k]};
}

int64_t pack(int32_t m, int32_t p) { return ((int64_t)m << 32) | (uint32_t)p; }

uint64_t key_hash(const Node& n) {
  uint64_t h = 1469598103934665603ull ^ (uint64_t)n.j;
  for (int k = 0; k < n.j; ++k) {
    h ^= (uint64_t)n.key[k];
    h *= 1099511628211ull;
  }
  return h;
}

// The empty state (the root), with its key hash.
Node root_node() {
  Node r;
  std::memset(&r, 0, sizeof(r));
  r.parent = -1;
  r.h = key_hash(r);
  return r;
}

int cmp_key(const Node& a, const Node& b) {
  for (int k = 0; k < a.j && k < b.j; ++k)
    if (a.key[k] != b.key[k]) return a.key[k] < b.key[k] ? -1 : 1;
  return a.j == b.j ? 0 : (a.j < b.j ? -1 : 1);
}

// Open-addressing table of the states reached so far: per canonical key the node
// id that currently holds it.  Keys are compared by their hash, then in full; an
// entry is only ever replaced (a cheaper path re-opens the state), never removed.
// The key hash's low bits do not see the mesh ids (bits 32 and up of every key), so
// slots come from the hash after a 64-bit finaliser that mixes all its bits.
class StateTable {
 public:
  static size_t home(uint64_t h) {
    h ^= h >> 33;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
    h *= 0xc4ceb9fe1a85ec53ull;
    h ^= h >> 33;
    return (size_t)h;
  }
  explicit StateTable(const std::vector<Node>* nodes) : nodes_(nodes), slots_(1024, -1) {}
  // the slot holding node id's state, or the empty slot where it would go
  size_t slot_of(int id) const {
    const Node& n = (*nodes_)[id];
    const size_t mask = slots_.size() - 1;
    for (size_t s = home(n.h) & mask;; s = (s + 1) & mask) {
      const int e = slots_[s];
      if (e < 0) return s;
      const Node& m = (*nodes_)[e];
      if (m.h == n.h && cmp_key(m, n) == 0) return s;
    }
  }
  int at(size_t s) const { return slots_[s]; }
  // stores id at slot s (from slot_of(id)); the table may grow, moving slots
  void put(size_t s, int id) {
    const bool fresh = slots_[s] < 0;
    slots_[s] = id;
    if (fresh && 2 * ++used_ > slots_.size()) grow();
  }
  bool holds(int id) const { return slots_[slot_of(id)] == id; }

 private:
  void grow() {
    std::vector<int> old;
    old.swap(slots_);
    slots_.assign(2 * old.size(), -1);
    const size_t mask = slots_.size() - 1;
    for (int e : old) {
      if (e < 0) continue;
      size_t s = home((*nodes_)[e].h) & mask;
      while (slots_[s] >= 0) s = (s + 1) & mask;
      slots_[s] = e;
    }
  }
  const std::vector<Node>* nodes_;
  std::vector<int> slots_;
  size_t used_ = 0;
};

// A roctx range for rocprofv3 --marker-trace, closed by end() or at scope exit.
class Range {
 public:
  explicit Range(const char* msg) { roctxRangePushA(msg); }
  ~Range() { end(); }
  void end() {
    if (on_) roctxRangePop();
    on_ = false;
  }

 private:
  bool on_ = true;
};

struct Child {
  int32_t mesh, pose, cost, gain;  // gain: observed points the child adds to V_j
  float x, y, c, s;                // the child's pose values (grid or ICP-adjusted)
};

class Searcher {
 public:
  Searcher(perch_ctx* c, const perch_search_opts* o) : c_(c), o_(*o) {}

  perch_status init() {
    K_ = (int)c_->objects.size();
    if (K_ < 1) return fail(PERCH_E_STATE, "perch_set_objects not called");
    if (o_.pose_subset && o_.n_pose_subset > 0) {
      poses_.assign(o_.pose_subset, o_.pose_subset + o_.n_pose_subset);
      for (int p : poses_)
        if (p < 0 || p >= c_->P) return fail(PERCH_E_ARG, "pose subset index out of range");
    } else {
      poses_.resize(c_->P);
      for (int p = 0; p < c_->P; ++p) poses_[p] = p;
    }
    int distinct = 0;
    std::vector<int> seen;
    for (int m : c_->objects)
      if (std::find(seen.begin(), seen.end(), m) == seen.end()) seen.push_back(m), ++distinct;
    distinct_ = distinct;
    // rotationally symmetric meshes (Sec. IV-E) are tried once per (x, y): the
    // first pose of the list at each distinct position
    bool any_sym = false;
    for (int m : seen) {
      std::vector<int>& L = mesh_poses_[m];
      const bool sym = m < (int)c_->symmetric.size() && c_->symmetric[m];
      any_sym |= sym;
      if (!sym) {
        L = poses_;
        continue;
      }
      std::unordered_map<uint64_t, int> first;
      for (int p : poses_) {
        uint32_t bx, by;
        std::memcpy(&bx, &c_->h_poses[4 * (size_t)p], 4);
        std::memcpy(&by, &c_->h_poses[4 * (size_t)p + 1], 4);
        if (first.emplace(((uint64_t)bx << 32) | by, p).second) L.push_back(p);
      }
    }
    if (any_sym && (o_.mode == PERCH_SEARCH_LEARNED || o_.mode == PERCH_SEARCH_LEARNED_MHA))
      return fail(PERCH_E_ARG, "symmetric meshes are not available to the learned searches");
    const size_t cap = (size_t)distinct * poses_.size();
    HIP_TRY(c_->s_cands.ensure(cap * sizeof(int2)));
    HIP_TRY(c_->s_out.ensure(cap * 3 * sizeof(int32_t)));
    HIP_TRY(c_->s_hcands.ensure(cap * sizeof(int2)));
    HIP_TRY(c_->s_hout.ensure(cap * 3 * sizeof(int32_t)));
    if (o_.icp_iters > 0) {
      if (o_.mode != PERCH_SEARCH_UCS && o_.mode != PERCH_SEARCH_FOCAL &&
          o_.mode != PERCH_SEARCH_MHA)
        return fail(PERCH_E_ARG, "ICP alignment is available to UCS, FOCAL and MHA");
      if (c_->arena_cap < (int)cap)
        return fail(PERCH_E_ARG, "pose arena (%d) smaller than one expansion (%zu)",
                    c_->arena_cap, cap);
      c_->arena_used = 0;  // this search's adjusted poses start the arena afresh
      c_->parent_j = -1;
    }
    t0_ = Clock::now();
    return PERCH_OK;
  }

  float icp_radius() const { return o_.icp_radius > 0.0f ? o_.icp_radius : 0.02f; }

  double elapsed() const { return std::chrono::duration<double>(Clock::now() - t0_).count(); }

  bool over_budget() const {
    if (o_.budget_expansions > 0 && n_expanded_ >= o_.budget_expansions) return true;
    if (o_.budget_s > 0 && elapsed() >= o_.budget_s) return true;
    return false;
  }

  // distinct mesh ids still to place (multiset difference), ascending
  std::vector<int> remaining(const Node& n) const {
    std::vector<int> left(c_->objects.begin(), c_->objects.end());
    for (int k = 0; k < n.j; ++k) {
      auto it = std::find(left.begin(), left.end(), (int32_t)(n.key[k] >> 32));
      if (it != left.end()) left.erase(it);
    }
    std::sort(left.begin(), left.end());
    left.erase(std::unique(left.begin(), left.end()), left.end());
    return left;
  }

  // Materialises n on the GPU and evaluates every child; valid ones go to out.
  // with_gain: also the overlap heuristic's decrease per child.
  perch_status expand(const Node& n, std::vector<Child>& out, bool with_gain = false) {
    Range r("perch_search: expand");
    return expand_impl(n, out, with_gain);
  }

  perch_status expand_impl(const Node& n, std::vector<Child>& out, bool with_gain) {
    out.clear();
    const std::vector<int> rest = remaining(n);
    int2* hc = c_->s_hcands.as<int2>();
    int cnt = 0;
    for (int m : rest)
      for (int p : mesh_poses_.at(m)) hc[cnt++] = make_int2(m, p);
    HIP_TRY(hipMemcpyAsync(c_->s_cands.p, hc, cnt * sizeof(int2), hipMemcpyHostToDevice,
                           c_->stream));
    perch_object po[PERCH_MAX_OBJECTS];
    objs_of(n, po);
    perch_status st = perch_set_parent(c_, po, n.j);
    if (st) return st;
    int32_t* dcost = c_->s_out.as<int32_t>();
    int32_t* dstat = dcost + cnt;
    int32_t* dgain = dstat + cnt;
    const perch_object* dc = reinterpret_cast<const perch_object*>(c_->s_cands.p);
    int icp_base = -1;
    if (o_.icp_iters > 0) {  // align every child first; evaluate it at the adjusted pose
      if ((int64_t)c_->arena_used + cnt > c_->arena_cap) return PERCH_E_BUDGET;  // arena full
      HIP_TRY(c_->s_adj.ensure((size_t)cnt * (sizeof(int2) + 2 * sizeof(int32_t))));
      perch_object* adj = c_->s_adj.as<perch_object>();
      int32_t* nmatch = reinterpret_cast<int32_t*>(adj + cnt);
      icp_base = c_->P + c_->arena_used;
      st = perch_icp_children(c_, dc, cnt, o_.icp_iters, icp_radius(), adj, nmatch, nmatch + cnt);
      if (st) return st;
      dc = adj;
    }
    st = with_gain ? perch_overlap_gain(c_, dc, cnt, dcost, dstat, dgain)
                   : perch_eval_children(c_, dc, cnt, dcost, dstat, nullptr);
    if (st) return st;
    int32_t* hout = c_->s_hout.as<int32_t>();
    HIP_TRY(hipMemcpyAsync(hout, dcost, (with_gain ? 3 : 2) * (size_t)cnt * sizeof(int32_t),
                           hipMemcpyDeviceToHost, c_->stream));
    float* hpose = nullptr;
    if (icp_base >= 0) {
      HIP_TRY(c_->s_hposes.ensure((size_t)cnt * 4 * sizeof(float)));
      hpose = c_->s_hposes.as<float>();
      HIP_TRY(hipMemcpyAsync(hpose, c_->poses.as<float4>() + icp_base,
                             (size_t)cnt * 4 * sizeof(float), hipMemcpyDeviceToHost, c_->stream));
    }
    HIP_TRY(hipStreamSynchronize(c_->stream));
    ++n_expanded_;
    n_evaluated_ += cnt;
    for (int i = 0; i < cnt; ++i) {
      const int s = hout[cnt + i];
      if (s == 1) {
        const float* q = hpose ? hpose + 4 * (size_t)i : &c_->h_poses[4 * (size_t)hc[i].y];
        out.push_back({hc[i].x, icp_base >= 0 ? icp_base + i : hc[i].y, hout[i],
                       with_gain ? hout[2 * cnt + i] : 0, q[0], q[1], q[2], q[3]});
      }
      else if (s == 0)
        ++n_invalid_;
      else
        return fail(PERCH_E_UNSUPPORTED, "successor (%d, %d) failed with status %d", hc[i].x,
                    hc[i].y, s);
    }
    if (hpose) merge_aligned_siblings(out, hpose, icp_base);
    return PERCH_OK;
  }

  // Local ICP pulls neighbouring grid poses of one object onto the same place:
  // siblings of one mesh whose adjusted poses fall in one 1 mm x 1 mm x 0.5 degree
  // cell (well inside the explanation radius) are
  // one child (the cheapest, then the lowest index), so that the search does not
  // expand the same state dozens of times.
  void merge_aligned_siblings(std::vector<Child>& out, const float* hpose, int base) {
    std::unordered_map<uint64_t, size_t> best;
    std::vector<Child> kept;
    kept.reserve(out.size());
    for (const Child& ch : out) {
      const float* q = hpose + 4 * (size_t)(ch.pose - base);
      const int64_t kx = (int64_t)std::llround(q[0] / 1e-3);
      const int64_t ky = (int64_t)std::llround(q[1] / 1e-3);
      const double deg = std::atan2((double)q[3], (double)q[2]) * (180.0 / 3.14159265358979323846);
      const int64_t kt = ((int64_t)std::llround(deg / 0.5) % 720 + 720) % 720;
      const uint64_t key = ((uint64_t)(ch.mesh & 0xFFF) << 52) ^
                           ((uint64_t)(kx & 0xFFFFF) << 32) ^ ((uint64_t)(ky & 0xFFFFF) << 12) ^
                           (uint64_t)kt;
      auto it = best.find(key);
      if (it == best.end()) {
        best.emplace(key, kept.size());
        kept.push_back(ch);
      } else {
        Child& b = kept[it->second];
        if (ch.cost < b.cost || (ch.cost == b.cost && ch.pose < b.pose)) b = ch;
        ++n_merged_;
      }
    }
    out.swap(kept);
  }

  Node child_of(const Node& n, int32_t id, const Child& ch) const {
    Node m;
    m.j = n.j + 1;
    m.g = n.g + ch.cost;
    m.parent = id;
    m.edge = ch.cost;
    m.lazy = 0;
    m.last = perch_object{ch.mesh, ch.pose};
    // the parent's sorted key with the new object inserted in place
    const int64_t nk = pack(ch.mesh, ch.pose);
    int k = n.j;
    while (k > 0 && n.key[k - 1] > nk) {
      m.key[k] = n.key[k - 1];
      --k;
    }
    m.key[k] = nk;
    std::memcpy(m.key, n.key, sizeof(int64_t) * k);
    m.h = key_hash(m);
    m.hov = n.hov - ch.gain;
    m.hpr = n.hpr + prior_term(ch);
    return m;
  }

  // ||O - O'|| of the pose-prior heuristic: the smallest distance from the child's
  // object to an estimate of the same mesh, table-plane metres plus
  // prior_rad_m metres per radian of yaw (yaw ignored for symmetric meshes); 0
  // when the mesh has no estimate.
  double prior_term(const Child& ch) const {
    double best = -1.0;
    const bool sym = ch.mesh < (int)c_->symmetric.size() && c_->symmetric[ch.mesh];
    const double th = std::atan2((double)ch.s, (double)ch.c);
    for (int k = 0; k < o_.n_priors; ++k) {
      const perch_pose_prior& q = o_.priors[k];
      if (q.mesh_id != ch.mesh) continue;
      double d = std::hypot((double)ch.x - q.x, (double)ch.y - q.y);
      if (!sym) {
        double a = std::fabs(th - (double)q.theta);
        a = std::fmod(a, 2.0 * 3.14159265358979323846);
        if (a > 3.14159265358979323846) a = 2.0 * 3.14159265358979323846 - a;
        d += prior_rad_m() * a;
      }
      if (best < 0.0 || d < best) best = d;
    }
    return best < 0.0 ? 0.0 : best;
  }
  double prior_rad_m() const { return o_.prior_rad_m > 0.0f ? o_.prior_rad_m : 0.05; }
  double prior_slot_m() const { return o_.prior_slot_m > 0.0f ? o_.prior_slot_m : 0.1; }

  // Anytime trace: an entry whenever the incumbent cost improves (force) and at
  // most every 0.25 s otherwise; the last slot is kept for the end of the search.
  void trace(bool force) {
    const double t = elapsed();
    if (!force && n_trace_ > 0 && t - trace_t_[n_trace_ - 1] < 0.25) return;
    const int k = n_trace_ < PERCH_TRACE ? n_trace_++ : PERCH_TRACE - 1;
    trace_t_[k] = t;
    trace_cost_[k] = have_ ? best_.g : -1;
    trace_lb_[k] = lower_bound_;
  }

  void offer_goal(const Node& g, const std::vector<Node>* store) {
    if (have_ && (g.g > best_.g || (g.g == best_.g && cmp_key(g, best_) >= 0))) return;
    const bool cost_improved = !have_ || g.g < best_.g;
    have_ = true;
    best_ = g;
    if (cost_improved) {
      t_best_ = elapsed();
      n_eval_best_ = n_evaluated_;
      trace(true);
    }
    // objects in insertion order and edge costs along the path (without a store
    // the caller fills them in)
    std::memset(best_edges_, 0, sizeof(best_edges_));
    if (store) {
      best_edges_[g.j - 1] = g.edge;
      best_objs_[g.j - 1] = g.last;
      for (int id = g.parent, k = g.j - 2; id >= 0 && k >= 0; id = (*store)[id].parent, --k) {
        best_edges_[k] = (*store)[id].edge;
        best_objs_[k] = (*store)[id].last;
      }
    }
  }

  // ---- exhaustive ----
  perch_status exhaustive() {
    const Node root = root_node();
    path_edges_.assign(K_, 0);
    path_objs_.assign(K_, perch_object{0, 0});
    return dfs(root);
  }

  perch_status dfs(const Node& n) {
    if (over_budget()) return PERCH_E_BUDGET;
    std::vector<Child> kids;
    perch_status st = expand(n, kids);
    if (st) return st;
    for (const Child& ch : kids) {
      Node m = child_of(n, -1, ch);
      path_edges_[n.j] = ch.cost;
      path_objs_[n.j] = m.last;
      if (m.j == K_) {
        const bool better = !have_ || m.g < best_.g || (m.g == best_.g && cmp_key(m, best_) < 0);
        offer_goal(m, nullptr);
        if (better) {
          std::copy(path_edges_.begin(), path_edges_.end(), best_edges_);
          std::copy(path_objs_.begin(), path_objs_.end(), best_objs_);
        }
      } else {
        st = dfs(m);
        if (st) return st;
      }
    }
    return PERCH_OK;
  }

  // ---- uniform-cost and focal ----
  // n_inad inadmissible queues: 0 uniform-cost, 1 focal (h_depth), 2 Focal-MHA*
  // (h_depth and h_overlap, round robin).
  perch_status best_first(int n_inad) {
    const bool focal = n_inad > 0;
    std::vector<Node> nodes;
    nodes.reserve(1 << 16);
    Node root = root_node();
    root.hov = c_->n_points;  // h_overlap(root) = |I|
    nodes.push_back(root);
    StateTable table(&nodes);
    table.put(table.slot_of(0), 0);
    std::vector<char> closed(1, 0);
    // priority: smaller g, deeper, smaller key; entries carry g and depth so that
    // most comparisons need not read the nodes
    struct GEntry {
      int64_t g;
      int32_t j, id;
    };
    auto g_less = [&](const GEntry& a, const GEntry& b) {
      if (a.g != b.g) return a.g > b.g;
      if (a.j != b.j) return a.j < b.j;
      return cmp_key(nodes[a.id], nodes[b.id]) > 0;
    };
    auto g_entry = [&](int id) { return GEntry{nodes[id].g, nodes[id].j, id}; };
    std::priority_queue<GEntry, std::vector<GEntry>, decltype(g_less)> open(g_less);
    // focal heap: deeper first (h_depth = K - |s|), then smaller g, then key
    auto d_less = [&](int a, int b) {
      const Node &x = nodes[a], &y = nodes[b];
      if (x.j != y.j) return x.j < y.j;
      if (x.g != y.g) return x.g > y.g;
      return cmp_key(x, y) > 0;
    };
    std::priority_queue<int, std::vector<int>, decltype(d_less)> focal_q(d_less);
    // overlap heap: fewer observed points outside V_j first, then smaller g, then key
    auto o_less = [&](int a, int b) {
      const Node &x = nodes[a], &y = nodes[b];
      if (x.hov != y.hov) return x.hov > y.hov;
      if (x.g != y.g) return x.g > y.g;
      return cmp_key(x, y) > 0;
    };
    std::priority_queue<int, std::vector<int>, decltype(o_less)> over_q(o_less);
    // pose-prior heap: the sum of distances to the estimates plus prior_slot_m for
    // each object still to place, then smaller g, then key
    auto hp = [&](const Node& x) { return x.hpr + prior_slot_m() * (K_ - x.j); };
    auto p_less = [&](int a, int b) {
      const Node &x = nodes[a], &y = nodes[b];
      const double hx = hp(x), hy = hp(y);
      if (hx != hy) return hx > hy;
      if (x.g != y.g) return x.g > y.g;
      return cmp_key(x, y) > 0;
    };
    std::priority_queue<int, std::vector<int>, decltype(p_less)> prior_q(p_less);
    // states waiting for the focal bound, ordered by g
    std::priority_queue<GEntry, std::vector<GEntry>, decltype(g_less)> pending(g_less);
    open.push(g_entry(0));
    if (focal) pending.push(g_entry(0));
    std::vector<Child> kids;
    auto live = [&](int id) { return !closed[id] && table.holds(id); };
    const double w = std::max(1.0f, o_.w);
    for (;;) {
      while (!open.empty() && !live(open.top().id)) open.pop();
      if (open.empty()) break;
      const int64_t gmin = open.top().g;
      lower_bound_ = gmin;
      trace(false);
      if (have_ && best_.g <= gmin) break;  // incumbent proven optimal
      if (over_budget()) return PERCH_E_BUDGET;
      int pick = -1;
      if (focal) {
        while (!pending.empty() && (double)pending.top().g <= w * (double)gmin) {
          const int id = pending.top().id;
          if (live(id)) {
            focal_q.push(id);
            if (n_inad > 1) over_q.push(id);
            if (n_inad > 2) prior_q.push(id);
          }
          pending.pop();
        }
        while (!focal_q.empty() && !live(focal_q.top())) focal_q.pop();
        while (!over_q.empty() && !live(over_q.top())) over_q.pop();
        while (!prior_q.empty() && !live(prior_q.top())) prior_q.pop();
        // round robin over the inadmissible queues, and the anchor when anytime
        const int cycle = n_inad + (o_.anytime ? 1 : 0);
        const int slot = (int)(expansions_ % cycle);
        for (int t = 0; t < n_inad && pick < 0 && slot < n_inad; ++t) {
          const int q = (slot + t) % n_inad;
          if (q == 0 && !focal_q.empty()) {
            pick = focal_q.top();
            focal_q.pop();
          } else if (q == 1 && !over_q.empty()) {
            pick = over_q.top();
            over_q.pop();
          } else if (q == 2 && !prior_q.empty()) {
            pick = prior_q.top();
            prior_q.pop();
          }
        }
      }
      if (pick < 0) {
        pick = open.top().id;
        open.pop();
      }
      ++expansions_;
      const Node cur = nodes[pick];
      closed[pick] = 1;
      if (cur.j == K_) {
        offer_goal(cur, &nodes);
        if (!focal || !o_.anytime) break;  // first goal popped / chosen from FOCAL
        continue;
      }
      perch_status st = expand(cur, kids, n_inad > 1);
      if (st) return st;
      grow_for(nodes, kids.size());  // one reallocation for the whole batch of children
      grow_for(closed, kids.size());
      for (const Child& ch : kids) {
        if (have_ && cur.g + ch.cost >= best_.g) continue;  // cannot improve the incumbent
        nodes.push_back(child_of(cur, pick, ch));
        closed.push_back(0);
        const int id = (int)nodes.size() - 1;
        const size_t slot = table.slot_of(id);
        const int prev = table.at(slot);
        // a cheaper path re-opens the state, also after its expansion: a state closed
        // from FOCAL may carry a g above its optimum, and the anchor's min g stays a
        // lower bound on the optimum only if it is re-opened
        if (prev >= 0 && !(nodes[id].g < nodes[prev].g)) {
          nodes.pop_back();
          closed.pop_back();
          continue;
        }
        table.put(slot, id);
        open.push(g_entry(id));
        if (focal) pending.push(g_entry(id));
        if (nodes[id].j == K_ && focal && o_.anytime) offer_goal(nodes[id], &nodes);
      }
    }
    return PERCH_OK;
  }

  // ---- learned ----
  // with_overlap: the paper's h_overlap as a second inadmissible queue over the
  // children the network lets through (and those of popped lazy blocks).
  perch_status learned(bool with_overlap) {
    if (!o_.cnn) return fail(PERCH_E_ARG, "the learned search needs a network");
    const int topk = o_.topk > 0 ? o_.topk : 64;
    const int P = (int)poses_.size();
    // pose cells: one crop per distinct (x, y) of the pose set
    std::vector<float> cells;
    std::vector<int> cell_of(poses_.size());
    {
      std::map<std::pair<float, float>, int> idx;
      for (size_t k = 0; k < poses_.size(); ++k) {
        const float* pz = &c_->h_poses[4 * (size_t)poses_[k]];
        auto it = idx.find({pz[0], pz[1]});
        if (it == idx.end()) {
          it = idx.emplace(std::make_pair(pz[0], pz[1]), (int)(cells.size() / 2)).first;
          cells.push_back(pz[0]);
          cells.push_back(pz[1]);
        }
        cell_of[k] = it->second;
      }
    }
    const int n_cells = (int)(cells.size() / 2);
    // the distinct meshes of the multiset; child id = (position in this list) P + pose
    std::vector<int> dist(c_->objects.begin(), c_->objects.end());
    std::sort(dist.begin(), dist.end());
    dist.erase(std::unique(dist.begin(), dist.end()), dist.end());
    const int nd = (int)dist.size();
    if (nd > kMaxMeshes) return fail(PERCH_E_UNSUPPORTED, "more than %d distinct meshes", kMaxMeshes);
    const size_t maxp = (size_t)nd * P;
    // everything a ranking needs stays on the device for the whole search
    std::vector<cnn::CropDesc> hdesc(n_cells);
    const Cam& cam = c_->cam;
    if (!cnn::crop_descriptors(cam.M, cam.fx, cam.fy, cam.cx, cam.cy, cells.data(), n_cells,
                               hdesc.data(), cnn_crop_step(o_.cnn)))
      return fail(PERCH_E_ARG, "a pose cell lies behind the camera");
    std::vector<perch_cnn_pair> hp(maxp);
    for (int a = 0; a < nd; ++a)
      for (int b = 0; b < P; ++b) {
        const float* pz = &c_->h_poses[4 * (size_t)poses_[b]];
        hp[(size_t)a * P + b] = perch_cnn_pair{cell_of[b], dist[a], pz[2], pz[3]};
      }
    // device buffers kept by the context between searches (grown on demand)
    DevBuf* lb = c_->learned_bufs;
    DevBuf &d_desc = lb[0], &d_pairs = lb[1], &d_dist = lb[2], &d_pose = lb[3];
    DevBuf& d_pred = lb[5];  // lb[4] unused (crops are sampled inside the network's first
                             // kernel); lb[6..10]: the ranking's buffers (rank_children)
    HIP_TRY(d_desc.ensure(sizeof(cnn::CropDesc) * n_cells));
    HIP_TRY(d_pairs.ensure(sizeof(perch_cnn_pair) * maxp));
    HIP_TRY(d_dist.ensure(sizeof(int) * nd));
    HIP_TRY(d_pose.ensure(sizeof(int) * P));
    HIP_TRY(d_pred.ensure(sizeof(float) * maxp));
    hipStream_t st0 = c_->stream;
    // stream-ordered uploads; the host arrays outlive the search's first synchronisation
    HIP_TRY(hipMemcpyAsync(d_desc.p, hdesc.data(), sizeof(cnn::CropDesc) * n_cells,
                           hipMemcpyHostToDevice, st0));
    HIP_TRY(hipMemcpyAsync(d_pairs.p, hp.data(), sizeof(perch_cnn_pair) * maxp,
                           hipMemcpyHostToDevice, st0));
    HIP_TRY(hipMemcpyAsync(d_dist.p, dist.data(), sizeof(int) * nd, hipMemcpyHostToDevice, st0));
    HIP_TRY(hipMemcpyAsync(d_pose.p, poses_.data(), sizeof(int) * P, hipMemcpyHostToDevice,
                           st0));

    // Children of n: materialise n, crop every cell, predict every (mesh, pose),
    // rank on the device (children of meshes already placed rank last), evaluate
    // the k best exactly; one synchronisation.  all = nothing is left over.
    auto learned_expand = [&](const Node& n, std::vector<Child>& out, bool& all) -> perch_status {
      Range r("learned: expansion");
      out.clear();
      const std::vector<int> rest = remaining(n);
      const int cnt = (int)rest.size() * P;
      MeshMask mask{};
      for (int a = 0; a < nd; ++a)
        mask.allow[a] = std::find(rest.begin(), rest.end(), dist[a]) != rest.end() ? 1 : 0;
      perch_object po[PERCH_MAX_OBJECTS];
      objs_of(n, po);
      perch_status st = perch_set_parent(c_, po, n.j);
      if (st) return st;
      st = cnn_predict_scene_on(o_.cnn, c_, d_desc.p, n_cells, d_pairs.p, (int)maxp,
                                d_pred.as<float>(), st0);
      if (st) return st;
      const int k = std::min(topk, cnt);
      all = k == cnt;
      int2* dc = c_->s_cands.as<int2>();
      st = rank_children(c_, d_pred.as<float>(), P, nd, mask, k, d_dist.as<int>(),
                         d_pose.as<int>(), dc, st0);
      if (st) return st;
      int32_t* dcost = c_->s_out.as<int32_t>();
      int32_t* dstat = dcost + k;
      int32_t* dgain = dstat + k;
      const perch_object* dco = reinterpret_cast<const perch_object*>(dc);
      st = with_overlap ? perch_overlap_gain(c_, dco, k, dcost, dstat, dgain)
                        : perch_eval_children(c_, dco, k, dcost, dstat, nullptr);
      if (st) return st;
      int2* hc = c_->s_hcands.as<int2>();
      int32_t* hout = c_->s_hout.as<int32_t>();
      HIP_TRY(hipMemcpyAsync(hc, dc, k * sizeof(int2), hipMemcpyDeviceToHost, st0));
      HIP_TRY(hipMemcpyAsync(hout, dcost, (with_overlap ? 3 : 2) * (size_t)k * sizeof(int32_t),
                             hipMemcpyDeviceToHost, st0));
      HIP_TRY(hipStreamSynchronize(st0));
      ++n_expanded_;
      n_evaluated_ += k;
      for (int i = 0; i < k; ++i) {
        const int s2 = hout[k + i];
        if (s2 == 1)
          out.push_back({hc[i].x, hc[i].y, hout[i], with_overlap ? hout[2 * k + i] : 0});
        else if (s2 == 0)
          ++n_invalid_;
        else
          return fail(PERCH_E_UNSUPPORTED, "successor (%d, %d) failed with status %d", hc[i].x,
                      hc[i].y, s2);
      }
      return PERCH_OK;
    };

    std::vector<Node> nodes;
    nodes.reserve(1 << 16);
    nodes.push_back(root_node());
    StateTable table(&nodes);
    table.put(table.slot_of(0), 0);
    std::vector<char> closed(1, 0);
    auto a_less = [&](int a, int b) {  // anchor: smaller key g, deeper, states before blocks
      const Node &x = nodes[a], &y = nodes[b];
      if (x.g != y.g) return x.g > y.g;
      if (x.j != y.j) return x.j < y.j;
      if (x.lazy != y.lazy) return x.lazy > y.lazy;
      return cmp_key(x, y) > 0;
    };
    auto d_less = [&](int a, int b) {  // inadmissible: deeper first, then smaller g
      const Node &x = nodes[a], &y = nodes[b];
      if (x.j != y.j) return x.j < y.j;
      if (x.g != y.g) return x.g > y.g;
      return cmp_key(x, y) > 0;
    };
    std::priority_queue<int, std::vector<int>, decltype(a_less)> open(a_less), pending(a_less);
    std::priority_queue<int, std::vector<int>, decltype(d_less)> focal_q(d_less);
    auto o_less = [&](int a, int b) {  // inadmissible: fewer points outside V_j, then g
      const Node &x = nodes[a], &y = nodes[b];
      if (x.hov != y.hov) return x.hov > y.hov;
      if (x.g != y.g) return x.g > y.g;
      return cmp_key(x, y) > 0;
    };
    std::priority_queue<int, std::vector<int>, decltype(o_less)> over_q(o_less);
    nodes[0].hov = c_->n_points;  // h_overlap(root) = |I|
    auto live = [&](int id) {
      if (closed[id]) return false;
      if (nodes[id].lazy) return true;
      return table.holds(id);
    };
    auto push_child = [&](const Node& parent, int pid, const Child& ch) {
      Node m = child_of(parent, pid, ch);
      if (m.j == K_) offer_goal(m, &nodes);
      if (have_ && m.g >= best_.g) return;  // cannot improve the incumbent
      nodes.push_back(m);
      closed.push_back(0);
      const int id = (int)nodes.size() - 1;
      const size_t slot = table.slot_of(id);
      const int prev = table.at(slot);
      if (prev >= 0 && !(m.g < nodes[prev].g)) {  // re-open on a cheaper path, as above
        nodes.pop_back();
        closed.pop_back();
        return;
      }
      table.put(slot, id);
      open.push(id);
      pending.push(id);
    };
    open.push(0);
    pending.push(0);
    std::vector<Child> kids;
    const double w = std::max(1.0f, o_.w);
    const int n_inad = with_overlap ? 2 : 1;
    // Next state to expand, as the single-state search picks it (round robin over
    // the inadmissible queues restricted to FOCAL, and the anchor when anytime);
    // -1 when the open list is empty.
    auto next_pick = [&]() -> int {
      while (!open.empty() && !live(open.top())) open.pop();
      if (open.empty()) return -1;
      const int64_t gmin = nodes[open.top()].g;
      while (!pending.empty() && (double)nodes[pending.top()].g <= w * (double)gmin) {
        if (live(pending.top())) {
          focal_q.push(pending.top());
          if (with_overlap) over_q.push(pending.top());
        }
        pending.pop();
      }
      while (!focal_q.empty() && !live(focal_q.top())) focal_q.pop();
      while (!over_q.empty() && !live(over_q.top())) over_q.pop();
      const int slot = (int)(expansions_ % (n_inad + (o_.anytime ? 1 : 0)));
      int pick = -1;
      for (int t = 0; t < n_inad && pick < 0 && slot < n_inad; ++t) {
        const int q = (slot + t) % n_inad;
        if (q == 0 && !focal_q.empty()) {
          pick = focal_q.top();
          focal_q.pop();
        } else if (q == 1 && !over_q.empty()) {
          pick = over_q.top();
          over_q.pop();
        }
      }
      if (pick < 0) {
        pick = open.top();
        open.pop();
      }
      ++expansions_;
      closed[pick] = 1;
      return pick;
    };
    const int B = o_.batch > 1 ? o_.batch : 1;
    if (B > 1) {
      // Several states per step: the learned part (crops, network, ranking) of every
      // picked state and the exact evaluation of all their chosen children, and of
      // every popped lazy block's children, in one persistent batched launch, with
      // one synchronisation.  The queues, the selection rule and the stopping rules
      // are those of the single-state search, applied between steps.
      if (with_overlap)
        return fail(PERCH_E_ARG, "the learned search with h_overlap expands one state per step");
      int cap_crops = 0, cap_pairs = 0;
      perch_status cst = cnn_capacity(o_.cnn, &cap_crops, &cap_pairs);
      if (cst) return cst;
      if ((int64_t)cap_crops < (int64_t)B * n_cells || (int64_t)cap_pairs < (int64_t)B * maxp)
        return fail(PERCH_E_ARG,
                    "network capacity (%d crops, %d pairs) below %d states per step (%lld, %lld)",
                    cap_crops, cap_pairs, B, (long long)B * n_cells, (long long)B * maxp);
      const size_t crop_elems = (size_t)64 * 64 * 2;
      const size_t max_items = (size_t)B * maxp;
      HIP_TRY(c_->s_bcrops.ensure((size_t)B * n_cells * crop_elems * sizeof(uint16_t)));
      HIP_TRY(c_->s_bpairs.ensure((size_t)B * maxp * sizeof(perch_cnn_pair)));
      HIP_TRY(c_->s_bpred.ensure((size_t)B * maxp * sizeof(float)));
      HIP_TRY(c_->s_bcands.ensure((size_t)B * topk * sizeof(int2)));
      HIP_TRY(c_->s_items.ensure(max_items * sizeof(int4)));
      HIP_TRY(c_->s_bout.ensure(max_items * 2 * sizeof(int32_t)));
      HIP_TRY(c_->s_hitems.ensure(max_items * sizeof(int4)));
      HIP_TRY(c_->s_hbout.ensure(max_items * 2 * sizeof(int32_t)));
      // the pair table once per state slot, crop indices offset by the slot's crops
      std::vector<perch_cnn_pair> hpb((size_t)B * maxp);
      for (int k = 0; k < B; ++k)
        for (size_t i = 0; i < maxp; ++i) {
          hpb[(size_t)k * maxp + i] = hp[i];
          hpb[(size_t)k * maxp + i].crop += k * n_cells;
        }
      HIP_TRY(hipMemcpyAsync(c_->s_bpairs.p, hpb.data(), hpb.size() * sizeof(perch_cnn_pair),
                             hipMemcpyHostToDevice, st0));
      HIP_TRY(hipStreamSynchronize(st0));  // hpb is freed at the end of this block
      if (!c_->s_batch) {
        perch_ctx* self = c_;
        perch_status st = perch_batch_create(&self, 1, st0, &c_->s_batch);
        if (st) return st;
      }
      perch_batch* bat = c_->s_batch;
      perch_status st = perch_batch_set_tuning(bat, 0, 0, 0, -1);  // sizes vary: no graph
      if (st) return st;
      int4* d_items = c_->s_items.as<int4>();
      int32_t* d_out = c_->s_bout.as<int32_t>();
      uint16_t* d_bcrops = c_->s_bcrops.as<uint16_t>();
      float* d_bpred = c_->s_bpred.as<float>();
      int2* d_bcands = c_->s_bcands.as<int2>();
      int4* h_items = c_->s_hitems.as<int4>();
      int32_t* h_out = c_->s_hbout.as<int32_t>();
      std::vector<int> learn, lazy, owner;  // owner[slot]: node whose children the slot holds
      std::vector<perch_parent> pars;
      std::vector<char> full;  // learned slots whose top-k covered every child
      for (;;) {
        while (!open.empty() && !live(open.top())) open.pop();
        if (open.empty()) {
          if (have_) lower_bound_ = best_.g;
          break;
        }
        const int64_t gmin = nodes[open.top()].g;
        lower_bound_ = gmin;
        trace(false);
        if (have_ && best_.g <= gmin) break;
        if (have_ && !o_.anytime && (double)best_.g <= w * (double)gmin) break;
        if (over_budget()) return PERCH_E_BUDGET;
        learn.clear();
        lazy.clear();
        while ((int)(learn.size() + lazy.size()) < B) {
          const int pick = next_pick();
          if (pick < 0) break;
          if (nodes[pick].lazy)
            lazy.push_back(pick);
          else if (nodes[pick].j < K_)  // goals were offered when generated
            learn.push_back(pick);
        }
        if (learn.empty() && lazy.empty()) continue;
        const int L = (int)learn.size(), Z = (int)lazy.size();
        pars.assign(L + Z, perch_parent{});
        owner.assign(L + Z, -1);
        for (int k = 0; k < L + Z; ++k) {
          owner[k] = k < L ? learn[k] : nodes[lazy[k - L]].parent;
          const Node& n = nodes[owner[k]];
          pars[k].ctx = 0;
          pars[k].j = n.j;
          objs_of(n, pars[k].objs);
        }
        Range r_par("learned batch: parents");
        st = perch_batch_set_parents(bat, pars.data(), L + Z);
        r_par.end();
        if (st) return st;
        // the learned part of the picked states
        Range r_net("learned batch: network");
        for (int k = 0; k < L; ++k)
          cnn::launch_crops(c_->obs.as<float>(), batch_slot_depth(bat, k), cam.W, cam.H,
                            d_desc.as<cnn::CropDesc>(), n_cells, d_bcrops + (size_t)k * n_cells * crop_elems,
                            st0);
        if (L > 0) {
          st = cnn_predict_on(o_.cnn, d_bcrops, L * n_cells, c_->s_bpairs.p, (int)(L * maxp),
                              d_bpred, st0);
          if (st) return st;
        }
        r_net.end();
        Range r_rank("learned batch: ranking");
        size_t n_items = 0;
        full.assign(L, 0);
        for (int k = 0; k < L; ++k) {
          const std::vector<int> rest = remaining(nodes[learn[k]]);
          const int cnt = (int)rest.size() * P;
          MeshMask mask{};
          for (int a = 0; a < nd; ++a)
            mask.allow[a] = std::find(rest.begin(), rest.end(), dist[a]) != rest.end() ? 1 : 0;
          const int kk = std::min(topk, cnt);
          full[k] = kk == cnt;
          st = rank_children(c_, d_bpred + (size_t)k * maxp, P, nd, mask, kk, d_dist.as<int>(),
                             d_pose.as<int>(), d_bcands + (size_t)k * topk, st0);
          if (st) return st;
          launch_items_from_cands(d_bcands + (size_t)k * topk, kk, k, d_items + n_items, st0);
          n_items += kk;
        }
        for (int z = 0; z < Z; ++z) {  // every child of a popped lazy block's parent
          const std::vector<int> rest = remaining(nodes[owner[L + z]]);
          MeshList ml{};
          for (size_t a = 0; a < rest.size(); ++a) ml.id[a] = rest[a];
          launch_items_all(L + z, ml, (int)rest.size(), d_pose.as<int>(), P, d_items + n_items,
                           st0);
          n_items += rest.size() * (size_t)P;
        }
        HIP_TRY(hipGetLastError());
        r_rank.end();
        Range r_exact("learned batch: exact evaluation");
        st = perch_batch_eval(bat, reinterpret_cast<const perch_work*>(d_items), (int)n_items,
                              d_out, d_out + n_items, nullptr);
        if (st) return st;
        HIP_TRY(hipMemcpyAsync(h_items, d_items, n_items * sizeof(int4), hipMemcpyDeviceToHost,
                               st0));
        HIP_TRY(hipMemcpyAsync(h_out, d_out, n_items * 2 * sizeof(int32_t),
                               hipMemcpyDeviceToHost, st0));
        HIP_TRY(hipStreamSynchronize(st0));
        r_exact.end();
        Range r_q("learned batch: queues");
        n_expanded_ += L + Z;
        n_evaluated_ += (int64_t)n_items;
        for (size_t i = 0; i < n_items; ++i) {
          const int4 it = h_items[i];
          const int s2 = h_out[n_items + i];
          if (s2 == 1) {
            const int pid = owner[it.x];
            const Node par = nodes[pid];
            push_child(par, pid, Child{it.y, it.z, h_out[i], 0});
          } else if (s2 == 0) {
            ++n_invalid_;
          } else {
            return fail(PERCH_E_UNSUPPORTED, "successor (%d, %d) failed with status %d", it.y,
                        it.z, s2);
          }
        }
        for (int k = 0; k < L; ++k) {  // the rest of each picked state's children wait
          if (full[k]) continue;
          Node lz = nodes[learn[k]];
          lz.lazy = 1;
          lz.parent = learn[k];
          nodes.push_back(lz);
          closed.push_back(0);
          open.push((int)nodes.size() - 1);
        }
      }
      return PERCH_OK;
    }
    for (;;) {
      while (!open.empty() && !live(open.top())) open.pop();
      if (open.empty()) {  // every state was expanded: the incumbent is optimal
        if (have_) lower_bound_ = best_.g;
        break;
      }
      const int64_t gmin = nodes[open.top()].g;
      lower_bound_ = gmin;
      trace(false);
      if (have_ && best_.g <= gmin) break;  // incumbent proven optimal
      if (have_ && !o_.anytime && (double)best_.g <= w * (double)gmin) break;  // w-bound met
      if (over_budget()) return PERCH_E_BUDGET;
      while (!pending.empty() && (double)nodes[pending.top()].g <= w * (double)gmin) {
        if (live(pending.top())) {
          focal_q.push(pending.top());
          if (with_overlap) over_q.push(pending.top());
        }
        pending.pop();
      }
      while (!focal_q.empty() && !live(focal_q.top())) focal_q.pop();
      while (!over_q.empty() && !live(over_q.top())) over_q.pop();
      // round robin over the inadmissible queues, and the anchor when anytime
      const int n_inad = with_overlap ? 2 : 1;
      const int slot = (int)(expansions_ % (n_inad + (o_.anytime ? 1 : 0)));
      int pick = -1;
      for (int t = 0; t < n_inad && pick < 0 && slot < n_inad; ++t) {
        const int q = (slot + t) % n_inad;
        if (q == 0 && !focal_q.empty()) {
          pick = focal_q.top();
          focal_q.pop();
        } else if (q == 1 && !over_q.empty()) {
          pick = over_q.top();
          over_q.pop();
        }
      }
      if (pick < 0) {
        pick = open.top();
        open.pop();
      }
      ++expansions_;
      closed[pick] = 1;
      const Node cur = nodes[pick];
      if (cur.lazy) {  // the rest of a parent's children: evaluate them all
        const Node par = nodes[cur.parent];
        perch_status st = expand(par, kids, with_overlap);
        if (st) return st;
        for (const Child& ch : kids) push_child(par, cur.parent, ch);
        continue;
      }
      if (cur.j == K_) continue;  // goals were offered when generated
      bool all = false;
      perch_status st = learned_expand(cur, kids, all);
      if (st) return st;
      for (const Child& ch : kids) push_child(cur, pick, ch);
      if (all) continue;
      Node lz = cur;
      lz.lazy = 1;
      lz.parent = pick;
      nodes.push_back(lz);
      closed.push_back(0);
      open.push((int)nodes.size() - 1);
    }
    return PERCH_OK;
  }

  void fill(perch_result* r) const {
    std::memset(r, 0, sizeof(*r));
    r->K = K_;
    r->found = have_;
    if (have_) {
      r->cost = best_.g;
      for (int k = 0; k < best_.j; ++k) {
        r->objs[k] = best_objs_[k];
        r->edge_cost[k] = best_edges_[k];
      }
    } else {
      r->cost = -1;
    }
    r->n_expanded = n_expanded_;
    r->n_evaluated = n_evaluated_;
    r->n_invalid = n_invalid_;
    r->n_merged = n_merged_;
    r->t_total_s = elapsed();
    r->t_best_s = have_ ? t_best_ : -1.0;
    r->n_evaluated_best = have_ ? n_eval_best_ : -1;
    r->lower_bound = lower_bound_;
    r->n_trace = n_trace_;
    for (int k = 0; k < n_trace_; ++k) {
      r->trace_t[k] = trace_t_[k];
      r->trace_cost[k] = trace_cost_[k];
      r->trace_lb[k] = trace_lb_[k];
    }
  }

 private:
  perch_ctx* c_;
  perch_search_opts o_;
  int K_ = 0;
  int distinct_ = 0;
  std::vector<int> poses_;
  std::map<int, std::vector<int>> mesh_poses_;  // per object mesh: the poses it is tried at
  Clock::time_point t0_;
  int64_t n_expanded_ = 0, n_evaluated_ = 0, n_invalid_ = 0, expansions_ = 0, n_merged_ = 0;
  int64_t lower_bound_ = 0;
  bool have_ = false;
  Node best_{};
  int32_t best_edges_[PERCH_MAX_OBJECTS] = {0};
  perch_object best_objs_[PERCH_MAX_OBJECTS] = {};
  std::vector<int32_t> path_edges_;
  std::vector<perch_object> path_objs_;
  double t_best_ = -1.0;
  int64_t n_eval_best_ = -1;
  int n_trace_ = 0;
  double trace_t_[PERCH_TRACE] = {0};
  int64_t trace_cost_[PERCH_TRACE] = {0}, trace_lb_[PERCH_TRACE] = {0};
};

}  // namespace

// One JSON line per search appended to the file named by PERCH_SEARCH_LOG (when set
// and non-empty): the options, the outcome and the anytime trace.  A file that cannot
// be opened is skipped silently; the search's result does not depend on it.
static void log_search(const perch_search_opts* o, const perch_result& r, perch_status st) {
  const char* path = std::getenv("PERCH_SEARCH_LOG");
  if (!path || !*path) return;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f,
               "{\"mode\": %d, \"w\": %.9g, \"anytime\": %d, \"budget_s\": %.9g, "
               "\"budget_expansions\": %lld, \"topk\": %d, \"batch\": %d, \"icp_iters\": %d, "
               "\"n_priors\": %d, \"status\": %d, \"K\": %d, \"found\": %d, \"cost\": %lld, "
               "\"lower_bound\": %lld, \"n_expanded\": %lld, \"n_evaluated\": %lld, "
               "\"n_invalid\": %lld, \"n_merged\": %lld, \"n_evaluated_best\": %lld, "
               "\"t_total_s\": %.9g, \"t_best_s\": %.9g, \"objs\": [",
               o->mode, (double)o->w, o->anytime, o->budget_s, (long long)o->budget_expansions,
               o->topk, o->batch, o->icp_iters, o->n_priors, (int)st, r.K, r.found,
               (long long)r.cost, (long long)r.lower_bound, (long long)r.n_expanded,
               (long long)r.n_evaluated, (long long)r.n_invalid, (long long)r.n_merged,
               (long long)r.n_evaluated_best, r.t_total_s, r.t_best_s);
  for (int k = 0; r.found && k < r.K; ++k)
    std::fprintf(f, "%s[%d, %d, %d]", k ? ", " : "", r.objs[k].mesh_id, r.objs[k].pose_idx,
                 r.edge_cost[k]);
  std::fprintf(f, "], \"trace\": [");
  for (int k = 0; k < r.n_trace; ++k)
    std::fprintf(f, "%s[%.6g, %lld, %lld]", k ? ", " : "", r.trace_t[k],
                 (long long)r.trace_cost[k], (long long)r.trace_lb[k]);
  std::fprintf(f, "]}\n");
  std::fclose(f);
}

extern "C" perch_status perch_search(perch_ctx* c, const perch_search_opts* opts,
                                     perch_result* out) {
  if (!c || !opts || !out) return fail(PERCH_E_ARG, "null argument");
  if (opts->mode < PERCH_SEARCH_EXHAUSTIVE || opts->mode > PERCH_SEARCH_LEARNED_MHA)
    return fail(PERCH_E_ARG, "unknown search mode %d", opts->mode);
  if (opts->n_priors < 0 || (opts->n_priors > 0 && !opts->priors))
    return fail(PERCH_E_ARG, "bad pose priors");
  if (opts->n_priors > 0 && opts->mode != PERCH_SEARCH_MHA)
    return fail(PERCH_E_ARG, "pose priors are a queue of the multi-heuristic search");
  if (opts->mode >= PERCH_SEARCH_FOCAL && !(opts->w >= 1.0f))
    return fail(PERCH_E_ARG, "focal, learned and multi-heuristic searches need w >= 1");
  Searcher s(c, opts);
  perch_status st = s.init();
  if (st) return st;

  Range r("perch_search");
  if (opts->mode == PERCH_SEARCH_EXHAUSTIVE)
    st = s.exhaustive();
  else if (opts->mode == PERCH_SEARCH_LEARNED || opts->mode == PERCH_SEARCH_LEARNED_MHA)
    st = s.learned(opts->mode == PERCH_SEARCH_LEARNED_MHA);
  else if (opts->mode == PERCH_SEARCH_MHA)
    st = s.best_first(opts->n_priors > 0 ? 3 : 2);
  else
    st = s.best_first(opts->mode == PERCH_SEARCH_FOCAL ? 1 : 0);
  r.end();
  s.trace(true);  // the trace's last entry: the state the search ends in
  s.fill(out);
  log_search(opts, *out, st);
  if (st == PERCH_E_BUDGET) return fail(PERCH_E_BUDGET, "search budget exhausted");
  return st;
}
