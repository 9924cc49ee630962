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
//     best goal, until the incumbent is no worse than the anchor's min g.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <queue>
#include <unordered_map>
#include <vector>

#include "perch_ctx.h"

using namespace perch;

namespace {

using Clock = std::chrono::steady_clock;

struct Node {
  int64_t g;
  int32_t j;
  int32_t parent;  // node index, -1 for the root
  int32_t edge;    // cost of the edge from the parent
  perch_object objs[8];  // insertion order
  int64_t key[8];        // canonical: sorted (mesh << 32 | pose)
};

int64_t pack(int32_t m, int32_t p) { return ((int64_t)m << 32) | (uint32_t)p; }

void make_key(Node& n) {
  for (int k = 0; k < n.j; ++k) n.key[k] = pack(n.objs[k].mesh_id, n.objs[k].pose_idx);
  std::sort(n.key, n.key + n.j);
}

int cmp_key(const Node& a, const Node& b) {
  for (int k = 0; k < a.j && k < b.j; ++k)
    if (a.key[k] != b.key[k]) return a.key[k] < b.key[k] ? -1 : 1;
  return a.j == b.j ? 0 : (a.j < b.j ? -1 : 1);
}

struct KeyHash {
  const std::vector<Node>* nodes;
  size_t operator()(int id) const {
    const Node& n = (*nodes)[id];
    uint64_t h = 1469598103934665603ull ^ (uint64_t)n.j;
    for (int k = 0; k < n.j; ++k) {
      h ^= (uint64_t)n.key[k];
      h *= 1099511628211ull;
    }
    return (size_t)h;
  }
};
struct KeyEq {
  const std::vector<Node>* nodes;
  bool operator()(int a, int b) const { return cmp_key((*nodes)[a], (*nodes)[b]) == 0; }
};

struct Child {
  int32_t mesh, pose, cost;
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
    const size_t cap = (size_t)distinct * poses_.size();
    HIP_TRY(c_->s_cands.ensure(cap * sizeof(int2)));
    HIP_TRY(c_->s_out.ensure(cap * 2 * sizeof(int32_t)));
    HIP_TRY(c_->s_hcands.ensure(cap * sizeof(int2)));
    HIP_TRY(c_->s_hout.ensure(cap * 2 * sizeof(int32_t)));
    t0_ = Clock::now();
    return PERCH_OK;
  }

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
      auto it = std::find(left.begin(), left.end(), n.objs[k].mesh_id);
      if (it != left.end()) left.erase(it);
    }
    std::sort(left.begin(), left.end());
    left.erase(std::unique(left.begin(), left.end()), left.end());
    return left;
  }

  // Materialises n on the GPU and evaluates every child; valid ones go to out.
  perch_status expand(const Node& n, std::vector<Child>& out) {
    out.clear();
    const std::vector<int> rest = remaining(n);
    const int P = (int)poses_.size();
    const int cnt = (int)rest.size() * P;
    int2* hc = c_->s_hcands.as<int2>();
    for (size_t a = 0; a < rest.size(); ++a)
      for (int b = 0; b < P; ++b) hc[a * P + b] = make_int2(rest[a], poses_[b]);
    HIP_TRY(hipMemcpyAsync(c_->s_cands.p, hc, cnt * sizeof(int2), hipMemcpyHostToDevice,
                           c_->stream));
    perch_status st = perch_set_parent(c_, n.objs, n.j);
    if (st) return st;
    int32_t* dcost = c_->s_out.as<int32_t>();
    int32_t* dstat = dcost + cnt;
    st = perch_eval_children(c_, reinterpret_cast<const perch_object*>(c_->s_cands.p), cnt, dcost,
                             dstat, nullptr);
    if (st) return st;
    int32_t* hout = c_->s_hout.as<int32_t>();
    HIP_TRY(hipMemcpyAsync(hout, dcost, 2 * (size_t)cnt * sizeof(int32_t), hipMemcpyDeviceToHost,
                           c_->stream));
    HIP_TRY(hipStreamSynchronize(c_->stream));
    ++n_expanded_;
    n_evaluated_ += cnt;
    for (int i = 0; i < cnt; ++i) {
      const int s = hout[cnt + i];
      if (s == 1)
        out.push_back({hc[i].x, hc[i].y, hout[i]});
      else if (s == 0)
        ++n_invalid_;
      else
        return fail(PERCH_E_UNSUPPORTED, "successor (%d, %d) failed with status %d", hc[i].x,
                    hc[i].y, s);
    }
    return PERCH_OK;
  }

  Node child_of(const Node& n, int32_t id, const Child& ch) const {
    Node m;
    std::memset(&m, 0, sizeof(m));
    m.j = n.j + 1;
    m.g = n.g + ch.cost;
    m.parent = id;
    m.edge = ch.cost;
    std::memcpy(m.objs, n.objs, sizeof(perch_object) * n.j);
    m.objs[n.j].mesh_id = ch.mesh;
    m.objs[n.j].pose_idx = ch.pose;
    make_key(m);
    return m;
  }

  void offer_goal(const Node& g, const std::vector<Node>* store) {
    if (have_ && (g.g > best_.g || (g.g == best_.g && cmp_key(g, best_) >= 0))) return;
    const bool cost_improved = !have_ || g.g < best_.g;
    have_ = true;
    best_ = g;
    if (cost_improved) t_best_ = elapsed();
    // edge costs along the path
    std::memset(best_edges_, 0, sizeof(best_edges_));
    if (store) {
      best_edges_[g.j - 1] = g.edge;
      for (int id = g.parent, k = g.j - 2; id >= 0 && k >= 0; id = (*store)[id].parent, --k)
        best_edges_[k] = (*store)[id].edge;
    }
  }

  // ---- exhaustive ----
  perch_status exhaustive() {
    Node root;
    std::memset(&root, 0, sizeof(root));
    root.parent = -1;
    path_edges_.assign(K_, 0);
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
      if (m.j == K_) {
        const bool better = !have_ || m.g < best_.g || (m.g == best_.g && cmp_key(m, best_) < 0);
        offer_goal(m, nullptr);
        if (better) std::copy(path_edges_.begin(), path_edges_.end(), best_edges_);
      } else {
        st = dfs(m);
        if (st) return st;
      }
    }
    return PERCH_OK;
  }

  // ---- uniform-cost and focal ----
  perch_status best_first(bool focal) {
    std::vector<Node> nodes;
    nodes.reserve(1 << 16);
    Node root;
    std::memset(&root, 0, sizeof(root));
    root.parent = -1;
    nodes.push_back(root);
    std::unordered_map<int, int, KeyHash, KeyEq> table(1024, KeyHash{&nodes}, KeyEq{&nodes});
    table.emplace(0, 0);
    std::vector<char> closed(1, 0);
    auto g_less = [&](int a, int b) {  // priority: smaller g, deeper, smaller key
      const Node &x = nodes[a], &y = nodes[b];
      if (x.g != y.g) return x.g > y.g;
      if (x.j != y.j) return x.j < y.j;
      return cmp_key(x, y) > 0;
    };
    std::priority_queue<int, std::vector<int>, decltype(g_less)> open(g_less);
    // focal heap: deeper first (h_depth = K - |s|), then smaller g, then key
    auto d_less = [&](int a, int b) {
      const Node &x = nodes[a], &y = nodes[b];
      if (x.j != y.j) return x.j < y.j;
      if (x.g != y.g) return x.g > y.g;
      return cmp_key(x, y) > 0;
    };
    std::priority_queue<int, std::vector<int>, decltype(d_less)> focal_q(d_less);
    // states waiting for the focal bound, ordered by g
    std::priority_queue<int, std::vector<int>, decltype(g_less)> pending(g_less);
    open.push(0);
    if (focal) pending.push(0);
    std::vector<Child> kids;
    auto live = [&](int id) {
      auto it = table.find(id);
      return it != table.end() && it->second == id && !closed[id];
    };
    const double w = std::max(1.0f, o_.w);
    for (;;) {
      while (!open.empty() && !live(open.top())) open.pop();
      if (open.empty()) break;
      const int64_t gmin = nodes[open.top()].g;
      lower_bound_ = gmin;
      if (have_ && best_.g <= gmin) break;  // incumbent proven optimal
      if (over_budget()) return PERCH_E_BUDGET;
      int pick = -1;
      if (focal) {
        while (!pending.empty() && (double)nodes[pending.top()].g <= w * (double)gmin) {
          if (live(pending.top())) focal_q.push(pending.top());
          pending.pop();
        }
        while (!focal_q.empty() && !live(focal_q.top())) focal_q.pop();
        if (!focal_q.empty() && (expansions_ % 2 == 0 || !o_.anytime)) {
          pick = focal_q.top();
          focal_q.pop();
        }
      }
      if (pick < 0) {
        pick = open.top();
        open.pop();
      }
      ++expansions_;
      Node cur = nodes[pick];
      closed[pick] = 1;
      if (cur.j == K_) {
        offer_goal(cur, &nodes);
        if (!focal || !o_.anytime) break;  // first goal popped / chosen from FOCAL
        continue;
      }
      perch_status st = expand(cur, kids);
      if (st) return st;
      for (const Child& ch : kids) {
        Node m = child_of(cur, pick, ch);
        if (have_ && m.g >= best_.g) continue;  // cannot improve the incumbent
        nodes.push_back(m);
        closed.push_back(0);
        const int id = (int)nodes.size() - 1;
        auto it = table.find(id);
        if (it != table.end()) {
          const int old = it->second;
          if (closed[old] || !(m.g < nodes[old].g)) {
            nodes.pop_back();
            closed.pop_back();
            continue;
          }
          table.erase(it);
        }
        table.emplace(id, id);
        open.push(id);
        if (focal) pending.push(id);
        if (m.j == K_ && focal && o_.anytime) offer_goal(m, &nodes);
      }
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
        r->objs[k] = best_.objs[k];
        r->edge_cost[k] = best_edges_[k];
      }
    } else {
      r->cost = -1;
    }
    r->n_expanded = n_expanded_;
    r->n_evaluated = n_evaluated_;
    r->n_invalid = n_invalid_;
    r->t_total_s = elapsed();
    r->t_best_s = have_ ? t_best_ : -1.0;
    r->lower_bound = lower_bound_;
  }

 private:
  perch_ctx* c_;
  perch_search_opts o_;
  int K_ = 0;
  std::vector<int> poses_;
  Clock::time_point t0_;
  int64_t n_expanded_ = 0, n_evaluated_ = 0, n_invalid_ = 0, expansions_ = 0;
  int64_t lower_bound_ = 0;
  bool have_ = false;
  Node best_{};
  int32_t best_edges_[8] = {0};
  std::vector<int32_t> path_edges_;
  double t_best_ = -1.0;
};

}  // namespace

extern "C" perch_status perch_search(perch_ctx* c, const perch_search_opts* opts,
                                     perch_result* out) {
  if (!c || !opts || !out) return fail(PERCH_E_ARG, "null argument");
  if (opts->mode < PERCH_SEARCH_EXHAUSTIVE || opts->mode > PERCH_SEARCH_FOCAL)
    return fail(PERCH_E_ARG, "unknown search mode %d", opts->mode);
  if (opts->mode == PERCH_SEARCH_FOCAL && !(opts->w >= 1.0f))
    return fail(PERCH_E_ARG, "focal search needs w >= 1");
  Searcher s(c, opts);
  perch_status st = s.init();
  if (st) return st;
  if (opts->mode == PERCH_SEARCH_EXHAUSTIVE)
    st = s.exhaustive();
  else
    st = s.best_first(opts->mode == PERCH_SEARCH_FOCAL);
  s.fill(out);
  if (st == PERCH_E_BUDGET) return fail(PERCH_E_BUDGET, "search budget exhausted");
  return st;
}
