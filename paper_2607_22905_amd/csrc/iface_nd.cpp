// Nested-dissection layout of the interface system (host, set-up only).
//
// S[n][m] is nonzero exactly when the basis functions n and m share a
// subdomain (eq. interface-problem-alg: the MBF of m lives on its two
// subdomains, the edges of E_n touch the two subdomains of n).  Cutting the
// subdomain graph into two sets of subdomains therefore splits the basis
// functions into three groups: those with both subdomains on the left, those
// with both on the right (no coupling between these two), and the separator
// (one subdomain on each side).  Repeating the cut on each side for D levels
// gives up to 2^D mutually uncoupled diagonal blocks plus the separators of
// the levels above ("top" rows).  With S = [S_BB S_BT; S_TB S_TT] in that
// order, S_BB is block diagonal, and
//   eta_T = C^{-1} (b_T - S_TB S_BB^{-1} b_B),  C = S_TT - S_TB S_BB^{-1} S_BT
//   eta_B = S_BB^{-1} (b_B - S_BT eta_T)
// (block elimination; in this order C^{-1} is the bottom-right block of
// S^{-1}).  The depth is chosen to minimise the bytes that one solve reads:
// two passes over the block inverses and one over C^{-1} (one pass over the
// blocks when there are no top rows).
#include <algorithm>
#include <cstdint>
#include <deque>
#include <limits>
#include <numeric>
#include <string>
#include <vector>

#include "am_host.h"

namespace am {

namespace {

struct Graph {
  std::vector<std::vector<int32_t>> adj;  // subdomain adjacency (sorted, unique)
};

// BFS distances from `start` inside the subdomain set marked `in` (-1 when
// unreachable); neighbours are visited in ascending order.
void bfs(const Graph& g, const std::vector<char>& in, int32_t start, std::vector<int32_t>& dist,
         const std::vector<int32_t>& subs) {
  for (int32_t s : subs) dist[s] = -1;
  std::deque<int32_t> q;
  dist[start] = 0;
  q.push_back(start);
  while (!q.empty()) {
    const int32_t u = q.front();
    q.pop_front();
    for (int32_t v : g.adj[u])
      if (in[v] && dist[v] < 0) {
        dist[v] = dist[u] + 1;
        q.push_back(v);
      }
  }
}

// farthest subdomain from the last BFS (ties: smallest id)
int32_t farthest(const std::vector<int32_t>& dist, const std::vector<int32_t>& subs) {
  int32_t best = subs[0], bd = -2;
  for (int32_t s : subs)
    if (dist[s] > bd) {
      bd = dist[s];
      best = s;
    }
  return best;
}

struct Node {
  int depth = 0;
  bool leaf = false;
  int child[2] = {-1, -1};
  std::vector<int32_t> sep;  // separator interfaces (internal nodes) or all interfaces (leaves)
};

class Dissector {
 public:
  Dissector(const Structure& st, const Graph& g)
      : st_(st), g_(g), in_(st.m, 0), left_(st.m, 0), du_(st.m), dv_(st.m) {}

  // interfaces with both subdomains in `subs` are `ifs` (ascending)
  int build(const std::vector<int32_t>& subs, const std::vector<int32_t>& ifs, int depth) {
    const int id = (int)nodes_.size();
    nodes_.emplace_back();
    nodes_[id].depth = depth;
    if ((int64_t)ifs.size() <= kLeafRows || subs.size() < 2) {
      nodes_[id].leaf = true;
      nodes_[id].sep = ifs;
      return id;
    }
    std::vector<int32_t> lsubs, rsubs;
    split(subs, ifs, lsubs, rsubs);
    for (int32_t s : subs) left_[s] = 0;
    for (int32_t s : lsubs) left_[s] = 1;
    std::vector<int32_t> L, R, S;
    for (int32_t n : ifs) {
      const bool a = left_[st_.iface_ij[2 * (size_t)n]] != 0, b = left_[st_.iface_ij[2 * (size_t)n + 1]] != 0;
      (a && b ? L : (!a && !b ? R : S)).push_back(n);
    }
    for (int32_t s : subs) left_[s] = 0;
    nodes_[id].sep = S;
    const int c0 = build(lsubs, L, depth + 1);
    const int c1 = build(rsubs, R, depth + 1);
    nodes_[id].child[0] = c0;
    nodes_[id].child[1] = c1;
    return id;
  }

  std::vector<Node> nodes_;
  static constexpr int64_t kLeafRows = 32;

 private:
  // Candidate cuts, keeping the one with the fewest separator interfaces
  // (first candidate on ties): contiguous subdomain-id ranges cut at 40 .. 60
  // percent (subdomains numbered by a recursive partitioner keep its cuts),
  // and orderings by d_u - d_v for the end u of a double BFS and several
  // v (the farthest subdomain from u, and the subdomains of least degree,
  // typically the corners of a box of subdomains), cut in half.
  void split(const std::vector<int32_t>& subs, const std::vector<int32_t>& ifs,
             std::vector<int32_t>& lsubs, std::vector<int32_t>& rsubs) {
    const int64_t n = (int64_t)subs.size();
    for (int32_t s : subs) in_[s] = 1;
    int64_t best = std::numeric_limits<int64_t>::max();
    std::vector<int32_t> best_order;
    int64_t best_cut = n / 2;
    auto consider = [&](const std::vector<int32_t>& order, int64_t cut) {
      if (cut < 1 || cut >= n) return;
      for (int64_t t = 0; t < n; ++t) left_[order[t]] = t < cut ? 1 : 0;
      int64_t sep = 0;
      for (int32_t f : ifs)
        sep += left_[st_.iface_ij[2 * (size_t)f]] != left_[st_.iface_ij[2 * (size_t)f + 1]];
      for (int32_t s : subs) left_[s] = 0;
      if (sep < best) {
        best = sep;
        best_order = order;
        best_cut = cut;
      }
    };
    for (int frac = 40; frac <= 60; frac += 2) consider(subs, n * frac / 100);
    bfs(g_, in_, subs[0], du_, subs);
    const int32_t u = farthest(du_, subs);
    bfs(g_, in_, u, du_, subs);
    std::vector<int32_t> cands{farthest(du_, subs)};
    int mindeg = std::numeric_limits<int>::max();
    std::vector<int> deg(subs.size());
    for (size_t t = 0; t < subs.size(); ++t) {
      int c = 0;
      for (int32_t v : g_.adj[subs[t]]) c += in_[v];
      deg[t] = c;
      mindeg = std::min(mindeg, c);
    }
    for (size_t t = 0; t < subs.size() && cands.size() < 9; ++t)
      if (deg[t] == mindeg && subs[t] != u && subs[t] != cands[0]) cands.push_back(subs[t]);
    const int64_t kFar = (int64_t)1 << 40;
    std::vector<int64_t> key(st_.m);
    for (int32_t v : cands) {
      bfs(g_, in_, v, dv_, subs);
      for (int32_t s : subs)
        key[s] = du_[s] < 0 ? kFar : (int64_t)du_[s] - (dv_[s] < 0 ? 0 : dv_[s]);
      std::vector<int32_t> order(subs);
      std::stable_sort(order.begin(), order.end(),
                       [&](int32_t a, int32_t b) { return key[a] < key[b]; });
      consider(order, n / 2);
    }
    for (int32_t s : subs) in_[s] = 0;
    lsubs.assign(best_order.begin(), best_order.begin() + best_cut);
    rsubs.assign(best_order.begin() + best_cut, best_order.end());
    std::sort(lsubs.begin(), lsubs.end());
    std::sort(rsubs.begin(), rsubs.end());
  }

  const Structure& st_;
  const Graph& g_;
  std::vector<char> in_, left_;
  std::vector<int32_t> du_, dv_;
};

int64_t pad64(int64_t x) { return (x + 63) / 64 * 64; }

// all interfaces of the subtree of node id, in postorder
void collect(const std::vector<Node>& nodes, int id, std::vector<int32_t>& out) {
  const Node& nd = nodes[id];
  if (!nd.leaf) {
    collect(nodes, nd.child[0], out);
    collect(nodes, nd.child[1], out);
  }
  out.insert(out.end(), nd.sep.begin(), nd.sep.end());
}

// blocks at depth D (or leaves above it) and separators above D
void cut_at(const std::vector<Node>& nodes, int id, int D, std::vector<int>& blocks,
            std::vector<int>& seps) {
  const Node& nd = nodes[id];
  if (nd.leaf || nd.depth == D) {
    blocks.push_back(id);
    return;
  }
  cut_at(nodes, nd.child[0], D, blocks, seps);
  cut_at(nodes, nd.child[1], D, blocks, seps);
  seps.push_back(id);  // postorder
}

}  // namespace

am_status build_iface_nd(const Structure& st, int64_t max_rows, double max_growth, IfaceND& nd,
                         std::string& err) {
  nd = IfaceND{};
  const int64_t NL = st.n_iface();
  if (NL <= 0) {
    err = "no interfaces";
    return AM_ERR_ARG;
  }
  Graph g;
  g.adj.assign(st.m, {});
  for (int64_t f = 0; f < NL; ++f) {
    const int32_t i = st.iface_ij[2 * f], j = st.iface_ij[2 * f + 1];
    g.adj[i].push_back(j);
    g.adj[j].push_back(i);
  }
  for (auto& a : g.adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  std::vector<int32_t> subs(st.m), ifs(NL);
  std::iota(subs.begin(), subs.end(), 0);
  std::iota(ifs.begin(), ifs.end(), 0);
  Dissector dis(st, g);
  dis.build(subs, ifs, 0);
  const std::vector<Node>& nodes = dis.nodes_;
  int maxd = 0;
  for (const Node& x : nodes) maxd = std::max(maxd, x.depth);

  // depth with the fewest bytes per solve: 2 sum s_b^2 + R ldC (entries),
  // blocks of at most max_rows rows, padded dimension within max_growth
  int bestD = -1;
  double best = 0.0;
  for (int D = 0; D <= maxd; ++D) {
    std::vector<int> blocks, seps;
    cut_at(nodes, 0, D, blocks, seps);
    int64_t R = 0;
    for (int s : seps) R += (int64_t)nodes[s].sep.size();
    double bytes = 0.0;
    int64_t padded = 0, smax = 0;
    for (int b : blocks) {
      std::vector<int32_t> rows;
      collect(nodes, b, rows);
      const int64_t s = (int64_t)rows.size();
      smax = std::max(smax, s);
      bytes += 2.0 * (double)s * (double)s;
      padded += pad64(s);
    }
    if (R > 0)
      bytes += (double)R * (double)pad64(R);
    else
      bytes *= 0.5;
    padded = pad64(padded + R);
    if (smax > max_rows || (double)padded > max_growth * (double)pad64(NL)) continue;
    if (bestD < 0 || bytes < best) {
      best = bytes;
      bestD = D;
    }
  }
  if (bestD < 0) {
    err = "no nested-dissection depth keeps the interface blocks within " + std::to_string(max_rows) +
          " rows";
    return AM_ERR_UNSUPPORTED;
  }
  std::vector<int> blocks, seps;
  cut_at(nodes, 0, bestD, blocks, seps);
  nd.depth = bestD;
  nd.blk_off.push_back(0);
  nd.pad_off.push_back(0);
  for (int b : blocks) {
    std::vector<int32_t> rows;
    collect(nodes, b, rows);
    if (rows.empty()) continue;  // a side with no interfaces of its own
    nd.order.insert(nd.order.end(), rows.begin(), rows.end());
    nd.blk_off.push_back((int64_t)nd.order.size());
    nd.pad_off.push_back(nd.pad_off.back() + pad64((int64_t)rows.size()));
  }
  nd.nblk = (int32_t)nd.blk_off.size() - 1;
  nd.nrows = (int64_t)nd.order.size();
  for (int s : seps) nd.order.insert(nd.order.end(), nodes[s].sep.begin(), nodes[s].sep.end());
  nd.ntop = (int64_t)nd.order.size() - nd.nrows;
  nd.ld = pad64(nd.pad_off.back() + nd.ntop);
  if ((int64_t)nd.order.size() != NL) {
    err = "internal: nested dissection lost interfaces";
    return AM_ERR_ARG;
  }
  // couplings between the top rows and the block rows: S[n][m] != 0 when n
  // and m share a subdomain
  std::vector<int64_t> pos(NL);  // interface -> ND position
  for (int64_t p = 0; p < NL; ++p) pos[nd.order[p]] = p;
  auto coupled = [&](int32_t f, auto&& take) {
    for (int side = 0; side < 2; ++side) {
      const int32_t s = st.iface_ij[2 * (size_t)f + side];
      for (int64_t q = st.isub_ptr[s]; q < st.isub_ptr[s + 1]; ++q) take(st.isub_list[q]);
    }
  };
  std::vector<int64_t> tmp;
  nd.t_ptr.assign(1, 0);
  for (int64_t t = 0; t < nd.ntop; ++t) {
    tmp.clear();
    coupled(nd.order[nd.nrows + t], [&](int32_t q) {
      if (pos[q] < nd.nrows) tmp.push_back(pos[q]);
    });
    std::sort(tmp.begin(), tmp.end());
    tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
    nd.t_pos.insert(nd.t_pos.end(), tmp.begin(), tmp.end());
    nd.t_ptr.push_back((int64_t)nd.t_pos.size());
  }
  nd.b_ptr.assign(1, 0);
  for (int64_t r = 0; r < nd.nrows; ++r) {
    tmp.clear();
    coupled(nd.order[r], [&](int32_t q) {
      if (pos[q] >= nd.nrows) tmp.push_back(pos[q] - nd.nrows);
    });
    std::sort(tmp.begin(), tmp.end());
    tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
    nd.b_top.insert(nd.b_top.end(), tmp.begin(), tmp.end());
    nd.b_ptr.push_back((int64_t)nd.b_top.size());
  }
  return AM_OK;
}

}  // namespace am
