// Host structure of AlgMortar (paper Sec. 3.1-3.2): validation of A and of
// the partition, the two deterministic partitioners, the permutation P, the
// interface edge sets E_ij with their consistent ordering, the mortar
// numbering and I_i, and the local band-ordering plan used by the device.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <tuple>

#include "am_host.h"

namespace am {

static bool find_entry(const HostCSR& A, int64_t row, int32_t col, double* v) {
  const int32_t* b = A.ci + A.rp[row];
  const int32_t* e = A.ci + A.rp[row + 1];
  const int32_t* it = std::lower_bound(b, e, col);
  if (it == e || *it != col) return false;
  *v = A.v[A.rp[row] + (it - b)];
  return true;
}

int host_threads() {
  if (const char* e = std::getenv("ALGMORTAR_HOST_THREADS")) {
    const int v = std::atoi(e);
    if (v >= 1) return std::min(v, 256);
  }
  const unsigned hw = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(hw, 16u));
}

am_status validate_csr(const HostCSR& A, std::string& err) {
  if (A.n <= 0 || A.n > INT32_MAX || !A.rp || !A.ci || !A.v) {
    err = "A: null pointer or n out of range";
    return AM_ERR_ARG;
  }
  if (A.rp[0] != 0 || A.rp[A.n] != A.nnz) {
    err = "A: row_ptr[0] must be 0 and row_ptr[n] must equal nnz";
    return AM_ERR_ARG;
  }
  // Each pass checks rows in parallel; the error reported is that of the
  // lowest failing row, as a row-by-row scan would find it.
  constexpr int64_t kGrain = 4096;
  const int64_t nch = (A.n + kGrain - 1) / kGrain;
  std::vector<int64_t> bad_row(nch, -1);
  std::vector<am_status> bad_code(nch, AM_OK);
  auto first_bad = [&]() -> int64_t {
    for (int64_t c = 0; c < nch; ++c)
      if (bad_row[c] >= 0) return c;
    return -1;
  };
  // pass 1: pattern, finiteness, diagonal
  auto row_ok = [&](int64_t k, am_status& code) -> bool {
    if (A.rp[k + 1] < A.rp[k]) {
      code = AM_ERR_ARG;
      return false;
    }
    bool diag = false;
    for (int64_t p = A.rp[k]; p < A.rp[k + 1]; ++p) {
      const int32_t c = A.ci[p];
      if (c < 0 || c >= A.n || (p > A.rp[k] && c <= A.ci[p - 1]) || !std::isfinite(A.v[p])) {
        code = AM_ERR_ARG;
        return false;
      }
      if (c == k) {
        diag = true;
        if (!(A.v[p] > 0)) {
          code = AM_ERR_NOT_SPD;
          return false;
        }
      }
    }
    if (!diag) {
      code = AM_ERR_NOT_SPD;
      return false;
    }
    return true;
  };
  parallel_for(nch, 1, [&](int64_t c) {
    const int64_t hi = std::min(A.n, (c + 1) * kGrain);
    for (int64_t k = c * kGrain; k < hi; ++k) {
      am_status code = AM_OK;
      if (!row_ok(k, code)) {
        bad_row[c] = k;
        bad_code[c] = code;
        return;
      }
    }
  });
  if (int64_t c = first_bad(); c >= 0) {
    // rebuild the message of the failing row serially
    const int64_t k = bad_row[c];
    if (A.rp[k + 1] < A.rp[k]) {
      err = "A: row_ptr not monotone at row " + std::to_string(k);
      return AM_ERR_ARG;
    }
    bool diag = false;
    for (int64_t p = A.rp[k]; p < A.rp[k + 1]; ++p) {
      const int32_t cc = A.ci[p];
      if (cc < 0 || cc >= A.n || (p > A.rp[k] && cc <= A.ci[p - 1])) {
        err = "A: columns must be in range and strictly ascending (row " + std::to_string(k) + ")";
        return AM_ERR_ARG;
      }
      if (!std::isfinite(A.v[p])) {
        err = "A: non-finite value at row " + std::to_string(k);
        return AM_ERR_ARG;
      }
      if (cc == k) {
        diag = true;
        if (!(A.v[p] > 0)) {
          err = "A: nonpositive diagonal at row " + std::to_string(k);
          return AM_ERR_NOT_SPD;
        }
      }
    }
    if (!diag) {
      err = "A: missing diagonal at row " + std::to_string(k);
      return AM_ERR_NOT_SPD;
    }
    err = "A: invalid row " + std::to_string(k);
    return bad_code[c];
  }
  // pass 2: bitwise symmetry and the sign of the couplings
  std::vector<int64_t> bad_p(nch, -1);
  parallel_for(nch, 1, [&](int64_t c) {
    const int64_t hi = std::min(A.n, (c + 1) * kGrain);
    for (int64_t k = c * kGrain; k < hi; ++k)
      for (int64_t p = A.rp[k]; p < A.rp[k + 1]; ++p) {
        const int32_t cc = A.ci[p];
        if (cc == k) continue;
        double v = A.v[p], t = 0.0;
        if (!find_entry(A, cc, (int32_t)k, &t)) t = 0.0;
        const bool asym = std::memcmp(&v, &t, sizeof(double)) != 0 && !(v == 0.0 && t == 0.0);
        if (asym || v > 0) {
          bad_row[c] = k;
          bad_p[c] = p;
          return;
        }
      }
  });
  if (int64_t c = first_bad(); c >= 0) {
    const int64_t k = bad_row[c], p = bad_p[c];
    const int32_t cc = A.ci[p];
    double v = A.v[p], t = 0.0;
    if (!find_entry(A, cc, (int32_t)k, &t)) t = 0.0;
    if (std::memcmp(&v, &t, sizeof(double)) != 0 && !(v == 0.0 && t == 0.0)) {
      err = "A not symmetric at (" + std::to_string(k) + "," + std::to_string(cc) + ")";
      return AM_ERR_NOT_SYMMETRIC;
    }
    err = "positive off-diagonal at (" + std::to_string(k) + "," + std::to_string(cc) +
          "): interface weights must be negative";
    return AM_ERR_POSITIVE_COUPLING;
  }
  return AM_OK;
}

am_status validate_partition(int64_t n, const int32_t* part, int32_t nparts, std::string& err) {
  if (!part || nparts <= 0 || nparts > n) {
    err = "partition: null pointer or nparts out of range";
    return AM_ERR_ARG;
  }
  std::vector<int64_t> cnt(nparts, 0);
  for (int64_t k = 0; k < n; ++k) {
    if (part[k] < 0 || part[k] >= nparts) {
      err = "partition: id out of range at cell " + std::to_string(k);
      return AM_ERR_ARG;
    }
    cnt[part[k]]++;
  }
  for (int32_t i = 0; i < nparts; ++i)
    if (cnt[i] == 0) {
      err = "partition: subdomain " + std::to_string(i) + " is empty";
      return AM_ERR_ARG;
    }
  return AM_OK;
}

am_status build_structure(const HostCSR& A, const int32_t* part, int32_t nparts, int mortar,
                          Structure& st, std::string& err) {
  if (mortar != AM_MORTAR_PER_INTERFACE && mortar != AM_MORTAR_PER_EDGE) {
    err = "unknown mortar space";
    return AM_ERR_ARG;
  }
  const int64_t n = A.n;
  st.n = n;
  st.m = nparts;
  st.part.assign(part, part + n);
  // permutation: stable counting sort by part (ascending index inside a part)
  st.sub_ptr.assign(nparts + 1, 0);
  for (int64_t k = 0; k < n; ++k) st.sub_ptr[part[k] + 1]++;
  for (int32_t i = 0; i < nparts; ++i) st.sub_ptr[i + 1] += st.sub_ptr[i];
  st.perm.assign(n, 0);
  {
    std::vector<int64_t> fill(st.sub_ptr.begin(), st.sub_ptr.end() - 1);
    for (int64_t k = 0; k < n; ++k) st.perm[fill[part[k]]++] = (int32_t)k;
  }
  // interface edges: stored a_kl != 0 with part[k] < part[l], ordered by
  // (part k, part l, k, l).  Counting sort by part k (rows in index order),
  // then each part's edges sorted by (part l, k, l) on its own; the keys are
  // unique, so the order is that of one sort over all edges.
  struct E { int32_t pk, pl, k, l; double a; };
  auto is_edge = [&](int64_t k, int64_t p) {
    return A.v[p] != 0.0 && part[k] < part[A.ci[p]];
  };
  constexpr int64_t kRows = 4096;
  const int64_t nch = (n + kRows - 1) / kRows;
  std::vector<int64_t> rcnt(n, 0);
  parallel_for(nch, 1, [&](int64_t c) {
    const int64_t hi = std::min(n, (c + 1) * kRows);
    for (int64_t k = c * kRows; k < hi; ++k) {
      int64_t e = 0;
      for (int64_t p = A.rp[k]; p < A.rp[k + 1]; ++p) e += is_edge(k, p) ? 1 : 0;
      rcnt[k] = e;
    }
  });
  std::vector<int64_t> gptr(nparts + 1, 0);
  for (int64_t k = 0; k < n; ++k) gptr[part[k] + 1] += rcnt[k];
  for (int32_t i = 0; i < nparts; ++i) gptr[i + 1] += gptr[i];
  std::vector<int64_t> rpos(n);
  {
    std::vector<int64_t> fill(gptr.begin(), gptr.end() - 1);
    for (int64_t k = 0; k < n; ++k) {
      rpos[k] = fill[part[k]];
      fill[part[k]] += rcnt[k];
    }
  }
  std::vector<E> edges((size_t)gptr[nparts]);
  parallel_for(nch, 1, [&](int64_t c) {
    const int64_t hi = std::min(n, (c + 1) * kRows);
    for (int64_t k = c * kRows; k < hi; ++k) {
      int64_t o = rpos[k];
      for (int64_t p = A.rp[k]; p < A.rp[k + 1]; ++p)
        if (is_edge(k, p)) edges[o++] = {part[k], part[A.ci[p]], (int32_t)k, A.ci[p], A.v[p]};
    }
  });
  parallel_for(nparts, 1, [&](int64_t g) {
    std::sort(edges.begin() + gptr[g], edges.begin() + gptr[g + 1], [](const E& x, const E& y) {
      return std::tie(x.pl, x.k, x.l) < std::tie(y.pl, y.k, y.l);
    });
  });
  const int64_t ne = (int64_t)edges.size();
  st.edge_k.resize(ne);
  st.edge_l.resize(ne);
  st.edge_a.resize(ne);
  st.iface_ptr.clear();
  st.iface_ij.clear();
  for (int64_t e = 0; e < ne; ++e) {
    st.edge_k[e] = edges[e].k;
    st.edge_l[e] = edges[e].l;
    st.edge_a[e] = edges[e].a;
    bool start = (mortar == AM_MORTAR_PER_EDGE) || e == 0 || edges[e].pk != edges[e - 1].pk ||
                 edges[e].pl != edges[e - 1].pl;
    if (start) {
      st.iface_ptr.push_back(e);
      st.iface_ij.push_back(edges[e].pk);
      st.iface_ij.push_back(edges[e].pl);
    }
  }
  st.iface_ptr.push_back(ne);
  const int64_t NL = st.n_iface();
  // I_i: basis functions touching subdomain i, ascending
  st.isub_ptr.assign(nparts + 1, 0);
  for (int64_t q = 0; q < NL; ++q) {
    st.isub_ptr[st.iface_ij[2 * q] + 1]++;
    st.isub_ptr[st.iface_ij[2 * q + 1] + 1]++;
  }
  for (int32_t i = 0; i < nparts; ++i) st.isub_ptr[i + 1] += st.isub_ptr[i];
  st.isub_list.assign(2 * NL, 0);
  {
    std::vector<int64_t> fill(st.isub_ptr.begin(), st.isub_ptr.end() - 1);
    for (int64_t q = 0; q < NL; ++q) {  // q ascending => each list ascending
      st.isub_list[fill[st.iface_ij[2 * q]]++] = (int32_t)q;
      st.isub_list[fill[st.iface_ij[2 * q + 1]]++] = (int32_t)q;
    }
  }
  return AM_OK;
}

am_status partition_blocks(int32_t nx, int32_t ny, int32_t nz, int32_t bx, int32_t by,
                           int32_t bz, int32_t* part, int32_t* nparts, std::string& err) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || bx <= 0 || by <= 0 || bz <= 0 || !part || !nparts) {
    err = "partition_blocks: bad argument";
    return AM_ERR_ARG;
  }
  if (nx % bx || ny % by || nz % bz) {
    err = "partition_blocks: block sizes must divide the grid";
    return AM_ERR_ARG;
  }
  const int64_t mx = nx / bx, my = ny / by;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i)
        part[i + nx * (j + ny * k)] = (int32_t)(i / bx + mx * (j / by + my * (k / bz)));
  *nparts = (int32_t)(mx * my * (nz / bz));
  return AM_OK;
}

uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

namespace {

// Breadth-first hop counts from `src` inside the set whose local ids are
// given by loc[] (>= 0 for members).  dist[t] = -1 for unreachable members.
void bfs(const HostCSR& A, const std::vector<int32_t>& cells, const std::vector<int32_t>& loc,
         int32_t src, std::vector<int32_t>& dist, std::vector<int32_t>& queue) {
  const int32_t ns = (int32_t)cells.size();
  dist.assign(ns, -1);
  queue.clear();
  dist[src] = 0;
  queue.push_back(src);
  for (size_t h = 0; h < queue.size(); ++h) {
    int32_t t = queue[h];
    int64_t g = cells[t];
    for (int64_t p = A.rp[g]; p < A.rp[g + 1]; ++p) {
      int32_t c = A.ci[p];
      if (c == g || A.v[p] == 0.0) continue;
      int32_t lc = loc[c];
      if (lc >= 0 && dist[lc] < 0) {
        dist[lc] = dist[t] + 1;
        queue.push_back(lc);
      }
    }
  }
}

int32_t farthest(const std::vector<int32_t>& d) {
  int32_t best = -1, arg = 0;
  for (int32_t t = 0; t < (int32_t)d.size(); ++t)
    if (d[t] > best) {
      best = d[t];
      arg = t;
    }
  return arg;
}

}  // namespace

am_status partition_bisect(const HostCSR& A, int32_t lo, int32_t hi, uint64_t seed,
                           int32_t* part, int32_t* nparts, std::string& err) {
  if (lo < 1 || hi < 2 * lo || !part || !nparts) {
    err = "partition_bisect: need 1 <= lo and hi >= 2*lo";
    return AM_ERR_ARG;
  }
  const int64_t n = A.n;
  std::vector<int32_t> loc(n, -1);
  std::vector<std::pair<uint64_t, std::vector<int32_t>>> stack;
  std::vector<int32_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  stack.emplace_back(1, std::move(all));
  int32_t np = 0;
  std::vector<int32_t> d0, du, dv, comp, queue;
  while (!stack.empty()) {
    uint64_t node = stack.back().first;
    std::vector<int32_t> cells = std::move(stack.back().second);
    stack.pop_back();
    const int64_t ns = (int64_t)cells.size();
    if (ns <= hi) {
      for (int32_t c : cells) part[c] = np;
      ++np;
      continue;
    }
    for (int64_t t = 0; t < ns; ++t) loc[cells[t]] = (int32_t)t;
    bfs(A, cells, loc, 0, d0, queue);
    int32_t u = farthest(d0);
    bfs(A, cells, loc, u, du, queue);
    int32_t v = farthest(du);
    bfs(A, cells, loc, v, dv, queue);
    std::vector<int64_t> key(ns);
    comp.assign(ns, -1);
    int32_t ncomp = 0;
    for (int64_t t = 0; t < ns; ++t) {
      if (du[t] >= 0) {
        key[t] = (int64_t)du[t] - (int64_t)dv[t];
      } else {
        if (comp[t] < 0) {  // label the component of t (smallest vertex first)
          std::vector<int32_t> dc;
          bfs(A, cells, loc, (int32_t)t, dc, queue);
          for (int32_t w : queue) comp[w] = ncomp;
          ++ncomp;
        }
        key[t] = ((int64_t)1 << 40) + comp[t];
      }
    }
    std::vector<int32_t> order(ns);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return key[a] != key[b] ? key[a] < key[b] : a < b;
    });
    int64_t rho = 40 + (int64_t)(splitmix64(seed ^ node) % 21);
    int64_t cut = std::min(std::max((ns * rho) / 100, (int64_t)lo), ns - lo);
    std::vector<int32_t> left(cut), right(ns - cut);
    for (int64_t t = 0; t < cut; ++t) left[t] = cells[order[t]];
    for (int64_t t = cut; t < ns; ++t) right[t - cut] = cells[order[t]];
    std::sort(left.begin(), left.end());
    std::sort(right.begin(), right.end());
    for (int64_t t = 0; t < ns; ++t) loc[cells[t]] = -1;
    stack.emplace_back(2 * node + 1, std::move(right));
    stack.emplace_back(2 * node, std::move(left));
  }
  *nparts = np;
  return AM_OK;
}

// ---------------------------------------------------------------------------
// Local ordering plan.
namespace {

// Cells of subdomain s are those with part[c] == s; loc[c] is their local
// index (written only for them, so subdomains can be planned concurrently).
int64_t bandwidth(const HostCSR& A, const std::vector<int32_t>& cells,
                  const std::vector<int32_t>& loc, const int32_t* part, int32_t s) {
  int64_t bw = 0;
  for (size_t t = 0; t < cells.size(); ++t) {
    int64_t g = cells[t];
    for (int64_t p = A.rp[g]; p < A.rp[g + 1]; ++p) {
      int32_t c = A.ci[p];
      if (c == g || A.v[p] == 0.0 || part[c] != s) continue;
      bw = std::max<int64_t>(bw, std::abs((int64_t)loc[c] - (int64_t)t));
    }
  }
  return bw;
}

// Reverse Cuthill-McKee of the set `cells` (local graph), components taken
// in order of their smallest member, each started from a pseudo-peripheral
// vertex (farthest from the component's smallest member, ties to the
// smallest degree then index); neighbours enqueued by (degree, index).
std::vector<int32_t> rcm(const HostCSR& A, const std::vector<int32_t>& cells,
                         const std::vector<int32_t>& loc, const int32_t* part, int32_t s) {
  const int32_t ns = (int32_t)cells.size();
  std::vector<int32_t> deg(ns, 0);
  std::vector<std::vector<int32_t>> adj(ns);
  for (int32_t t = 0; t < ns; ++t) {
    int64_t g = cells[t];
    for (int64_t p = A.rp[g]; p < A.rp[g + 1]; ++p) {
      int32_t c = A.ci[p];
      if (c == g || A.v[p] == 0.0 || part[c] != s) continue;
      adj[t].push_back(loc[c]);
    }
    deg[t] = (int32_t)adj[t].size();
  }
  std::vector<int32_t> order;
  std::vector<char> seen(ns, 0);
  std::vector<int32_t> dist(ns, -1), q;
  for (int32_t s0 = 0; s0 < ns; ++s0) {
    if (seen[s0]) continue;
    // BFS from s0 to find the component and a far vertex
    q.clear();
    q.push_back(s0);
    dist[s0] = 0;
    for (size_t h = 0; h < q.size(); ++h)
      for (int32_t w : adj[q[h]])
        if (dist[w] < 0) {
          dist[w] = dist[q[h]] + 1;
          q.push_back(w);
        }
    int32_t start = s0;
    for (int32_t w : q) {
      if (dist[w] > dist[start] || (dist[w] == dist[start] && (deg[w] < deg[start] ||
                                                               (deg[w] == deg[start] && w < start))))
        start = w;
    }
    for (int32_t w : q) dist[w] = -1;
    // Cuthill-McKee from start
    size_t base = order.size();
    order.push_back(start);
    seen[start] = 1;
    for (size_t h = base; h < order.size(); ++h) {
      std::vector<int32_t> nb;
      for (int32_t w : adj[order[h]])
        if (!seen[w]) nb.push_back(w);
      std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
        return deg[a] != deg[b] ? deg[a] < deg[b] : a < b;
      });
      for (int32_t w : nb) {
        seen[w] = 1;
        order.push_back(w);
      }
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

}  // namespace

am_status plan_local(const HostCSR& A, const Structure& st, LocalPlan& lp, std::string& err) {
  const int64_t n = st.n;
  lp.dperm.assign(n, 0);
  lp.dpos.assign(n, 0);
  lp.wp.assign(st.m, 64);
  lp.fac_off.assign(st.m + 1, 0);
  lp.roff.assign(st.m + 1, 0);
  lp.max_wp = 64;
  lp.max_ni = 0;
  lp.max_sub = 0;
  std::vector<int32_t> loc(n, -1);
  std::vector<int64_t> bws(st.m, 0);
  const int32_t* part = st.part.data();
  // each subdomain independently (its own cells of loc, dperm and dpos)
  parallel_for(st.m, 8, [&](int64_t s64) {
    const int32_t s = (int32_t)s64;
    const int64_t b = st.sub_ptr[s], e = st.sub_ptr[s + 1];
    std::vector<int32_t> cells(st.perm.begin() + b, st.perm.begin() + e);
    const int32_t ns = (int32_t)cells.size();
    for (int32_t t = 0; t < ns; ++t) loc[cells[t]] = t;
    const int64_t bw_id = bandwidth(A, cells, loc, part, s);
    std::vector<int32_t> chosen = cells;
    int64_t bw = bw_id;
    if (bw_id > 64) {
      std::vector<int32_t> ord = rcm(A, cells, loc, part, s);
      std::vector<int32_t> rc(ns);
      for (int32_t t = 0; t < ns; ++t) rc[t] = cells[ord[t]];
      for (int32_t t = 0; t < ns; ++t) loc[rc[t]] = t;
      const int64_t bw_rc = bandwidth(A, rc, loc, part, s);
      if (bw_rc < bw_id) {
        chosen = rc;
        bw = bw_rc;
      }
    }
    bws[s] = bw;
    for (int32_t t = 0; t < ns; ++t) {
      lp.dperm[b + t] = chosen[t];
      lp.dpos[chosen[t]] = (int32_t)(b + t);
    }
  });
  for (int32_t s = 0; s < st.m; ++s) {
    const int64_t bw = bws[s];
    const int32_t ns = (int32_t)(st.sub_ptr[s + 1] - st.sub_ptr[s]);
    int32_t wp = 64 * (int32_t)std::max<int64_t>(1, (bw + 63) / 64);
    if (wp > 128) {
      err = "subdomain " + std::to_string(s) + " has local bandwidth " + std::to_string(bw) +
            " > 128 (the band kernels support windows up to 128)";
      return AM_ERR_UNSUPPORTED;
    }
    lp.wp[s] = wp;
    lp.max_wp = std::max(lp.max_wp, wp);
    lp.max_sub = std::max(lp.max_sub, ns);
    lp.max_ni = std::max<int32_t>(lp.max_ni, (int32_t)(st.isub_ptr[s + 1] - st.isub_ptr[s]));
    const int64_t np = ((int64_t)ns + 63) / 64 * 64;
    lp.roff[s + 1] = lp.roff[s] + np;
    lp.fac_off[s + 1] = lp.fac_off[s] + np * wp;
  }
  return AM_OK;
}

}  // namespace am
