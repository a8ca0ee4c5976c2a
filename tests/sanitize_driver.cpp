// Host set-up code of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_host_sanitizers.py with g++,
// no GPU code): the matrix checks (good and bad inputs), both partitioners,
// the interface structure, the local orderings and the nested-dissection
// layout of the interface system, on TPFA-like M-matrices of 3-D grids, with
// several host threads.  Prints one line per case; exits nonzero on an
// unexpected status (the sanitizers abort on their own findings).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "am_host.h"

using namespace am;

namespace {

struct Grid {
  int64_t n = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
  HostCSR csr() const { return HostCSR{n, (int64_t)ci.size(), rp.data(), ci.data(), v.data()}; }
};

// 7-point M-matrix of an nx x ny x nz grid: random couplings -w (w > 0), the
// diagonal their sum plus a Dirichlet term on the x = 0 face
Grid grid(int nx, int ny, int nz, unsigned seed) {
  std::mt19937 rng(seed);
  std::uniform_real_distribution<double> U(0.1, 10.0);
  const int64_t n = (int64_t)nx * ny * nz;
  std::vector<std::vector<std::pair<int32_t, double>>> rows(n);
  auto id = [&](int i, int j, int k) { return (int32_t)(i + nx * (j + ny * k)); };
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int32_t c = id(i, j, k);
        const int nb[3][3] = {{i + 1, j, k}, {i, j + 1, k}, {i, j, k + 1}};
        for (auto& q : nb)
          if (q[0] < nx && q[1] < ny && q[2] < nz) {
            const int32_t o = id(q[0], q[1], q[2]);
            const double w = U(rng);
            rows[c].emplace_back(o, -w);
            rows[o].emplace_back(c, -w);
          }
      }
  Grid g;
  g.n = n;
  g.rp.assign(n + 1, 0);
  for (int64_t c = 0; c < n; ++c) {
    double d = (c % nx == 0) ? 2.0 : 0.0;
    for (auto& e : rows[c]) d -= e.second;
    rows[c].emplace_back((int32_t)c, d);
    std::sort(rows[c].begin(), rows[c].end());
    for (auto& e : rows[c]) {
      g.ci.push_back(e.first);
      g.v.push_back(e.second);
    }
    g.rp[c + 1] = (int64_t)g.ci.size();
  }
  return g;
}

int failures = 0;
void expect(bool ok, const std::string& what) {
  std::printf("%s %s\n", ok ? "ok  " : "FAIL", what.c_str());
  if (!ok) ++failures;
}

void structure_case(const Grid& g, const std::vector<int32_t>& part, int32_t m,
                    const std::string& name) {
  const HostCSR A = g.csr();
  std::string err;
  Structure st;
  expect(build_structure(A, part.data(), m, AM_MORTAR_PER_INTERFACE, st, err) == AM_OK,
         name + ": structure (" + std::to_string(st.n_iface()) + " interfaces)");
  LocalPlan lp;
  const am_status ps = plan_local(A, st, lp, err);
  expect(ps == AM_OK || ps == AM_ERR_UNSUPPORTED, name + ": local orderings");
  if (st.n_iface() > 0)
    for (int64_t rows : {64, 496, 4096}) {
      IfaceND nd;
      const am_status s = build_iface_nd(st, rows, 1.15, nd, err);
      expect(s == AM_OK || s == AM_ERR_UNSUPPORTED,
             name + ": dissection, blocks of at most " + std::to_string(rows) + " rows");
      if (s == AM_OK) expect((int64_t)nd.order.size() == st.n_iface(), name + ": dissection order size");
    }
  Structure se;
  expect(build_structure(A, part.data(), m, AM_MORTAR_PER_EDGE, se, err) == AM_OK,
         name + ": per-edge structure");
}

}  // namespace

int main() {
  for (int t : {1, 3, 16}) {
    setenv("ALGMORTAR_HOST_THREADS", std::to_string(t).c_str(), 1);
    const std::string th = " [" + std::to_string(t) + " threads]";
    const Grid g = grid(24, 16, 12, 7);
    const HostCSR A = g.csr();
    std::string err;
    expect(validate_csr(A, err) == AM_OK, "validate" + th);
    std::vector<int32_t> part(g.n);
    int32_t m = 0;
    expect(partition_blocks(24, 16, 12, 8, 8, 4, part.data(), &m, err) == AM_OK, "blocks" + th);
    expect(validate_partition(g.n, part.data(), m, err) == AM_OK, "block partition valid" + th);
    structure_case(g, part, m, "blocks" + th);
    std::vector<int32_t> bp(g.n);
    int32_t mb = 0;
    expect(partition_bisect(A, 30, 120, 11, bp.data(), &mb, err) == AM_OK, "bisect" + th);
    structure_case(g, bp, mb, "bisect" + th);
    // one subdomain, one-cell subdomains
    std::vector<int32_t> one(g.n, 0);
    structure_case(g, one, 1, "one subdomain" + th);
    std::vector<int32_t> cells(g.n);
    for (int64_t c = 0; c < g.n; ++c) cells[c] = (int32_t)c;
    structure_case(g, cells, (int32_t)g.n, "one-cell subdomains" + th);
    // bad inputs: asymmetric value, positive coupling, broken pattern, bad partition
    Grid b1 = g;
    b1.v[1] *= 0.5;
    expect(validate_csr(b1.csr(), err) == AM_ERR_NOT_SYMMETRIC, "asymmetric rejected" + th);
    Grid b2 = g;
    for (int64_t c = 0; c < b2.n && b2.ci[b2.rp[c]] == c; ++c) {}
    b2.v[g.rp[5]] = std::fabs(b2.v[g.rp[5]]);
    b2.v[g.rp[5] + 1] = std::fabs(b2.v[g.rp[5] + 1]);
    expect(validate_csr(b2.csr(), err) != AM_OK, "changed entries rejected" + th);
    Grid b3 = g;
    std::swap(b3.ci[3], b3.ci[4]);
    expect(validate_csr(b3.csr(), err) == AM_ERR_ARG, "unsorted columns rejected" + th);
    std::vector<int32_t> bad(part);
    bad[7] = m + 3;
    expect(validate_partition(g.n, bad.data(), m, err) == AM_ERR_ARG, "out-of-range part rejected" + th);
    expect(partition_blocks(24, 16, 12, 7, 8, 4, part.data(), &m, err) == AM_ERR_ARG,
           "non-dividing block rejected" + th);
  }
  std::printf("%d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
