// Host-side structure of AlgMortar: validation, partitioners, permutation,
// interface edge sets and mortar numbering (paper Sec. 3.1-3.2), and the
// device-oriented layout plan derived from them.  Plain C++17, no HIP.
#pragma once

#include <algorithm>

#include <atomic>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

#include "algmortar.h"

namespace am {

// Host threads for the set-up loops: ALGMORTAR_HOST_THREADS if set, else the
// hardware threads, at most 16.
int host_threads();

// Runs f(i) for every i in [0, n) on up to host_threads() threads (the
// caller's included), handing out chunks of `grain` indices in increasing
// order.  f must write only data that belongs to its own index; results are
// then independent of the thread count and the schedule.
template <typename F>
void parallel_for(int64_t n, int64_t grain, F&& f) {
  const int nt = (int)std::min<int64_t>(host_threads(), (n + grain - 1) / grain);
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int64_t> next{0};
  auto work = [&]() {
    for (;;) {
      const int64_t lo = next.fetch_add(grain);
      if (lo >= n) return;
      const int64_t hi = std::min(n, lo + grain);
      for (int64_t i = lo; i < hi; ++i) f(i);
    }
  };
  std::vector<std::thread> pool;
  pool.reserve(nt - 1);
  for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
}

struct HostCSR {
  int64_t n = 0, nnz = 0;
  const int64_t* rp = nullptr;
  const int32_t* ci = nullptr;
  const double* v = nullptr;
};

// Validates pattern (monotone row_ptr, strictly ascending in-range columns),
// finiteness, bitwise symmetry of values (a missing transpose counts as 0)
// and the sign of every off-diagonal (< 0 or an explicit zero).
am_status validate_csr(const HostCSR& A, std::string& err);
am_status validate_partition(int64_t n, const int32_t* part, int32_t nparts, std::string& err);

struct Structure {
  int64_t n = 0;
  int32_t m = 0;
  std::vector<int32_t> part;      // [n]
  std::vector<int32_t> perm;      // [n] perm[new] = old (ascending inside a part)
  std::vector<int64_t> sub_ptr;   // [m+1]
  std::vector<int32_t> edge_k, edge_l;  // [|E|] original indices, k in the lower part
  std::vector<double> edge_a;           // [|E|] a_kl
  std::vector<int64_t> iface_ptr;       // [NL+1]
  std::vector<int32_t> iface_ij;        // [2 NL]
  std::vector<int64_t> isub_ptr;        // [m+1]   I_i as CSR
  std::vector<int32_t> isub_list;       // [2 NL]  ascending basis ids per part
  int64_t n_iface() const { return (int64_t)iface_ptr.size() - 1; }
  int64_t n_edges() const { return (int64_t)edge_k.size(); }
};

am_status build_structure(const HostCSR& A, const int32_t* part, int32_t nparts, int mortar,
                          Structure& st, std::string& err);

am_status partition_blocks(int32_t nx, int32_t ny, int32_t nz, int32_t bx, int32_t by,
                           int32_t bz, int32_t* part, int32_t* nparts, std::string& err);
am_status partition_bisect(const HostCSR& A, int32_t lo, int32_t hi, uint64_t seed,
                           int32_t* part, int32_t* nparts, std::string& err);

uint64_t splitmix64(uint64_t x);

// Band layout of the local factors.  Inside every subdomain the device uses
// an ordering (identity or reverse Cuthill-McKee, whichever has the smaller
// bandwidth) and a window width Wp = 64 * ceil(bandwidth / 64).
struct LocalPlan {
  std::vector<int32_t> dperm;      // [n] device order: dperm[new] = old
  std::vector<int32_t> dpos;       // [n] inverse: dpos[old] = new
  std::vector<int32_t> wp;         // [m] window width per subdomain
  std::vector<int64_t> roff;       // [m+1] padded row offsets (rows padded to a multiple of 64)
  std::vector<int64_t> fac_off;    // [m+1] offsets (elements) of Lc / Lr blocks = roff * wp
  int32_t max_wp = 64;
  int32_t max_ni = 0;              // max |I_i|
  int32_t max_sub = 0;             // max subdomain size
};

am_status plan_local(const HostCSR& A, const Structure& st, LocalPlan& lp, std::string& err);

// Nested-dissection layout of the interface system (iface_nd.cpp): the basis
// functions in an order where the first nrows form nblk mutually uncoupled
// diagonal blocks of S and the last ntop are the separators above them.
struct IfaceND {
  int32_t depth = 0;              // dissection levels above the blocks
  int32_t nblk = 0;
  int64_t nrows = 0;              // rows in blocks
  int64_t ntop = 0;               // separator ("top") rows
  std::vector<int32_t> order;     // [NL] ND position -> basis function
  std::vector<int64_t> blk_off;   // [nblk+1] ND positions of the blocks
  std::vector<int64_t> pad_off;   // [nblk+1] positions with every block padded to 64 rows;
                                  // pad_off[nblk] is where the top rows start
  int64_t ld = 0;                 // padded dimension, a multiple of 64
  std::vector<int64_t> t_ptr;     // [ntop+1] per top row ..
  std::vector<int64_t> t_pos;     // .. the ND positions (< nrows) of the block rows it couples to
  std::vector<int64_t> b_ptr;     // [nrows+1] per block row ..
  std::vector<int64_t> b_top;     // .. the top indices (ND position - nrows) it couples to
};

// Builds the layout from the interface structure; blocks have at most
// max_rows rows and the padded dimension is at most max_growth times that of
// S (the depth minimises the bytes of one solve under these limits).
// AM_ERR_UNSUPPORTED when no depth meets the limits.
am_status build_iface_nd(const Structure& st, int64_t max_rows, double max_growth, IfaceND& nd,
                         std::string& err);

}  // namespace am
