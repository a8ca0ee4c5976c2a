// C-ABI of the AlgMortar-PCG library (include/algmortar.h): argument checks,
// the set-up driver (Algorithm 1), the apply (Algorithm 2), the PCG driver
// with hipGraph-captured chunks of iterations, and the differentiation form.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "algmortar.h"
#include "am_device.h"
#include "am_host.h"

using namespace am;

struct am_handle_s {
  std::string err;
  am_options opt{};
  Structure st;
  LocalPlan lp;
  DeviceState d;
  hipStream_t own = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evf[2] = {nullptr, nullptr};  // stop-flag copies of consecutive chunks
  hipEvent_t evp[8] = {};                   // per-launch timing of a profiled solve
  double* tres = nullptr;  // [kMaxNRHS] ||b - Ax||^2
  double* bp = nullptr;    // permuted right-hand side
  // block-Jacobi smoothing (Sec. 5.4): the handle of the plain diagonal
  // blocks, the order maps and the correction buffers (owned here)
  am_handle bj = nullptr;
  SmoothDevice sm;
  std::vector<void*> sm_allocs;
  // the set-up's CSR pattern (checked by algmortar_update_values), the maps
  // of that entry point, and whether the numeric set-up is valid (false
  // after an update whose factorization failed)
  std::vector<int64_t> pat_rp;
  std::vector<int32_t> pat_ci;
  ValueMaps vm;
  bool numeric_ok = true;
};

struct am_tpfa_s {
  std::string err;
  TpfaDevice t;
};

namespace {

thread_local std::string g_err;

am_status fail(am_handle h, am_status s, const std::string& msg) {
  if (h) h->err = msg;
  g_err = msg;
  return s;
}

#define HCHK(expr)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(h, e_ == hipErrorOutOfMemory ? AM_ERR_OOM : AM_ERR_HIP,                  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)

template <class T>
hipError_t dalloc(std::vector<void*>& allocs, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return e;
  allocs.push_back(q);
  *p = (T*)q;
  return hipSuccess;
}

template <class T>
hipError_t upload(std::vector<void*>& allocs, T** p, const T* v, size_t count, hipStream_t s) {
  hipError_t e = dalloc(allocs, p, count);
  if (e != hipSuccess || count == 0) return e;
  e = hipMemcpyAsync(*p, v, count * sizeof(T), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

template <class T>
hipError_t upload(std::vector<void*>& allocs, T** p, const std::vector<T>& v, hipStream_t s) {
  return upload(allocs, p, v.data(), v.size(), s);
}

// host array without the zero fill of std::vector (for large arrays that a
// parallel loop writes in full)
template <class T>
struct HostBuf {
  std::unique_ptr<T[]> p;
  size_t n = 0;
  explicit HostBuf(size_t m) : p(new T[m]), n(m) {}
  T& operator[](size_t i) { return p[i]; }
  const T& operator[](size_t i) const { return p[i]; }
};

int pow2_at_least(int x) {
  int r = 1;
  while (r < x) r *= 2;
  return r;
}

am_status host_csr(const am_csr* A, HostCSR& H, std::vector<double>& vals, am_handle h) {
  if (!A || !A->row_ptr || !A->col_idx || !A->val || A->n <= 0)
    return fail(h, AM_ERR_ARG, "A: null pointer or empty matrix");
  H.n = A->n;
  H.nnz = A->nnz;
  H.rp = A->row_ptr;
  H.ci = A->col_idx;
  if (A->values_on_device) {
    vals.resize((size_t)A->nnz);
    hipError_t e = hipMemcpy(vals.data(), A->val, sizeof(double) * (size_t)A->nnz,
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(h, AM_ERR_HIP, std::string("copy of A values: ") + hipGetErrorString(e));
    H.v = vals.data();
  } else {
    H.v = A->val;
  }
  return AM_OK;
}

}  // namespace

extern "C" {

const char* algmortar_last_error(am_handle h) { return h ? h->err.c_str() : g_err.c_str(); }

// ---------------------------------------------------------------------------
am_status am_partition_blocks(int32_t nx, int32_t ny, int32_t nz, int32_t bx, int32_t by,
                              int32_t bz, int32_t* part, int32_t* nparts) {
  std::string e;
  am_status s = partition_blocks(nx, ny, nz, bx, by, bz, part, nparts, e);
  if (s != AM_OK) g_err = e;
  return s;
}

am_status am_partition_bisect(const am_csr* A, int32_t lo, int32_t hi, uint64_t seed,
                              int32_t* part, int32_t* nparts) {
  if (!A || A->values_on_device) return fail(nullptr, AM_ERR_ARG, "A must be host resident");
  HostCSR H;
  std::vector<double> tmp;
  am_status s = host_csr(A, H, tmp, nullptr);
  if (s != AM_OK) return s;
  std::string e;
  s = validate_csr(H, e);
  if (s != AM_OK) return fail(nullptr, s, e);
  s = partition_bisect(H, lo, hi, seed, part, nparts, e);
  if (s != AM_OK) g_err = e;
  return s;
}

static am_status host_structure(const am_csr* A, const int32_t* part, int32_t nparts,
                                int32_t mortar, Structure& st) {
  if (!A || A->values_on_device) return fail(nullptr, AM_ERR_ARG, "A must be host resident");
  HostCSR H;
  std::vector<double> tmp;
  am_status s = host_csr(A, H, tmp, nullptr);
  if (s != AM_OK) return s;
  std::string e;
  if ((s = validate_csr(H, e)) != AM_OK) return fail(nullptr, s, e);
  if ((s = validate_partition(H.n, part, nparts, e)) != AM_OK) return fail(nullptr, s, e);
  if ((s = build_structure(H, part, nparts, mortar, st, e)) != AM_OK) return fail(nullptr, s, e);
  return AM_OK;
}

am_status am_structure_sizes(const am_csr* A, const int32_t* part, int32_t nparts,
                             int32_t mortar, int64_t* n_iface, int64_t* n_edges) {
  if (!n_iface || !n_edges) return fail(nullptr, AM_ERR_ARG, "null output");
  Structure st;
  am_status s = host_structure(A, part, nparts, mortar, st);
  if (s != AM_OK) return s;
  *n_iface = st.n_iface();
  *n_edges = st.n_edges();
  return AM_OK;
}

static void copy_structure(const Structure& st, int32_t* perm, int64_t* sub_ptr,
                           int64_t* iface_ptr, int32_t* iface_ij, int32_t* edge_k,
                           int32_t* edge_l) {
  if (perm) std::copy(st.perm.begin(), st.perm.end(), perm);
  if (sub_ptr) std::copy(st.sub_ptr.begin(), st.sub_ptr.end(), sub_ptr);
  if (iface_ptr) std::copy(st.iface_ptr.begin(), st.iface_ptr.end(), iface_ptr);
  if (iface_ij) std::copy(st.iface_ij.begin(), st.iface_ij.end(), iface_ij);
  if (edge_k) std::copy(st.edge_k.begin(), st.edge_k.end(), edge_k);
  if (edge_l) std::copy(st.edge_l.begin(), st.edge_l.end(), edge_l);
}

am_status am_structure(const am_csr* A, const int32_t* part, int32_t nparts, int32_t mortar,
                       int32_t* perm, int64_t* sub_ptr, int64_t* iface_ptr, int32_t* iface_ij,
                       int32_t* edge_k, int32_t* edge_l) {
  Structure st;
  am_status s = host_structure(A, part, nparts, mortar, st);
  if (s != AM_OK) return s;
  copy_structure(st, perm, sub_ptr, iface_ptr, iface_ij, edge_k, edge_l);
  return AM_OK;
}

am_status am_interface_nd(const am_csr* A, const int32_t* part, int32_t nparts, int32_t max_nrhs,
                          int32_t* order, int64_t* blk_off, int32_t* nblk, int64_t* ntop) {
  if (!order || !blk_off || !nblk || !ntop || max_nrhs < 1 || max_nrhs > kMaxNRHS)
    return fail(nullptr, AM_ERR_ARG, "bad argument");
  Structure st;
  am_status s = host_structure(A, part, nparts, AM_MORTAR_PER_INTERFACE, st);
  if (s != AM_OK) return s;
  IfaceND nd;
  std::string e;
  s = build_iface_nd(st, nd_max_rows(pow2_at_least(max_nrhs)), 1.15, nd, e);
  if (s != AM_OK) return fail(nullptr, s, e);
  std::copy(nd.order.begin(), nd.order.end(), order);
  std::copy(nd.blk_off.begin(), nd.blk_off.end(), blk_off);
  *nblk = nd.nblk;
  *ntop = nd.ntop;
  return AM_OK;
}

// ---------------------------------------------------------------------------
am_status algmortar_destroy(am_handle h) {
  if (!h) return AM_OK;
  const bool touched = h->own || !h->d.allocs.empty() || h->d.h_flags;
  if (!touched) {  // failed in host validation: no device state to release
    delete h;
    return AM_OK;
  }
  (void)hipSetDevice(h->d.device);
  for (void* p : h->sm_allocs) (void)hipFree(p);
  if (h->bj) algmortar_destroy(h->bj);
  if (h->d.graph) (void)hipGraphExecDestroy(h->d.graph);
  for (hipGraphExec_t g : h->d.graph_short)
    if (g) (void)hipGraphExecDestroy(g);
  for (void* p : h->d.allocs) (void)hipFree(p);
  for (void* p : h->vm.allocs) (void)hipFree(p);
  if (h->d.h_flags) (void)hipHostFree(h->d.h_flags);
  if (h->d.h_sc) (void)hipHostFree(h->d.h_sc);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  for (hipEvent_t e : h->evp)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->evf)
    if (e) (void)hipEventDestroy(e);
  if (h->own) (void)hipStreamDestroy(h->own);
  if (h->d.side) (void)hipStreamDestroy(h->d.side);
  if (h->d.ev_fork) (void)hipEventDestroy(h->d.ev_fork);
  if (h->d.ev_join) (void)hipEventDestroy(h->d.ev_join);
  delete h;
  return AM_OK;
}

// Device arrays of the nested-dissection interface solve from its host
// layout (structure only; nd_numeric fills the values).
static hipError_t nd_upload(DeviceState& d, const IfaceND& ndh, hipStream_t sm) {
  NdDevice& nd = d.nd;
  std::vector<void*>& al = d.allocs;
  const int64_t NL = d.NL;
  nd.nblk = ndh.nblk;
  nd.nrows = ndh.nrows;
  nd.R = (int32_t)ndh.ntop;
  nd.ldC = (int32_t)((ndh.ntop + 63) / 64 * 64);
  nd.ldp = (int32_t)ndh.ld;
  nd.h_blk_off = ndh.blk_off;
  nd.h_pad_off = ndh.pad_off;
  // padded position -> basis function
  nd.h_src.assign((size_t)nd.ldp, -1);
  for (int b = 0; b < nd.nblk; ++b)
    for (int64_t r = ndh.blk_off[b]; r < ndh.blk_off[b + 1]; ++r)
      nd.h_src[ndh.pad_off[b] + (r - ndh.blk_off[b])] = ndh.order[r];
  for (int64_t t = 0; t < ndh.ntop; ++t) nd.h_src[ndh.pad_off[nd.nblk] + t] = ndh.order[nd.nrows + t];
  std::vector<int64_t> inv_off(nd.nblk + 1, 0);
  std::vector<int32_t> wg_blk, wg_row0;
  for (int b = 0; b < nd.nblk; ++b) {
    const int64_t sb = ndh.blk_off[b + 1] - ndh.blk_off[b];
    inv_off[b + 1] = inv_off[b] + sb * sb;
    nd.smax = std::max(nd.smax, sb);
    for (int64_t r0 = 0; r0 < sb; r0 += 64) {
      wg_blk.push_back(b);
      wg_row0.push_back((int32_t)r0);
    }
  }
  nd.nwg = (int32_t)wg_blk.size();
  // row parts of the top product: about 2048 waves, at most what the
  // kernels keep in LDS
  const int64_t cap = nd_max_rows(d.max_nrhs);
  if (nd.R > 0) {
    // (parts of at least 16 rows with one or two right-hand sides, 64 with
    // more: the part sums grow with the columns)
    const int64_t nrb = nd.ldC / 64, minper = d.max_nrhs <= 2 ? 16 : 64;
    int64_t P = std::max<int64_t>(1, std::min<int64_t>((2048 + nrb - 1) / nrb, (nd.R + minper - 1) / minper));
    int64_t per = (nd.R + P - 1) / P;
    if (per > cap) {
      P = (nd.R + cap - 1) / cap;
      per = (nd.R + P - 1) / P;
    }
    nd.P = (int32_t)P;
    nd.per = (int32_t)per;
  }
  std::vector<int32_t> ord(ndh.order.begin(), ndh.order.end());
  std::vector<int32_t> t_pos(ndh.t_pos.begin(), ndh.t_pos.end());
  std::vector<int32_t> b_top(ndh.b_top.begin(), ndh.b_top.end());
  std::vector<int32_t> t_ri(t_pos.size()), t_ci(t_pos.size()), b_ri(b_top.size()), b_ci(b_top.size());
  for (int64_t t = 0; t < ndh.ntop; ++t)
    for (int64_t q = ndh.t_ptr[t]; q < ndh.t_ptr[t + 1]; ++q) {
      t_ri[q] = ord[nd.nrows + t];
      t_ci[q] = ord[ndh.t_pos[q]];
    }
  for (int64_t r = 0; r < nd.nrows; ++r)
    for (int64_t q = ndh.b_ptr[r]; q < ndh.b_ptr[r + 1]; ++q) {
      b_ri[q] = ord[r];
      b_ci[q] = ord[nd.nrows + ndh.b_top[q]];
    }
  nd.nt_pairs = (int64_t)t_pos.size();
  nd.nb_pairs = (int64_t)b_top.size();
  hipError_t e;
#define NDUP(p, v)                              \
  if ((e = upload(al, &(p), (v), sm)) != hipSuccess) return e
  NDUP(nd.ord, ord);
  NDUP(nd.src, nd.h_src);
  NDUP(nd.blk_off, ndh.blk_off);
  NDUP(nd.pad_off, ndh.pad_off);
  NDUP(nd.inv_off, inv_off);
  NDUP(nd.wg_blk, wg_blk);
  NDUP(nd.wg_row0, wg_row0);
  NDUP(nd.t_ptr, ndh.t_ptr);
  NDUP(nd.t_pos, t_pos);
  NDUP(nd.t_ri, t_ri);
  NDUP(nd.t_ci, t_ci);
  NDUP(nd.b_ptr, ndh.b_ptr);
  NDUP(nd.b_top, b_top);
  NDUP(nd.b_ri, b_ri);
  NDUP(nd.b_ci, b_ci);
#undef NDUP
  const int NR = d.max_nrhs;
  if ((e = dalloc(al, &nd.binv, (size_t)inv_off[nd.nblk])) != hipSuccess) return e;
  if ((e = dalloc(al, &nd.cinv, (size_t)nd.R * nd.ldC)) != hipSuccess) return e;
  if ((e = dalloc(al, &nd.t_val, (size_t)nd.nt_pairs)) != hipSuccess) return e;
  if ((e = dalloc(al, &nd.b_val, (size_t)nd.nb_pairs)) != hipSuccess) return e;
  if ((e = dalloc(al, &nd.y1, (size_t)std::max<int64_t>(nd.nrows, 1) * NR)) != hipSuccess) return e;
  if ((e = dalloc(al, &nd.eta2, (size_t)std::max<int32_t>(nd.R, 1) * NR)) != hipSuccess) return e;
  if ((e = dalloc(al, &nd.ypart, (size_t)nd.P * std::max<int32_t>(nd.ldC, 1) * NR)) != hipSuccess) return e;
  (void)NL;
  nd.on = 1;
  return hipSuccess;
}

// Device arrays of the inexact interface solve: the ELL pattern of S (row n
// couples to the basis functions of its two subdomains), the block layout,
// the vectors and partials of the inner PCG.
static hipError_t ix_upload(DeviceState& d, const Structure& st, hipStream_t sm) {
  IxDevice& ix = d.ix;
  std::vector<void*>& al = d.allocs;
  const int64_t NL = d.NL;
  std::vector<std::vector<int32_t>> rows((size_t)NL);
  int32_t w = 1;
  for (int64_t n = 0; n < NL; ++n) {
    auto& v = rows[n];
    for (int side = 0; side < 2; ++side) {
      const int32_t sd = st.iface_ij[2 * n + side];
      for (int64_t q = st.isub_ptr[sd]; q < st.isub_ptr[sd + 1]; ++q) v.push_back(st.isub_list[q]);
    }
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    w = std::max<int32_t>(w, (int32_t)v.size());
  }
  ix.w = w;
  std::vector<int32_t> scol((size_t)w * NL);
  std::vector<int8_t> pad((size_t)w * NL);
  for (int64_t n = 0; n < NL; ++n)
    for (int32_t e = 0; e < w; ++e) {
      const bool real = e < (int32_t)rows[n].size();
      scol[(size_t)e * NL + n] = real ? rows[n][e] : (int32_t)n;
      pad[(size_t)e * NL + n] = real ? 0 : 1;
    }
  ix.nblk = (int32_t)((NL + ix.bs - 1) / ix.bs);
  std::vector<int64_t> inv_off(ix.nblk + 1, 0);
  for (int b = 0; b < ix.nblk; ++b) {
    const int64_t sb = std::min<int64_t>(ix.bs, NL - (int64_t)b * ix.bs);
    inv_off[b + 1] = inv_off[b] + sb * sb;
  }
  hipError_t e;
  if ((e = upload(al, &ix.scol, scol, sm)) != hipSuccess) return e;
  if ((e = upload(al, &ix.pad, pad, sm)) != hipSuccess) return e;
  if ((e = upload(al, &ix.inv_off, inv_off, sm)) != hipSuccess) return e;
  const int NR = d.max_nrhs;
  if ((e = dalloc(al, &ix.sval, (size_t)w * NL)) != hipSuccess) return e;
  if ((e = dalloc(al, &ix.binv, (size_t)inv_off[ix.nblk])) != hipSuccess) return e;
  double** vecs[5] = {&ix.r, &ix.z, &ix.q, &ix.p[0], &ix.p[1]};
  for (double** v : vecs) {
    if ((e = dalloc(al, v, (size_t)NL * NR)) != hipSuccess) return e;
    if ((e = launch_fill(*v, NL * NR, 0.0, sm)) != hipSuccess) return e;
  }
  if ((e = dalloc(al, &ix.pa, (size_t)ix.nblk * NR)) != hipSuccess) return e;
  if ((e = dalloc(al, &ix.pb[0], (size_t)ix.nblk * 2 * NR)) != hipSuccess) return e;
  if ((e = dalloc(al, &ix.pb[1], (size_t)ix.nblk * 2 * NR)) != hipSuccess) return e;
  if ((e = dalloc(al, &ix.sc, kMaxNRHS)) != hipSuccess) return e;
  ix.on = 1;
  return hipSuccess;
}

// Interface factorization (Algorithm 1, last step), on the handle's S: the
// explicit S^{-1} (dense form) or the nested-dissection blocks and C^{-1};
// the temporaries are allocated and freed here.  Synchronizes `st`.
static hipError_t interface_inverse(DeviceState& d, hipStream_t st) {
  if (d.NL <= 0) return hipSuccess;
  const int64_t ld = d.nd.on ? d.nd.ldp : d.ldS;
  const size_t nS = (size_t)ld * ld;
  const int64_t ptiles = trtri_part_tiles((int)(ld / 64));
  double *L = nullptr, *Li = nullptr, *part = nullptr, *Sp = nullptr;
  hipError_t he = hipMalloc((void**)&L, nS * sizeof(double));
  if (he == hipSuccess) he = hipMalloc((void**)&Li, nS * sizeof(double));
  if (he == hipSuccess && ptiles > 0) he = hipMalloc((void**)&part, (size_t)ptiles * 4096 * sizeof(double));
  if (he == hipSuccess && (d.nd.on || d.ix.on)) he = hipMalloc((void**)&Sp, nS * sizeof(double));
  if (he == hipSuccess)
    he = d.nd.on   ? nd_numeric(d, Sp, L, Li, part, st)
         : d.ix.on ? ix_numeric(d, Sp, L, Li, part, st)
                   : dense_cholesky_inverse(d, L, Li, part, st);
  const hipError_t he2 = hipStreamSynchronize(st);
  if (he == hipSuccess) he = he2;
  (void)hipFree(L);
  (void)hipFree(Li);
  (void)hipFree(part);
  (void)hipFree(Sp);
  return he;
}

// row of S (original numbering) named by a failing pivot of the interface
// factorization (the nested-dissection form factors a reordered, padded S)
static int64_t iface_fail_row(const DeviceState& d, int32_t row) {
  if (!d.nd.on || row < 0 || row >= (int32_t)d.nd.h_src.size()) return row;
  return d.nd.h_src[row];
}

// plain: factor the diagonal blocks A_ii of the partition as they are (no
// interface, no basis functions, no S): the block solves of block-Jacobi
// smoothing (Sec. 5.4)
static am_status setup_impl(const am_csr* A, const int32_t* part, int32_t nparts,
                            const am_options* opt_in, void* stream, am_handle* out, bool plain) {
  if (!out) return fail(nullptr, AM_ERR_ARG, "out is null");
  *out = nullptr;
  am_options opt{AM_FP64, AM_MORTAR_PER_INTERFACE, 1, 0, 0u};
  if (opt_in) opt = *opt_in;
  if (opt.local_prec < AM_FP64 || opt.local_prec > AM_BF16 || opt.mortar < 0 || opt.mortar > 1 ||
      opt.max_nrhs < 1 || opt.max_nrhs > kMaxNRHS || opt.device < 0)
    return fail(nullptr, AM_ERR_ARG, "invalid options");
  am_handle h = new am_handle_s();
  h->opt = opt;
  auto bail = [&](am_status s) {
    std::string msg = h->err;
    algmortar_destroy(h);
    g_err = msg;
    return s;
  };
  // optional phase times on stderr (environment ALGMORTAR_SETUP_TIMES set):
  // a phase that queued device work ends with a stream synchronisation, so
  // the work is charged to it
  const bool ptimes = std::getenv("ALGMORTAR_SETUP_TIMES") != nullptr;
  std::vector<std::pair<const char*, double>> phases;
  auto t_last = std::chrono::steady_clock::now();
  auto mark = [&](const char* name, hipStream_t sync) {
    if (!ptimes) return;
    if (sync) (void)hipStreamSynchronize(sync);
    const auto t = std::chrono::steady_clock::now();
    phases.emplace_back(name, std::chrono::duration<double, std::milli>(t - t_last).count());
    t_last = t;
  };
  HostCSR H;
  std::vector<double> vals;
  if (A && A->values_on_device) {
    // device values may still be written by work queued on the caller's
    // stream (NULL: the null stream)
    if (hipSetDevice(opt.device) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
      fail(h, AM_ERR_HIP, "hipSetDevice / caller stream synchronization failed");
      return bail(AM_ERR_HIP);
    }
  }
  am_status s = host_csr(A, H, vals, h);
  if (s != AM_OK) return bail(s);
  mark("host copy of A", nullptr);
  std::string e;
  if ((s = validate_csr(H, e)) != AM_OK) { fail(h, s, e); return bail(s); }
  if ((s = validate_partition(H.n, part, nparts, e)) != AM_OK) { fail(h, s, e); return bail(s); }
  mark("validation", nullptr);
  if (!plain) {
    h->pat_rp.assign(H.rp, H.rp + H.n + 1);
    h->pat_ci.assign(H.ci, H.ci + H.nnz);
  }
  Structure& st = h->st;
  LocalPlan& lp = h->lp;
  if ((s = build_structure(H, part, nparts, opt.mortar, st, e)) != AM_OK) { fail(h, s, e); return bail(s); }
  mark("interface structure", nullptr);
  if (plain) {
    st.edge_k.clear();
    st.edge_l.clear();
    st.edge_a.clear();
    st.iface_ptr.assign(1, 0);
    st.iface_ij.clear();
    st.isub_ptr.assign((size_t)st.m + 1, 0);
    st.isub_list.clear();
  }
  if ((s = plan_local(H, st, lp, e)) != AM_OK) { fail(h, s, e); return bail(s); }
  mark("local orderings", nullptr);
  if (lp.max_ni > 128) {
    fail(h, AM_ERR_UNSUPPORTED, "a subdomain touches more than 128 mortar basis functions");
    return bail(AM_ERR_UNSUPPORTED);
  }
  if (lp.max_ni > 64 && pow2_at_least(std::max(opt.max_nrhs, 1)) >= 8) {
    fail(h, AM_ERR_UNSUPPORTED,
         "with 8 or more right-hand sides a subdomain may touch at most 64 mortar basis functions");
    return bail(AM_ERR_UNSUPPORTED);
  }

  DeviceState& d = h->d;
  d.plain = plain ? 1 : 0;
  d.device = opt.device;
  d.prec = opt.local_prec;
  d.n = H.n;
  d.m = st.m;
  d.NL = st.n_iface();
  d.NE = st.n_edges();
  d.ldS = (int32_t)((d.NL + kTile - 1) / kTile * kTile);
  d.max_nrhs = pow2_at_least(opt.max_nrhs);
  // small interface inverses are applied inside the local kernel (each
  // subdomain multiplies its own rows; every row is read twice)
  d.fuse_eta = (d.NL > 0 && (double)d.NL * d.NL * 8.0 <= 64.0 * 1024 * 1024) ? 1 : 0;
  // the tile kernel folds the per-wave partial rows in its second tile buffer
  // (at least 8 KB for every factor precision and window)
  if ((int64_t)lp.max_ni * pow2_at_least(std::max(opt.max_nrhs, 1)) * 8 * 8 > 8192) d.fuse_eta = 0;
  if (opt.flags & (AM_FLAG_SEPARATE_IFACE | AM_FLAG_INEXACT_IFACE)) d.fuse_eta = 0;
  d.bf16_ops = (opt.flags & AM_FLAG_BF16_PRODUCTS) && d.prec == AM_BF16 ? 1 : 0;
  const bool use_ix = !plain && d.NL > 0 && (opt.flags & AM_FLAG_INEXACT_IFACE);
  for (int32_t s2 = 0; s2 < st.m; ++s2)
    d.max_np = std::max<int32_t>(d.max_np, (int32_t)(lp.roff[s2 + 1] - lp.roff[s2]));
  // nested-dissection layout of S where eta is its own launches (the dense
  // explicit S^{-1} stays available with AM_FLAG_DENSE_IFACE, and is the
  // fall-back when no dissection depth fits the kernels)
  IfaceND ndh;
  bool use_nd = false;
  if (!plain && !d.fuse_eta && d.NL > 0 && !use_ix && !(opt.flags & AM_FLAG_DENSE_IFACE)) {
    std::string e2;
    use_nd = build_iface_nd(st, nd_max_rows(d.max_nrhs), 1.15, ndh, e2) == AM_OK;
  }

  auto hipfail = [&](hipError_t he, const char* what) {
    fail(h, he == hipErrorOutOfMemory ? AM_ERR_OOM : AM_ERR_HIP,
         std::string(what) + ": " + hipGetErrorString(he));
    return bail(he == hipErrorOutOfMemory ? AM_ERR_OOM : AM_ERR_HIP);
  };
#define SCHK(expr)                              \
  do {                                          \
    hipError_t he_ = (expr);                    \
    if (he_ != hipSuccess) return hipfail(he_, #expr); \
  } while (0)

  SCHK(hipSetDevice(d.device));
  // the device's address of the static scratch of algmortar_apply_static
  // (looked up once per device; a failure is reported by that entry point,
  // which looks it up again, and does not affect the rest of the library)
  (void)static_scratch_init(d.device);
  SCHK(hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking));
  SCHK(hipStreamCreateWithFlags(&d.side, hipStreamNonBlocking));
  SCHK(hipEventCreateWithFlags(&d.ev_fork, hipEventDisableTiming));
  SCHK(hipEventCreateWithFlags(&d.ev_join, hipEventDisableTiming));
  SCHK(hipEventCreate(&h->ev0));
  SCHK(hipEventCreate(&h->ev1));
  SCHK(hipEventCreateWithFlags(&h->evf[0], hipEventDisableTiming));
  SCHK(hipEventCreateWithFlags(&h->evf[1], hipEventDisableTiming));
  hipStream_t sm = h->own;
  // the caller's stream (NULL: the null stream) may still be writing A's
  // values; the library's own stream does not wait for it by itself
  SCHK(hipStreamSynchronize((hipStream_t)stream));
  mark("device context", nullptr);

  // ---- host-side layout ----
  const int64_t n = d.n;
  const std::vector<int32_t>& dperm = lp.dperm;
  const std::vector<int32_t>& dpos = lp.dpos;
  std::vector<int64_t> prp(n + 1, 0);
  HostBuf<int32_t> pci((size_t)H.nnz);
  HostBuf<double> pv((size_t)H.nnz);
  int32_t w = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t o = dperm[i];
    prp[i + 1] = prp[i] + (H.rp[o + 1] - H.rp[o]);
    w = std::max<int32_t>(w, (int32_t)(H.rp[o + 1] - H.rp[o]));
  }
  // rows of A in device order, columns ascending (each row its own range)
  parallel_for((n + 1023) / 1024, 1, [&](int64_t c) {
    std::vector<std::pair<int32_t, double>> row;
    const int64_t hi = std::min<int64_t>(n, (c + 1) * 1024);
    for (int64_t i = c * 1024; i < hi; ++i) {
      const int64_t o = dperm[i];
      row.clear();
      for (int64_t p = H.rp[o]; p < H.rp[o + 1]; ++p) row.emplace_back(dpos[H.ci[p]], H.v[p]);
      std::sort(row.begin(), row.end(),
                [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
                  return a.first < b.first;
                });
      for (size_t t = 0; t < row.size(); ++t) {
        pci[prp[i] + t] = row[t].first;
        pv[prp[i] + t] = row[t].second;
      }
    }
  });
  d.ell_w = w;
  HostBuf<int32_t> ell_col((size_t)w * n);
  HostBuf<double> ell_val((size_t)w * n);
  parallel_for((n + 4095) / 4096, 1, [&](int64_t cb) {
    const int64_t hi = std::min<int64_t>(n, (cb + 1) * 4096);
    for (int64_t i = cb * 4096; i < hi; ++i)
      for (int32_t c = 0; c < w; ++c) {
        const int64_t p = prp[i] + c;
        if (p < prp[i + 1]) {
          ell_col[(size_t)c * n + i] = pci[p];
          ell_val[(size_t)c * n + i] = pv[p];
        } else {
          ell_col[(size_t)c * n + i] = (int32_t)i;
          ell_val[(size_t)c * n + i] = 0.0;
        }
      }
  });
  for (int bk = 0; bk < 2; ++bk) d.bucket_sub[bk].clear();
  for (int32_t s2 = 0; s2 < st.m; ++s2) d.bucket_sub[lp.wp[s2] == 64 ? 0 : 1].push_back(s2);

  const int64_t NL = d.NL;
  const int64_t npair = 2 * NL;
  std::vector<int32_t> pair_sub(npair), pair_q(npair);
  std::vector<int64_t> bidx(npair);  // (interface, side) -> pair
  std::vector<int64_t> bdst(npair);  // pair -> (interface, side) slot 2n + side
  for (int32_t s2 = 0; s2 < st.m; ++s2)
    for (int64_t pi = st.isub_ptr[s2]; pi < st.isub_ptr[s2 + 1]; ++pi) {
      pair_sub[pi] = s2;
      pair_q[pi] = (int32_t)(pi - st.isub_ptr[s2]);
      const int32_t nidx = st.isub_list[pi];
      const int side = st.iface_ij[2 * nidx] == s2 ? 0 : 1;
      bidx[2 * nidx + side] = pi;
      bdst[pi] = 2 * (int64_t)nidx + side;
    }
  for (int bk = 0; bk < 2; ++bk) d.bucket_pair[bk].clear();
  for (int64_t pi = 0; pi < npair; ++pi)
    d.bucket_pair[lp.wp[pair_sub[pi]] == 64 ? 0 : 1].push_back((int32_t)pi);
  std::vector<int64_t> mbf_off(st.m + 1, 0);
  for (int32_t s2 = 0; s2 < st.m; ++s2)
    mbf_off[s2 + 1] = mbf_off[s2] + (st.isub_ptr[s2 + 1] - st.isub_ptr[s2]) *
                                        (st.sub_ptr[s2 + 1] - st.sub_ptr[s2]);
  // boundary weights -B_s psi_n: entry k collects -2 a_e over the edges of E_n
  // at k.  The slot (n, side) lists the edges of E_n in order, sorted stably
  // by local row and summed in that order; slots are independent, built in
  // parallel and concatenated in slot order.
  std::vector<int32_t> e_kloc(d.NE), e_lloc(d.NE);
  parallel_for(NL, 64, [&](int64_t nidx) {
    const int32_t i = st.iface_ij[2 * nidx], j = st.iface_ij[2 * nidx + 1];
    for (int64_t e2 = st.iface_ptr[nidx]; e2 < st.iface_ptr[nidx + 1]; ++e2) {
      e_kloc[e2] = dpos[st.edge_k[e2]] - (int32_t)st.sub_ptr[i];
      e_lloc[e2] = dpos[st.edge_l[e2]] - (int32_t)st.sub_ptr[j];
    }
  });
  std::vector<int64_t> pair_if(npair);
  for (int64_t nidx = 0; nidx < NL; ++nidx) {
    pair_if[bidx[2 * nidx]] = 2 * nidx;
    pair_if[bidx[2 * nidx + 1]] = 2 * nidx + 1;
  }
  std::vector<std::vector<std::pair<int32_t, double>>> wts(npair);
  parallel_for(npair, 16, [&](int64_t pi) {
    const int64_t nidx = pair_if[pi] / 2;
    const bool side1 = pair_if[pi] & 1;
    std::vector<std::pair<int32_t, double>> v;
    v.reserve((size_t)(st.iface_ptr[nidx + 1] - st.iface_ptr[nidx]));
    for (int64_t e2 = st.iface_ptr[nidx]; e2 < st.iface_ptr[nidx + 1]; ++e2)
      v.emplace_back(side1 ? e_lloc[e2] : e_kloc[e2], -2.0 * st.edge_a[e2]);
    std::stable_sort(v.begin(), v.end(),
                     [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
                       return a.first < b.first;
                     });
    auto& g = wts[pi];
    for (size_t t = 0; t < v.size(); ++t) {
      if (t > 0 && v[t].first == v[t - 1].first)
        g.back().second += v[t].second;
      else
        g.push_back(v[t]);
    }
  });
  std::vector<int64_t> bw_ptr(npair + 1, 0);
  for (int64_t pi = 0; pi < npair; ++pi) bw_ptr[pi + 1] = bw_ptr[pi] + (int64_t)wts[pi].size();
  std::vector<int32_t> bw_row((size_t)bw_ptr[npair]);
  std::vector<double> bw_val((size_t)bw_ptr[npair]);
  parallel_for(npair, 64, [&](int64_t pi) {
    for (size_t t = 0; t < wts[pi].size(); ++t) {
      bw_row[bw_ptr[pi] + t] = wts[pi][t].first;
      bw_val[bw_ptr[pi] + t] = wts[pi][t].second;
    }
  });
  std::vector<std::vector<std::pair<int32_t, double>>>().swap(wts);

  mark("host layout", nullptr);

  // ---- device upload ----
  std::vector<void*>& al = d.allocs;
  SCHK(upload(al, &d.dperm, dperm, sm));
  SCHK(upload(al, &d.ell_col, ell_col.p.get(), ell_col.n, sm));
  SCHK(upload(al, &d.ell_val, ell_val.p.get(), ell_val.n, sm));
  SCHK(upload(al, &d.prp, prp, sm));
  SCHK(upload(al, &d.pci, pci.p.get(), pci.n, sm));
  SCHK(upload(al, &d.pv, pv.p.get(), pv.n, sm));
  SCHK(upload(al, &d.sub_ptr, st.sub_ptr, sm));
  SCHK(upload(al, &d.wp, lp.wp, sm));
  SCHK(upload(al, &d.roff, lp.roff, sm));
  SCHK(upload(al, &d.fac_off, lp.fac_off, sm));
  for (int bk = 0; bk < 2; ++bk) {
    SCHK(upload(al, &d.d_bucket_sub[bk], d.bucket_sub[bk], sm));
    SCHK(upload(al, &d.d_bucket_pair[bk], d.bucket_pair[bk], sm));
  }
  SCHK(upload(al, &d.isub_ptr, st.isub_ptr, sm));
  SCHK(upload(al, &d.isub_list, st.isub_list, sm));
  SCHK(upload(al, &d.mbf_off, mbf_off, sm));
  SCHK(upload(al, &d.bw_ptr, bw_ptr, sm));
  SCHK(upload(al, &d.bw_row, bw_row, sm));
  SCHK(upload(al, &d.bw_val, bw_val, sm));
  SCHK(upload(al, &d.mbf_pair_sub, pair_sub, sm));
  SCHK(upload(al, &d.mbf_pair_q, pair_q, sm));
  SCHK(upload(al, &d.iface_ptr, st.iface_ptr, sm));
  SCHK(upload(al, &d.iface_ij, st.iface_ij, sm));
  SCHK(upload(al, &d.e_kloc, e_kloc, sm));
  SCHK(upload(al, &d.e_lloc, e_lloc, sm));
  SCHK(upload(al, &d.e_a, st.edge_a, sm));
  SCHK(upload(al, &d.bdst, bdst, sm));
  ell_val.p.reset();
  ell_col.p.reset();
  mark("uploads", sm);

  const size_t esz = d.prec == AM_FP64 ? 8 : (d.prec == AM_FP32 ? 4 : 2);
  const size_t isz = d.prec == AM_FP64 ? 8 : 4;
  const size_t nfac = (size_t)lp.fac_off[st.m];
  uint8_t *Lc = nullptr, *Lr = nullptr, *iv = nullptr;
  SCHK(dalloc(al, &Lc, nfac * esz));
  SCHK(dalloc(al, &Lr, nfac * esz));
  SCHK(dalloc(al, &iv, (size_t)lp.roff[st.m] * isz));
  d.Lc = Lc;
  d.Lr = Lr;
  d.invd = iv;
  SCHK(hipMemsetAsync(Lc, 0, nfac * esz, sm));
  SCHK(hipMemsetAsync(Lr, 0, nfac * esz, sm));
  SCHK(dalloc(al, &d.fail, 4));
  SCHK(hipMemsetAsync(d.fail, 0xFF, 4 * sizeof(int32_t), sm));
  SCHK(dalloc(al, &d.mbf, (size_t)mbf_off[st.m]));
  const size_t nS = (size_t)d.ldS * d.ldS;
  SCHK(dalloc(al, &d.S, nS));
  if (use_nd) {
    SCHK(nd_upload(d, ndh, sm));
    SCHK(dalloc(al, &d.Sinv, (size_t)d.nd.ldp * d.nd.ldp));  // reordered S^{-1}
  } else {
    SCHK(dalloc(al, &d.Sinv, nS));
  }
  if (use_ix) SCHK(ix_upload(d, st, sm));
  if (!d.fuse_eta && NL > 0 && !use_nd && !use_ix) {
    // enough (row block, part) waves to fill the chip, each part >= 64 rows
    const int64_t nrb = (NL + 63) / 64;
    d.op_parts = (int32_t)std::max<int64_t>(1, std::min<int64_t>({64, (8192 + nrb - 1) / nrb, NL / 64}));
    SCHK(dalloc(al, &d.ypart, (size_t)d.op_parts * d.ldS * d.max_nrhs));
  }

  const int NRm = d.max_nrhs;
  const size_t nv = (size_t)n * NRm;
  SCHK(dalloc(al, &d.x, nv));
  SCHK(dalloc(al, &d.r, nv));
  SCHK(dalloc(al, &d.z, nv));
  SCHK(dalloc(al, &d.p[0], nv));
  SCHK(dalloc(al, &d.p[1], nv));
  SCHK(dalloc(al, &d.q, nv));
  SCHK(dalloc(al, &h->bp, nv));
  SCHK(dalloc(al, &d.bpart, (size_t)std::max<int64_t>(npair, 1) * NRm));
  SCHK(dalloc(al, &d.eta, (size_t)std::max<int32_t>(d.ldS, 1) * NRm));
  SCHK(dalloc(al, &d.sc, kMaxNRHS));
  SCHK(dalloc(al, &d.shared, 1));
  SCHK(dalloc(al, &h->tres, kMaxNRHS));
  d.red.max_blocks = (int)std::max<int64_t>((n + 255) / 256, st.m) + 1;
  d.red.spmv_blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
  SCHK(dalloc(al, &d.red.partial, (size_t)d.red.max_blocks * 2 * kMaxNRHS));
  // (p, Ap) partials: per SpMV workgroup (1-4 columns) or per subdomain (8-16)
  SCHK(dalloc(al, &d.red.pa, (size_t)std::max<int64_t>(d.red.spmv_blocks, st.m) * kMaxNRHS));
  SCHK(dalloc(al, &d.red.pb, (size_t)st.m * kMaxNRHS));
  SCHK(dalloc(al, &d.red.pd, (size_t)st.m * 2 * kMaxNRHS));
  SCHK(dalloc(al, &d.red.coef, 2 * kMaxNRHS));
  SCHK(dalloc(al, &d.red.counter, 8));
  SCHK(hipMemsetAsync(d.red.counter, 0, 8 * sizeof(unsigned), sm));
  SCHK(hipMemsetAsync(d.shared, 0, sizeof(PcgShared), sm));
  SCHK(hipHostMalloc((void**)&d.h_flags, 4 * sizeof(int32_t), hipHostMallocDefault));
  SCHK(hipHostMalloc((void**)&d.h_sc, 2 * kMaxNRHS * sizeof(PcgScalars), hipHostMallocDefault));

  mark("device allocations", sm);

  // ---- Algorithm 1 on the device ----
  SCHK(launch_band_factor(d, sm));
  mark("local factors", sm);
  SCHK(launch_mbf(d, sm));
  mark("basis functions", sm);
  // solve-time form of the factor: inverted diagonal blocks, column layout only
  SCHK(launch_invert_diag(d, sm));
  mark("diagonal block inverses", sm);
  SCHK(launch_assemble_S(d, sm));
  mark("interface matrix S", sm);
  if (NL > 0) {
    hipError_t he = interface_inverse(d, sm);
    if (he != hipSuccess) return hipfail(he, "interface factorization");
    mark(d.nd.on ? "interface blocks (dissection)" : "interface inverse", nullptr);
  }
  SCHK(hipStreamSynchronize(sm));
  int32_t fl[4];
  SCHK(hipMemcpy(fl, d.fail, sizeof(fl), hipMemcpyDeviceToHost));
  if (fl[0] >= 0) {
    fail(h, AM_ERR_NOT_SPD, "A_i not SPD: subdomain " + std::to_string(fl[0]) + " pivot " +
                                std::to_string(fl[1]));
    return bail(AM_ERR_NOT_SPD);
  }
  if (fl[2] >= 0) {
    fail(h, AM_ERR_NOT_SPD,
         "interface matrix S not SPD at row " + std::to_string(iface_fail_row(d, fl[2])));
    return bail(AM_ERR_NOT_SPD);
  }
  // free set-up only arrays: the row layout of the factor served the
  // set-up solves of the basis functions only
  for (auto it = d.allocs.begin(); it != d.allocs.end(); ++it)
    if (*it == d.Lr) {
      (void)hipFree(*it);
      d.allocs.erase(it);
      break;
    }
  d.Lr = nullptr;
  mark("checks and frees", nullptr);
  for (const auto& ph : phases) std::fprintf(stderr, "algmortar set-up: %-24s %9.2f ms\n", ph.first, ph.second);
  *out = h;
  return AM_OK;
#undef SCHK
}

am_status algmortar_setup(const am_csr* A, const int32_t* part, int32_t nparts,
                          const am_options* opt_in, void* stream, am_handle* out) {
  return setup_impl(A, part, nparts, opt_in, stream, out, false);
}

// ---------------------------------------------------------------------------
static am_status check_vec_args(am_handle h, const void* a, const void* b, int32_t nrhs,
                                int64_t ld) {
  if (!h) return fail(nullptr, AM_ERR_ARG, "null handle");
  if (!a || !b) return fail(h, AM_ERR_ARG, "null vector");
  if (!h->numeric_ok)
    return fail(h, AM_ERR_NOT_SPD, "the last algmortar_update_values failed: no preconditioner");
  if (nrhs < 1 || pow2_at_least(nrhs) > h->d.max_nrhs)
    return fail(h, AM_ERR_ARG, "nrhs out of range (max_nrhs at set-up)");
  if (nrhs > 1 && ld < h->d.n) return fail(h, AM_ERR_ARG, "ld < n");
  return AM_OK;
}

// Autotuner of the tile kernel's wave layout: for nr right-hand sides it
// times every candidate layout (3 applies each, after one warm-up, on zeroed
// work vectors of this handle) and keeps the fastest for the handle's later
// applies and solves.  Runs once per right-hand-side count, outside any graph
// capture.
// The local kernel has a single layout: 16 right-hand sides with the
// interface solve as its own launches, or one right-hand side with BF16 x
// BF16 products where every subdomain is in the window-64 bucket (the
// matrix-core kernels in both cases).
static bool single_layout(const DeviceState& d, int nr) {
  if (d.fuse_eta) return false;
  return nr == 16 || (nr == 1 && d.bf16_ops && d.bucket_sub[1].empty());
}

static am_status autotune_tiles(am_handle h, int nr) {
  DeviceState& d = h->d;
  const int slot = tile_slot(nr);
  if (d.tile_cand[slot] >= 0) return AM_OK;
  const int nc = tile_candidates(nr);
  // the matrix-core kernels have one layout: nothing to choose
  if (single_layout(d, nr)) {
    d.tile_cand[slot] = 0;
    return AM_OK;
  }
  // ALGMORTAR_TILE=c pins candidate c (clamped to the list): the layouts
  // sum the waves' partial vectors in different orders, so results of
  // handles (or processes) whose timings chose differently can differ in
  // the last bits; a pinned layout makes them reproducible
  if (const char* env = std::getenv("ALGMORTAR_TILE")) {
    const int c = std::atoi(env);
    d.tile_cand[slot] = std::min(std::max(c, 0), nc - 1);
    return AM_OK;
  }
  // ALGMORTAR_AUTOTUNE_CACHE=file keeps the choices across processes: a
  // line "key choice" per tuned case, the key describing what the layouts
  // are timed on (sizes, window buckets, factor precision, interface form,
  // right-hand sides); a case found there is not timed again
  const char* cache = std::getenv("ALGMORTAR_AUTOTUNE_CACHE");
  std::string key;
  if (cache && *cache) {
    key = "n" + std::to_string(d.n) + "_m" + std::to_string(d.m) + "_nl" + std::to_string(d.NL) +
          "_b" + std::to_string(d.bucket_sub[0].size()) + "x" + std::to_string(d.bucket_sub[1].size()) +
          "_p" + std::to_string(d.prec) + "_f" + std::to_string(d.fuse_eta) + "_pl" +
          std::to_string(d.plain) + "_nr" + std::to_string(nr) + "_c" + std::to_string(nc);
    if (FILE* f = std::fopen(cache, "r")) {
      char k[256];
      int c = -1, found = -1;
      while (std::fscanf(f, "%255s %d", k, &c) == 2)
        if (key == k) found = c;  // the last entry of a key wins
      std::fclose(f);
      if (found >= 0 && found < nc) {
        d.tile_cand[slot] = found;
        return AM_OK;
      }
    }
  }
  hipStream_t st = h->own;
  HCHK(launch_fill(d.r, d.n * nr, 0.0, st));
  HCHK(launch_fill(d.z, d.n * nr, 0.0, st));
  if (d.NL > 0) {
    HCHK(launch_fill(d.bpart, 2 * d.NL * nr, 0.0, st));
    HCHK(launch_fill(d.eta, (int64_t)d.ldS * nr, 0.0, st));
  }
  // Timed as a solve runs the kernel: with the PCG dots (mode 2) on a live
  // state (a solve initialises its own afterwards), unless the interface
  // solve is fused in, whose stop test would end the launch early (mode 1);
  // the smoother's block factors without a coarse part (mode 0).  The
  // candidates take turns over three rounds and keep their fastest round,
  // so a clock ramp at the start does not favour the later ones.
  const int tmode = d.plain ? 0 : (d.fuse_eta ? 1 : 2);
  if (tmode == 2) HCHK(launch_pcg_init(d, nr, 1e-300, 1 << 30, 0, st));
  for (int c = 0; c < nc; ++c) d.tile_us[slot][c] = 0.f;
  for (int round = 0; round < 3; ++round)
    for (int c = 0; c < nc; ++c) {
      d.tile_cand[slot] = c;
      HCHK(launch_local_sweep(d, d.r, d.z, d.eta, nr, tmode, st));
      HCHK(hipEventRecord(h->ev0, st));
      for (int i = 0; i < 3; ++i) HCHK(launch_local_sweep(d, d.r, d.z, d.eta, nr, tmode, st));
      HCHK(hipEventRecord(h->ev1, st));
      HCHK(hipEventSynchronize(h->ev1));
      float ms = 0.f;
      HCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
      const float us = ms * 1000.f / 3.f;
      if (round == 0 || us < d.tile_us[slot][c]) d.tile_us[slot][c] = us;
    }
  int bc = 0;
  for (int c = 1; c < nc; ++c)
    if (d.tile_us[slot][c] < d.tile_us[slot][bc]) bc = c;
  d.tile_cand[slot] = bc;
  if (!key.empty())
    if (FILE* f = std::fopen(cache, "a")) {
      std::fprintf(f, "%s %d\n", key.c_str(), bc);
      std::fclose(f);
    }
  return AM_OK;
}

am_status algmortar_tile_choice(am_handle h, int32_t nrhs, int32_t* choice, int32_t* ncand,
                                double* us) {
  if (!h || !choice || !ncand || nrhs < 1 || pow2_at_least(nrhs) > h->d.max_nrhs)
    return fail(h, AM_ERR_ARG, "bad argument");
  HCHK(hipSetDevice(h->d.device));
  const int nr = pow2_at_least(nrhs);
  am_status s = autotune_tiles(h, nr);
  if (s != AM_OK) return s;
  const int slot = tile_slot(nr);
  *choice = h->d.tile_cand[slot];
  *ncand = single_layout(h->d, nr) ? 1 : tile_candidates(nr);
  if (us)
    for (int c = 0; c < *ncand; ++c) us[c] = h->d.tile_us[slot][c];
  return AM_OK;
}

static void drop_smoother(am_handle h) {
  for (void* p : h->sm_allocs) (void)hipFree(p);
  h->sm_allocs.clear();
  if (h->bj) algmortar_destroy(h->bj);
  h->bj = nullptr;
  h->sm = SmoothDevice{};
}

// ---------------------------------------------------------------------------
// New values on an existing handle.  The maps below are built from the
// set-up's pattern, partition and layout at the first update; they place each
// caller entry where the set-up put its value, in the set-up's order.
static am_status build_value_maps(am_handle h) {
  ValueMaps& vm = h->vm;
  DeviceState& d = h->d;
  const Structure& st = h->st;
  const LocalPlan& lp = h->lp;
  const int64_t n = d.n, nnz = (int64_t)h->pat_ci.size();
  const int64_t* rp = h->pat_rp.data();
  const int32_t* ci = h->pat_ci.data();
  auto find = [&](int64_t row, int32_t col) -> int64_t {
    const int32_t* b = ci + rp[row];
    const int32_t* e = ci + rp[row + 1];
    const int32_t* it = std::lower_bound(b, e, col);
    return (it == e || *it != col) ? -1 : rp[row] + (it - b);
  };
  // device-order rows with ascending device columns, as the set-up builds them
  std::vector<int64_t> prp(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t o = lp.dperm[i];
    prp[i + 1] = prp[i] + (rp[o + 1] - rp[o]);
  }
  std::vector<int64_t> vpos((size_t)nnz);
  parallel_for((n + 1023) / 1024, 1, [&](int64_t c) {
    std::vector<std::pair<int32_t, int64_t>> row;
    const int64_t hi = std::min<int64_t>(n, (c + 1) * 1024);
    for (int64_t i = c * 1024; i < hi; ++i) {
      const int64_t o = lp.dperm[i];
      row.clear();
      for (int64_t p = rp[o]; p < rp[o + 1]; ++p) row.emplace_back(lp.dpos[ci[p]], p);
      std::sort(row.begin(), row.end());
      for (size_t t = 0; t < row.size(); ++t) vpos[prp[i] + t] = row[t].second;
    }
  });
  vm.code_h.assign((size_t)nnz, 0);
  vm.cross_h.assign((size_t)nnz, 0);
  parallel_for((n + 4095) / 4096, 1, [&](int64_t c) {
    const int64_t hi = std::min<int64_t>(n, (c + 1) * 4096);
    for (int64_t k = c * 4096; k < hi; ++k)
      for (int64_t p = rp[k]; p < rp[k + 1]; ++p) {
        const int32_t col = ci[p];
        vm.code_h[p] = col == k ? -2 : find(col, (int32_t)k);
        if (st.part[col] != st.part[k]) vm.cross_h[p] = 2;
      }
  });
  std::vector<int64_t> epos((size_t)d.NE);
  for (int64_t e = 0; e < d.NE; ++e) {
    const int64_t p = find(st.edge_k[e], st.edge_l[e]);
    if (p < 0) return fail(h, AM_ERR_ARG, "internal: an interface edge is not in the pattern");
    epos[e] = p;
    vm.cross_h[p] = 1;
    if (vm.code_h[p] >= 0) vm.cross_h[vm.code_h[p]] = 1;
  }
  // boundary-weight entries: per (interface, side) slot, the edges grouped by
  // local row after a stable sort, summed in that order
  const int64_t NL = d.NL, npair = 2 * NL;
  std::vector<int64_t> bidx((size_t)npair);
  for (int32_t s2 = 0; s2 < st.m; ++s2)
    for (int64_t pi = st.isub_ptr[s2]; pi < st.isub_ptr[s2 + 1]; ++pi) {
      const int32_t nidx = st.isub_list[pi];
      bidx[2 * nidx + (st.iface_ij[2 * nidx] == s2 ? 0 : 1)] = pi;
    }
  std::vector<std::vector<std::pair<int32_t, int32_t>>> wts((size_t)npair);
  for (int64_t nidx = 0; nidx < NL; ++nidx) {
    const int32_t i = st.iface_ij[2 * nidx], j = st.iface_ij[2 * nidx + 1];
    for (int64_t e2 = st.iface_ptr[nidx]; e2 < st.iface_ptr[nidx + 1]; ++e2) {
      wts[bidx[2 * nidx]].emplace_back(lp.dpos[st.edge_k[e2]] - (int32_t)st.sub_ptr[i], (int32_t)e2);
      wts[bidx[2 * nidx + 1]].emplace_back(lp.dpos[st.edge_l[e2]] - (int32_t)st.sub_ptr[j], (int32_t)e2);
    }
  }
  std::vector<int64_t> bw_ptr(1, 0);
  std::vector<int32_t> bw_src;
  for (int64_t pi = 0; pi < npair; ++pi) {
    auto& v = wts[pi];
    std::stable_sort(v.begin(), v.end(),
                     [](const std::pair<int32_t, int32_t>& a, const std::pair<int32_t, int32_t>& b) {
                       return a.first < b.first;
                     });
    for (size_t t = 0; t < v.size(); ++t) {
      if (t == 0 || v[t].first != v[t - 1].first) bw_ptr.push_back(bw_ptr.back());
      bw_src.push_back(v[t].second);
      bw_ptr.back() += 1;
    }
  }
  vm.nnz = nnz;
  vm.nbw = (int64_t)bw_ptr.size() - 1;
  hipStream_t st0 = h->own;
  HCHK(upload(vm.allocs, &vm.vpos, vpos, st0));
  HCHK(upload(vm.allocs, &vm.code, vm.code_h, st0));
  HCHK(upload(vm.allocs, &vm.cross, vm.cross_h, st0));
  HCHK(upload(vm.allocs, &vm.epos, epos, st0));
  HCHK(upload(vm.allocs, &vm.bw_ptr, bw_ptr, st0));
  HCHK(upload(vm.allocs, &vm.bw_src, bw_src, st0));
  HCHK(dalloc(vm.allocs, &vm.vals, (size_t)nnz));
  HCHK(dalloc(vm.allocs, &vm.bad, 1));
  vm.built = true;
  return AM_OK;
}

am_status algmortar_update_values(am_handle h, const am_csr* A, void* stream) {
  if (!h) return fail(nullptr, AM_ERR_ARG, "null handle");
  if (!A || !A->row_ptr || !A->col_idx || !A->val) return fail(h, AM_ERR_ARG, "A: null pointer");
  if (h->pat_rp.empty()) return fail(h, AM_ERR_ARG, "the handle keeps no pattern");
  if (h->bj)
    return fail(h, AM_ERR_UNSUPPORTED, "remove the smoother (steps 0) before setting new values");
  const int64_t nnz = (int64_t)h->pat_ci.size();
  if (A->n != h->d.n || A->nnz != nnz ||
      std::memcmp(A->row_ptr, h->pat_rp.data(), sizeof(int64_t) * (size_t)(A->n + 1)) != 0 ||
      std::memcmp(A->col_idx, h->pat_ci.data(), sizeof(int32_t) * (size_t)nnz) != 0)
    return fail(h, AM_ERR_ARG, "A's pattern differs from the one the handle was set up with");
  DeviceState& d = h->d;
  HCHK(hipSetDevice(d.device));
  // work queued on the caller's stream (NULL: the null stream) may still be
  // writing the new values; h->own is a non-blocking stream and does not
  // wait for it by itself
  HCHK(hipStreamSynchronize((hipStream_t)stream));
  hipStream_t st = h->own;
  HCHK(hipStreamSynchronize(st));
  if (!h->vm.built) {
    am_status s = build_value_maps(h);
    if (s != AM_OK) return s;
  }
  ValueMaps& vm = h->vm;
  const double* v = A->val;
  if (!A->values_on_device) {
    HCHK(hipMemcpyAsync(vm.vals, A->val, sizeof(double) * (size_t)nnz, hipMemcpyHostToDevice, st));
    v = vm.vals;
  }
  // the set-up's checks; the handle is unchanged when they fail
  HCHK(launch_check_values(vm, v, st));
  unsigned long long bad = 0;
  HCHK(hipMemcpyAsync(&bad, vm.bad, sizeof(bad), hipMemcpyDeviceToHost, st));
  HCHK(hipStreamSynchronize(st));
  if (bad != ~0ull) {
    const int64_t p = (int64_t)bad, t = vm.code_h[p];
    double a = 0.0, b = 0.0;
    HCHK(hipMemcpy(&a, v + p, sizeof(double), hipMemcpyDefault));
    if (t >= 0) HCHK(hipMemcpy(&b, v + t, sizeof(double), hipMemcpyDefault));
    const int64_t k = (int64_t)(std::upper_bound(h->pat_rp.begin(), h->pat_rp.end(), p) - h->pat_rp.begin()) - 1;
    const std::string at = "(" + std::to_string(k) + "," + std::to_string(h->pat_ci[p]) + ")";
    if (!std::isfinite(a)) return fail(h, AM_ERR_ARG, "A: non-finite value at " + at);
    if (t == -2) return fail(h, AM_ERR_NOT_SPD, "A: nonpositive diagonal at " + at);
    if (std::memcmp(&a, &b, sizeof(double)) != 0 && !(a == 0.0 && b == 0.0))
      return fail(h, AM_ERR_NOT_SYMMETRIC, "A not symmetric at " + at);
    if (a > 0) return fail(h, AM_ERR_POSITIVE_COUPLING, "positive off-diagonal at " + at);
    return fail(h, AM_ERR_ARG, "A: the nonzero couplings between subdomains must stay those of the "
                               "set-up (entry " + at + ")");
  }
  // Algorithm 1's numeric part on the new values
  h->numeric_ok = false;
  HCHK(launch_place_values(d, vm, v, st));
  const size_t esz = d.prec == AM_FP64 ? 8 : (d.prec == AM_FP32 ? 4 : 2);
  const size_t nfac = (size_t)h->lp.fac_off[h->st.m];
  void* Lr = nullptr;
  HCHK(hipMalloc(&Lr, nfac * esz));
  d.Lr = Lr;
  hipError_t he = hipMemsetAsync(d.Lc, 0, nfac * esz, st);
  if (he == hipSuccess) he = hipMemsetAsync(Lr, 0, nfac * esz, st);
  if (he == hipSuccess) he = hipMemsetAsync(d.fail, 0xFF, 4 * sizeof(int32_t), st);
  if (he == hipSuccess) he = launch_band_factor(d, st);
  if (he == hipSuccess) he = launch_mbf(d, st);
  if (he == hipSuccess) he = launch_invert_diag(d, st);
  if (he == hipSuccess) he = launch_assemble_S(d, st);
  if (he == hipSuccess && d.NL > 0) he = interface_inverse(d, st);
  const hipError_t he3 = hipStreamSynchronize(st);
  if (he == hipSuccess) he = he3;
  (void)hipFree(Lr);
  d.Lr = nullptr;
  HCHK(he);
  int32_t fl[4];
  HCHK(hipMemcpy(fl, d.fail, sizeof(fl), hipMemcpyDeviceToHost));
  if (fl[0] >= 0)
    return fail(h, AM_ERR_NOT_SPD, "A_i not SPD: subdomain " + std::to_string(fl[0]) + " pivot " +
                                       std::to_string(fl[1]));
  if (fl[2] >= 0)
    return fail(h, AM_ERR_NOT_SPD,
                "interface matrix S not SPD at row " + std::to_string(iface_fail_row(d, fl[2])));
  h->numeric_ok = true;
  return AM_OK;
}

am_status algmortar_set_inexact(am_handle h, double rtol, int32_t maxit) {
  if (!h) return fail(nullptr, AM_ERR_ARG, "null handle");
  if (!h->d.ix.on) return fail(h, AM_ERR_ARG, "the handle was not set up with AM_FLAG_INEXACT_IFACE");
  if (!(rtol >= 0.0 && rtol < 1.0) || maxit < 1 || maxit > 1000)
    return fail(h, AM_ERR_ARG, "rtol must be in [0, 1) and maxit in [1, 1000]");
  h->d.ix.rtol = rtol;
  h->d.ix.maxit = maxit;
  h->d.graph_nrhs = 0;  // the captured chunks hold the old launch sequence
  return AM_OK;
}

am_status algmortar_set_smoother(am_handle h, const int32_t* blocks, int32_t nblocks,
                                 int32_t steps, void* stream) {
  if (!h) return fail(nullptr, AM_ERR_ARG, "null handle");
  if (steps < 0 || steps > 1000) return fail(h, AM_ERR_ARG, "steps must be in [0, 1000]");
  DeviceState& d = h->d;
  HCHK(hipSetDevice(d.device));
  // applies on any stream may still read the old smoother's buffers
  HCHK(hipDeviceSynchronize());
  (void)stream;
  drop_smoother(h);
  d.graph_nrhs = 0;  // the captured chunks hold the old launch sequence
  if (steps == 0) return AM_OK;
  if (!blocks) return fail(h, AM_ERR_ARG, "null block partition");
  std::string e;
  am_status s = validate_partition(d.n, blocks, nblocks, e);
  if (s != AM_OK) return fail(h, s, e);
  // A in the original order, from the device copy (ELL rows in device order;
  // padding entries sit on the row's own column with value 0, which the
  // positive diagonal never has)
  const int64_t n = d.n;
  const int32_t w = d.ell_w;
  std::vector<int32_t> ec((size_t)w * n);
  std::vector<double> ev((size_t)w * n);
  HCHK(hipMemcpy(ec.data(), d.ell_col, sizeof(int32_t) * ec.size(), hipMemcpyDeviceToHost));
  HCHK(hipMemcpy(ev.data(), d.ell_val, sizeof(double) * ev.size(), hipMemcpyDeviceToHost));
  const std::vector<int32_t>& dperm = h->lp.dperm;
  const std::vector<int32_t>& dpos = h->lp.dpos;
  std::vector<int64_t> rp((size_t)n + 1, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t c = 0; c < w; ++c) {
      const int32_t col = ec[(size_t)c * n + i];
      if (!(col == i && ev[(size_t)c * n + i] == 0.0)) rp[dperm[i] + 1] += 1;
    }
  for (int64_t o = 0; o < n; ++o) rp[o + 1] += rp[o];
  std::vector<int32_t> ci((size_t)rp[n]);
  std::vector<double> cv((size_t)rp[n]);
  {
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t i = 0; i < n; ++i) {
      row.clear();
      for (int32_t c = 0; c < w; ++c) {
        const int32_t col = ec[(size_t)c * n + i];
        const double v = ev[(size_t)c * n + i];
        if (!(col == i && v == 0.0)) row.emplace_back(dperm[col], v);
      }
      std::sort(row.begin(), row.end(),
                [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
                  return a.first < b.first;
                });
      const int64_t o = dperm[i];
      for (size_t t = 0; t < row.size(); ++t) {
        ci[rp[o] + t] = row[t].first;
        cv[rp[o] + t] = row[t].second;
      }
    }
  }
  am_csr A{n, rp[n], rp.data(), ci.data(), cv.data(), 0};
  am_options o = h->opt;
  o.mortar = AM_MORTAR_PER_INTERFACE;
  am_handle bj = nullptr;
  s = setup_impl(&A, blocks, nblocks, &o, nullptr, &bj, true);
  if (s != AM_OK) return fail(h, s, std::string("smoothing blocks: ") + algmortar_last_error(nullptr));
  h->bj = bj;
  std::vector<int32_t> to_bj((size_t)n), to_am((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    to_bj[i] = dpos[bj->lp.dperm[i]];
    to_am[i] = bj->lp.dpos[dperm[i]];
  }
  int32_t *d_to_bj = nullptr, *d_to_am = nullptr;
  double *t_am = nullptr, *w_am = nullptr;
  auto grab = [&](void** p, size_t bytes) -> hipError_t {
    hipError_t he = hipMalloc(p, bytes);
    if (he == hipSuccess) h->sm_allocs.push_back(*p);
    return he;
  };
  const size_t nv = (size_t)n * d.max_nrhs;
  hipError_t he;
  if ((he = grab((void**)&d_to_bj, sizeof(int32_t) * n)) != hipSuccess ||
      (he = grab((void**)&d_to_am, sizeof(int32_t) * n)) != hipSuccess ||
      (he = grab((void**)&t_am, sizeof(double) * nv)) != hipSuccess ||
      (he = grab((void**)&w_am, sizeof(double) * nv)) != hipSuccess ||
      (he = hipMemcpy(d_to_bj, to_bj.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice)) != hipSuccess ||
      (he = hipMemcpy(d_to_am, to_am.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice)) != hipSuccess) {
    drop_smoother(h);
    return fail(h, he == hipErrorOutOfMemory ? AM_ERR_OOM : AM_ERR_HIP,
                std::string("smoother buffers: ") + hipGetErrorString(he));
  }
  h->sm.bj = &bj->d;
  h->sm.steps = steps;
  h->sm.to_bj = d_to_bj;
  h->sm.to_am = d_to_am;
  h->sm.t_am = t_am;
  h->sm.w_am = w_am;
  return AM_OK;
}

am_status algmortar_apply(am_handle h, const double* r, double* z, int32_t nrhs, int64_t ld,
                          void* stream) {
  am_status s = check_vec_args(h, r, z, nrhs, ld);
  if (s != AM_OK) return s;
  if (nrhs == 1) ld = h->d.n;
  DeviceState& d = h->d;
  HCHK(hipSetDevice(d.device));
  hipStream_t st = (hipStream_t)stream;
  const int nr = pow2_at_least(nrhs);
  if (d.tile_cand[tile_slot(nr)] < 0) {
    HCHK(hipStreamSynchronize(st));
    am_status ts = autotune_tiles(h, nr);
    if (ts != AM_OK) return ts;
  }
  if (h->sm.steps > 0 && h->bj->d.tile_cand[tile_slot(nr)] < 0) {
    HCHK(hipStreamSynchronize(st));
    am_status ts = autotune_tiles(h->bj, nr);
    if (ts != AM_OK) return fail(h, ts, h->bj->err);
  }
  HCHK(launch_permute_in(d.dperm, d.n, r, ld, d.r, nrhs, st));
  if (h->sm.steps > 0) {
    HCHK(launch_smoothed_apply(d, h->sm, d.r, d.z, nr, st));
  } else {
    if (d.NL > 0) {
      HCHK(launch_bpart(d, d.r, nr, st));
      if (!d.fuse_eta) HCHK(launch_iface_gemv(d, nr, 0, 0, st));
    }
    HCHK(launch_local_sweep(d, d.r, d.z, d.eta, nr, 1, st));
  }
  HCHK(launch_permute_out(d.dperm, d.n, d.z, z, ld, nrhs, st));
  return AM_OK;
}

// Scratch layout of algmortar_apply_static inside the static array: the
// permuted input and output (n x nr each), the interface slots (2 NL x nr),
// eta (ldS x nr) and, when the interface solve is its own launches, the
// row-part sums (op_parts x ldS x nr); each piece starts on a 256-byte
// boundary.  Returns the doubles needed.
static int64_t static_layout(const DeviceState& d, int nr, double* base, double** r, double** z,
                             double** bpart, double** eta, double** ypart, double** y1 = nullptr,
                             double** eta2 = nullptr) {
  int64_t off = 0;
  auto take = [&](int64_t count, double** out) {
    if (out) *out = base ? base + off : nullptr;
    off += (count + 31) / 32 * 32;
  };
  // (the dissection form: y_B, eta_T and its part sums)
  take(d.n * nr, r);
  take(d.n * nr, z);
  if (d.NL > 0) {
    take(2 * d.NL * nr, bpart);
    take((int64_t)d.ldS * nr, eta);
    if (d.nd.on) {
      take(std::max<int64_t>(d.nd.nrows, 1) * nr, y1);
      take((int64_t)std::max<int32_t>(d.nd.R, 1) * nr, eta2);
      take((int64_t)d.nd.P * std::max<int32_t>(d.nd.ldC, 1) * nr, ypart);
    } else if (!d.fuse_eta) {
      take((int64_t)d.op_parts * d.ldS * nr, ypart);
    }
  }
  return off;
}

am_status algmortar_apply_static(am_handle h, const double* r, double* z, int32_t nrhs, int64_t ld,
                                 void* stream) {
  am_status s = check_vec_args(h, r, z, nrhs, ld);
  if (s != AM_OK) return s;
  if (nrhs == 1) ld = h->d.n;
  if (h->sm.steps > 0)
    return fail(h, AM_ERR_UNSUPPORTED, "algmortar_apply_static does not cover block-Jacobi smoothing");
  if (h->d.ix.on)
    return fail(h, AM_ERR_UNSUPPORTED, "algmortar_apply_static does not cover the inexact interface solve");
  DeviceState& d = h->d;
  const int nr = pow2_at_least(nrhs);
  const int64_t need = static_layout(d, nr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  if (need > kStaticScratchDoubles)
    return fail(h, AM_ERR_ARG,
                "algmortar_apply_static needs " + std::to_string(need * 8) +
                    " bytes of scratch for this handle and nrhs; its static scratch holds " +
                    std::to_string(kStaticScratchDoubles * 8) + " bytes");
  HCHK(hipSetDevice(d.device));
  double* base = static_scratch_ptr(d.device);
  if (!base) {  // first use on this device: the set-up's look-up did not succeed
    HCHK(static_scratch_init(d.device));
    base = static_scratch_ptr(d.device);
    if (!base) return fail(h, AM_ERR_HIP, "no address for the static scratch on this device");
  }
  hipStream_t st = (hipStream_t)stream;
  if (d.tile_cand[tile_slot(nr)] < 0) {
    HCHK(hipStreamSynchronize(st));
    am_status ts = autotune_tiles(h, nr);
    if (ts != AM_OK) return ts;
  }
  double *sr, *sz, *sb = nullptr, *se = nullptr, *sy = nullptr, *s1 = nullptr, *s2 = nullptr;
  static_layout(d, nr, base, &sr, &sz, &sb, &se, &sy, &s1, &s2);
  // the launchers read the work buffers from the handle's state: point them
  // at the static scratch for this call and put the handle's own back after
  struct Swap {
    DeviceState& d;
    double *r, *z, *bpart, *eta, *ypart, *y1, *eta2, *ndpart;
    ~Swap() {
      d.r = r;
      d.z = z;
      d.bpart = bpart;
      d.eta = eta;
      d.ypart = ypart;
      d.nd.y1 = y1;
      d.nd.eta2 = eta2;
      d.nd.ypart = ndpart;
    }
  } keep{d, d.r, d.z, d.bpart, d.eta, d.ypart, d.nd.y1, d.nd.eta2, d.nd.ypart};
  d.r = sr;
  d.z = sz;
  if (d.NL > 0) {
    d.bpart = sb;
    d.eta = se;
    if (d.nd.on) {
      d.nd.y1 = s1;
      d.nd.eta2 = s2;
      d.nd.ypart = sy;
    } else if (!d.fuse_eta) {
      d.ypart = sy;
    }
  }
  // columns nrhs .. nr-1 of the padded block: zeros (the array keeps the last
  // call's contents)
  if (nrhs < nr) HCHK(launch_fill(d.r, d.n * nr, 0.0, st));
  HCHK(launch_permute_in(d.dperm, d.n, r, ld, d.r, nrhs, st));
  if (d.NL > 0) {
    HCHK(launch_bpart(d, d.r, nr, st));
    if (!d.fuse_eta) HCHK(launch_iface_gemv(d, nr, 0, 0, st));
  }
  HCHK(launch_local_sweep(d, d.r, d.z, d.eta, nr, 1, st));
  HCHK(launch_permute_out(d.dperm, d.n, d.z, z, ld, nrhs, st));
  return AM_OK;
}

am_status algmortar_local_solve(am_handle h, const double* r, double* pbar, void* stream) {
  am_status s = check_vec_args(h, r, pbar, 1, 0);
  if (s != AM_OK) return s;
  DeviceState& d = h->d;
  HCHK(hipSetDevice(d.device));
  hipStream_t st = (hipStream_t)stream;
  HCHK(launch_permute_in(d.dperm, d.n, r, d.n, d.r, 1, st));
  HCHK(launch_local_sweep(d, d.r, d.z, d.eta, 1, 0, st));
  HCHK(launch_permute_out(d.dperm, d.n, d.z, pbar, d.n, 1, st));
  return AM_OK;
}

static constexpr int kChunk = 8;  // iterations per captured graph (even: p ping-pong)

// One PCG iteration of the smoothed preconditioner: the smoothed apply (some
// 4 nu + 10 launches), the (r, z), (q, z) partials, the SpMV, the update and
// the stop test.  After the stop, the apply and the partials still run (on
// the stopped r, into z and the partials, which nothing reads any more);
// the SpMV, update and stop test return at once.
static hipError_t smoothed_iteration(DeviceState& d, SmoothDevice& sm, int nr, int parity,
                                     hipStream_t st) {
  hipError_t e = launch_smoothed_apply(d, sm, d.r, d.z, nr, st);
  if (e == hipSuccess) e = launch_smooth_dots(d, nr, st);
  if (e == hipSuccess) e = launch_pcg_spmv(d, nr, parity, st);
  if (e == hipSuccess) e = launch_pcg_update(d, nr, parity, st);
  if (e == hipSuccess) e = launch_stop_test(d, nr, 0, st);
  return e;
}

// len iterations (even: the p ping-pong keeps its parity), smoothed when sm
// is given
static hipError_t run_chunk(DeviceState& d, int nr, hipStream_t st, int len = kChunk,
                            SmoothDevice* sm = nullptr) {
  for (int it = 0; it < len; ++it) {
    hipError_t e = sm ? smoothed_iteration(d, *sm, nr, it & 1, st)
                      : launch_pcg_iteration(d, nr, it & 1, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Per-kernel event timing of a profiled solve: launch kinds as in
// algmortar_time_kernel (0 local, 1 gemv, 3 spmv, 4 update).
struct KernelProfile {
  double ms[5] = {0, 0, 0, 0, 0};
  int64_t launches[5] = {0, 0, 0, 0, 0};
};

// One PCG iteration with every launch bracketed by events; the stop flag is
// read after each iteration so that no launch after convergence is timed.
static hipError_t profiled_iteration(am_handle h, int nr, int parity, KernelProfile& kp, bool& done) {
  DeviceState& d = h->d;
  hipStream_t st = h->own;
  for (int i = 0; i < 8; ++i)
    if (!h->evp[i]) {
      hipError_t e = hipEventCreate(&h->evp[i]);
      if (e != hipSuccess) return e;
    }
  int kinds[4];
  int nk = 0;
  hipError_t e;
  // each operation's first and last launch carry the two events of its slot
  // (the dispatches' own start and end); an operation that launched nothing
  // gets them recorded in place (zero time)
  auto timed = [&](int kind, auto&& fn) -> hipError_t {
    d.prof_ev[0] = h->evp[2 * nk];
    d.prof_ev[1] = h->evp[2 * nk + 1];
    d.prof_used[0] = d.prof_used[1] = false;
    hipError_t r = fn();
    d.prof_ev[0] = d.prof_ev[1] = nullptr;
    if (r != hipSuccess) return r;
    if (!d.prof_used[0] && (r = hipEventRecord(h->evp[2 * nk], st)) != hipSuccess) return r;
    if (!d.prof_used[1] && (r = hipEventRecord(h->evp[2 * nk + 1], st)) != hipSuccess) return r;
    kinds[nk++] = kind;
    return hipSuccess;
  };
  if ((e = timed(3, [&] { return launch_pcg_spmv(d, nr, parity, st); })) != hipSuccess) return e;
  if ((e = timed(4, [&] { return launch_pcg_update(d, nr, parity, st); })) != hipSuccess) return e;
  if (!d.fuse_eta && (e = timed(1, [&] { return launch_iface_gemv(d, nr, 1, 0, st); })) != hipSuccess)
    return e;
  if ((e = timed(0, [&] { return launch_local_sweep(d, d.r, d.z, d.eta, nr, 2, st); })) != hipSuccess)
    return e;
  int32_t flag = 0;
  if ((e = hipMemcpyAsync(&flag, &d.shared->all_done, sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  // the iteration whose local launch took the stop decision ran that launch
  // as an early exit: none of its launches are counted
  if (!flag) {
    for (int i = 0; i < nk; ++i) {
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, h->evp[2 * i], h->evp[2 * i + 1])) != hipSuccess) return e;
      kp.ms[kinds[i]] += ms;
      kp.launches[kinds[i]] += 1;
    }
  }
  done = flag != 0;
  return hipSuccess;
}

static am_status pcg_impl(am_handle h, const double* b, double* x, int32_t nrhs, int64_t ld,
                          double tol, int32_t maxit, am_info* info, void* stream,
                          KernelProfile* prof);

am_status algmortar_pcg(am_handle h, const double* b, double* x, int32_t nrhs, int64_t ld,
                        double tol, int32_t maxit, am_info* info, void* stream) {
  return pcg_impl(h, b, x, nrhs, ld, tol, maxit, info, stream, nullptr);
}

am_status algmortar_pcg_profile(am_handle h, const double* b, double* x, int32_t nrhs, int64_t ld,
                                double tol, int32_t maxit, am_info* info, double* kernel_ms,
                                int64_t* launches, void* stream) {
  if (!kernel_ms || !launches) return fail(h, AM_ERR_ARG, "null profile output");
  KernelProfile kp;
  am_status s = pcg_impl(h, b, x, nrhs, ld, tol, maxit, info, stream, &kp);
  for (int k = 0; k < 5; ++k) {
    kernel_ms[k] = kp.ms[k];
    launches[k] = kp.launches[k];
  }
  return s;
}

static am_status pcg_impl(am_handle h, const double* b, double* x, int32_t nrhs, int64_t ld,
                          double tol, int32_t maxit, am_info* info, void* stream,
                          KernelProfile* prof) {
  am_status s = check_vec_args(h, b, x, nrhs, ld);
  if (s != AM_OK) return s;
  if (!(tol > 0.0) || !(tol < 1.0)) return fail(h, AM_ERR_ARG, "tol must be in (0, 1)");
  if (maxit <= 0) maxit = 10000;
  const bool smooth = h->sm.steps > 0;
  if (smooth && prof)
    return fail(h, AM_ERR_UNSUPPORTED, "the profiled solve does not cover block-Jacobi smoothing");
  if (nrhs == 1) ld = h->d.n;
  DeviceState& d = h->d;
  HCHK(hipSetDevice(d.device));
  // b is read on h->own, a non-blocking stream: wait for the caller's stream
  // (NULL: the null stream, e.g. torch's default stream) to finish writing it
  HCHK(hipStreamSynchronize((hipStream_t)stream));
  hipStream_t st = h->own;
  const int nr = pow2_at_least(nrhs);
  const int64_t nv = d.n * nr;
  {
    am_status ts = autotune_tiles(h, nr);
    if (ts != AM_OK) return ts;
    if (smooth && (ts = autotune_tiles(h->bj, nr)) != AM_OK) return fail(h, ts, h->bj->err);
  }
  HCHK(hipEventRecord(h->ev0, st));
  HCHK(launch_permute_in(d.dperm, d.n, b, ld, d.r, nrhs, st));
  HCHK(launch_permute_in(d.dperm, d.n, b, ld, h->bp, nrhs, st));
  HCHK(launch_fill(d.x, nv, 0.0, st));
  HCHK(launch_fill(d.z, nv, 0.0, st));
  HCHK(launch_fill(d.q, nv, 0.0, st));
  HCHK(launch_fill(d.p[0], nv, 0.0, st));
  HCHK(launch_fill(d.p[1], nv, 0.0, st));
  HCHK(launch_fill(d.eta, (int64_t)std::max<int32_t>(d.ldS, 1) * nr, 0.0, st));
  // the flexible beta where the preconditioner is not a fixed symmetric
  // operator: reduced-precision factors, an interface solve stopped by a
  // tolerance
  HCHK(launch_pcg_init(d, nr, tol, maxit, (d.prec != AM_FP64 || d.ix.on) ? 1 : 0, st));
  // The smoothed preconditioner runs the same chunks of iterations, its
  // iteration being smoothed_iteration; its first residual norm and stop
  // test come from the update launch in its initial form.
  SmoothDevice* smp = smooth ? &h->sm : nullptr;
  if (smooth) {
    HCHK(launch_pcg_rr0(d, nr, st));
    HCHK(launch_stop_test(d, nr, 1, st));
  } else {
    HCHK(launch_pcg_start(d, nr, st));
  }
  {
  const bool use_graph = !(h->opt.flags & AM_FLAG_NO_GRAPH) && !prof;
  if (use_graph && (d.graph == nullptr || d.graph_nrhs != nr)) {
    // chunks of 8 iterations, and of 2, 4 and 6 for the end of a solve
    hipGraphExec_t* slots[4] = {&d.graph, &d.graph_short[0], &d.graph_short[1], &d.graph_short[2]};
    const int lens[4] = {kChunk, 2, 4, 6};
    for (int i = 0; i < 4; ++i) {
      if (*slots[i]) {
        HCHK(hipGraphExecDestroy(*slots[i]));
        *slots[i] = nullptr;
      }
    }
    d.graph_nrhs = 0;
    for (int i = 0; i < 4; ++i) {
      hipGraph_t g = nullptr;
      HCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      hipError_t ce = run_chunk(d, nr, st, lens[i], smp);
      hipError_t ee = hipStreamEndCapture(st, &g);
      if (ce != hipSuccess) return fail(h, AM_ERR_HIP, std::string("capture: ") + hipGetErrorString(ce));
      if (ee != hipSuccess) return fail(h, AM_ERR_HIP, std::string("end capture: ") + hipGetErrorString(ee));
      hipError_t ie = hipGraphInstantiate(slots[i], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        *slots[i] = nullptr;
        return fail(h, AM_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
      }
    }
    d.graph_nrhs = nr;
  }
  // Chunks of up to kChunk iterations (even lengths keep the p ping-pong
  // aligned).  The scalars of chunk c are copied to pinned memory behind it
  // and read while chunk c + 1 runs; a chunk launched after convergence runs
  // only early-exit launches.  From the relative residuals seen at the ends
  // of chunks the host predicts the iterations still needed (per column, at
  // the rate of the last chunk, plus a margin of 2) and shortens the last
  // chunks to that, or launches nothing until the running chunk is read when
  // it is predicted to converge.  Only the number of early-exit launches
  // depends on this, never the arithmetic of an iteration.
  const int limit = (maxit / kChunk + 2) * kChunk;
  if (prof) {
    bool done = false;
    for (int it = 0; it < limit && !done; ++it)
      HCHK(profiled_iteration(h, nr, it & 1, *prof, done));
  }
  if (!prof) {
    int prev_it[kMaxNRHS], last_it[kMaxNRHS];
    double prev_r[kMaxNRHS], last_r[kMaxNRHS];
    bool col_done[kMaxNRHS];
    for (int k = 0; k < kMaxNRHS; ++k) {
      prev_it[k] = last_it[k] = -1;
      prev_r[k] = last_r[k] = 0.0;
      col_done[k] = false;
    }
    int launched = 0, inflight = 0, c_launch = 0, c_read = 0;
    bool done = false;
    // reads the oldest chunk in flight: its stop state and residuals
    auto read_oldest = [&]() -> hipError_t {
      const int slot = c_read & 1;
      hipError_t e = hipEventSynchronize(h->evf[slot]);
      if (e != hipSuccess) return e;
      ++c_read;
      --inflight;
      const PcgScalars* S = d.h_sc + (size_t)slot * kMaxNRHS;
      bool all = true;
      for (int k = 0; k < nrhs; ++k) {
        col_done[k] = S[k].done != 0;
        if (col_done[k]) continue;
        all = false;
        if (S[k].it != last_it[k]) {
          prev_it[k] = last_it[k];
          prev_r[k] = last_r[k];
          last_it[k] = S[k].it;
          last_r[k] = S[k].bb > 0.0 ? S[k].rr / S[k].bb : 0.0;
        }
      }
      done = all;
      return hipSuccess;
    };
    // iterations still needed beyond those launched; -1 when not predictable
    auto remaining = [&]() -> int {
      int need = -1;
      for (int k = 0; k < nrhs; ++k) {
        if (col_done[k]) continue;
        if (last_it[k] < 0 || prev_it[k] < 0 || !(last_r[k] > 0.0) || !(prev_r[k] > last_r[k]))
          return -1;  // a column with no usable history (or not reducing)
        const double t2 = (double)tol * (double)tol;
        double left = 0.0;
        if (last_r[k] > t2) {
          const double rate = std::log(last_r[k] / prev_r[k]) / (last_it[k] - prev_it[k]);
          left = std::min(std::ceil(std::log(t2 / last_r[k]) / rate), 1e6);
        }
        need = std::max(need, last_it[k] + (int)left + 2 - launched);
      }
      return std::max(need, 0);
    };
    while (launched < limit) {
      int len = kChunk;
      const int rem = remaining();
      if (rem >= 0 && rem < kChunk) len = (rem + 1) & ~1;  // even, at most kChunk
      if (len == 0) {
        if (inflight > 0) {  // predicted to converge in a chunk in flight: read it first
          HCHK(read_oldest());
          if (done) break;
          continue;
        }
        len = 2;
      }
      len = std::min(len, limit - launched);
      if (use_graph)
        HCHK(hipGraphLaunch(len == kChunk ? d.graph : d.graph_short[len / 2 - 1], st));
      else
        HCHK(run_chunk(d, nr, st, len, smp));
      const int slot = c_launch & 1;
      HCHK(hipMemcpyAsync(d.h_sc + (size_t)slot * kMaxNRHS, d.sc, sizeof(PcgScalars) * nr,
                          hipMemcpyDeviceToHost, st));
      HCHK(hipEventRecord(h->evf[slot], st));
      ++c_launch;
      ++inflight;
      launched += len;
      if (inflight == 2) {
        HCHK(read_oldest());
        if (done) break;
      }
    }
  }
  }
  HCHK(launch_permute_out(d.dperm, d.n, d.x, x, ld, nrhs, st));
  HCHK(hipEventRecord(h->ev1, st));
  HCHK(launch_true_residual(d, h->bp, nr, h->tres, st));
  PcgScalars sc[kMaxNRHS];
  double tr[kMaxNRHS];
  HCHK(hipMemcpyAsync(sc, d.sc, sizeof(PcgScalars) * nr, hipMemcpyDeviceToHost, st));
  HCHK(hipMemcpyAsync(tr, h->tres, sizeof(double) * nr, hipMemcpyDeviceToHost, st));
  HCHK(hipStreamSynchronize(st));
  float ms = 0.f;
  HCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  am_status ret = AM_OK;
  for (int k = 0; k < nrhs; ++k) {
    const double bb = sc[k].bb;
    if (info) {
      info[k].iterations = sc[k].it;
      info[k].converged = sc[k].conv;
      info[k].rel_res = bb > 0 ? std::sqrt(sc[k].rr / bb) : 0.0;
      info[k].true_rel_res = bb > 0 ? std::sqrt(tr[k] / bb) : 0.0;
      info[k].solve_ms = ms;
    }
    if (!sc[k].done && ret == AM_OK) ret = AM_ERR_NO_CONVERGENCE;
    if (sc[k].status == AM_ERR_BREAKDOWN) ret = AM_ERR_BREAKDOWN;
    else if (sc[k].status == AM_ERR_NO_CONVERGENCE && ret == AM_OK) ret = AM_ERR_NO_CONVERGENCE;
  }
  if (ret == AM_ERR_BREAKDOWN) return fail(h, ret, "PCG breakdown: nonpositive curvature");
  if (ret == AM_ERR_NO_CONVERGENCE) return fail(h, ret, "PCG did not converge within maxit");
  return AM_OK;
}

am_status algmortar_interfaces(am_handle h, int32_t* perm, int64_t* sub_ptr, int64_t* iface_ptr,
                               int32_t* iface_ij, int32_t* edge_k, int32_t* edge_l) {
  if (!h) return fail(nullptr, AM_ERR_ARG, "null handle");
  copy_structure(h->st, perm, sub_ptr, iface_ptr, iface_ij, edge_k, edge_l);
  return AM_OK;
}

am_status algmortar_sizes(am_handle h, int64_t* n, int64_t* nparts, int64_t* n_iface,
                          int64_t* n_edges) {
  if (!h) return fail(nullptr, AM_ERR_ARG, "null handle");
  if (n) *n = h->d.n;
  if (nparts) *nparts = h->d.m;
  if (n_iface) *n_iface = h->d.NL;
  if (n_edges) *n_edges = h->d.NE;
  return AM_OK;
}

am_status algmortar_export_interface(am_handle h, int32_t which, double* out) {
  if (!h || !out || (which != 0 && which != 1)) return fail(h, AM_ERR_ARG, "bad argument");
  DeviceState& d = h->d;
  if (d.NL == 0) return AM_OK;
  HCHK(hipSetDevice(d.device));
  if (which == 1 && d.nd.on) {  // the reordered inverse of the dissection form
    const int64_t ldp = d.nd.ldp;
    std::vector<double> tmp((size_t)ldp * ldp);
    HCHK(hipMemcpy(tmp.data(), d.Sinv, sizeof(double) * tmp.size(), hipMemcpyDeviceToHost));
    std::vector<int64_t> pos((size_t)d.NL);
    for (int64_t a = 0; a < ldp; ++a)
      if (d.nd.h_src[a] >= 0) pos[d.nd.h_src[a]] = a;
    for (int64_t i = 0; i < d.NL; ++i)
      for (int64_t j = 0; j < d.NL; ++j) out[i * d.NL + j] = tmp[(size_t)pos[i] * ldp + pos[j]];
    return AM_OK;
  }
  const double* src = which == 0 ? d.S : d.Sinv;
  HCHK(hipMemcpy2D(out, sizeof(double) * d.NL, src, sizeof(double) * d.ldS, sizeof(double) * d.NL,
                   d.NL, hipMemcpyDeviceToHost));
  return AM_OK;
}

am_status algmortar_export_mbf(am_handle h, int64_t iface, int32_t sub, double* out) {
  if (!h || !out || iface < 0 || iface >= h->d.NL) return fail(h, AM_ERR_ARG, "bad argument");
  const Structure& st = h->st;
  if (st.iface_ij[2 * iface] != sub && st.iface_ij[2 * iface + 1] != sub)
    return fail(h, AM_ERR_ARG, "subdomain is not a side of the interface");
  int64_t q = -1;
  for (int64_t pi = st.isub_ptr[sub]; pi < st.isub_ptr[sub + 1]; ++pi)
    if (st.isub_list[pi] == iface) q = pi - st.isub_ptr[sub];
  int64_t off = 0;
  for (int32_t s2 = 0; s2 < sub; ++s2)
    off += (st.isub_ptr[s2 + 1] - st.isub_ptr[s2]) * (st.sub_ptr[s2 + 1] - st.sub_ptr[s2]);
  const int64_t N = st.sub_ptr[sub + 1] - st.sub_ptr[sub];
  std::vector<double> tmp((size_t)N);
  HCHK(hipSetDevice(h->d.device));
  HCHK(hipMemcpy(tmp.data(), h->d.mbf + off + q * N, sizeof(double) * N, hipMemcpyDeviceToHost));
  for (int64_t r = 0; r < N; ++r) {
    const int32_t o = st.perm[st.sub_ptr[sub] + r];
    out[r] = tmp[h->lp.dpos[o] - st.sub_ptr[sub]];
  }
  return AM_OK;
}

am_status algmortar_time_kernel(am_handle h, int32_t kernel, int32_t nrhs, int32_t reps,
                                double* avg_ms, double* bytes) {
  if (!h || !avg_ms || !bytes || reps < 1 || kernel < 0 || kernel > 5 || nrhs < 1 ||
      pow2_at_least(nrhs) > h->d.max_nrhs)
    return fail(h, AM_ERR_ARG, "bad argument");
  if (kernel == 5) {  // the smoother's block solves: kernel 0 of the block factors
    if (!h->bj) return fail(h, AM_ERR_ARG, "no smoother is set");
    HCHK(hipSetDevice(h->d.device));
    am_status ts = autotune_tiles(h->bj, pow2_at_least(nrhs));
    if (ts == AM_OK) ts = algmortar_time_kernel(h->bj, 0, nrhs, reps, avg_ms, bytes);
    return ts == AM_OK ? AM_OK : fail(h, ts, h->bj->err);
  }
  if (kernel == 1 && (h->d.fuse_eta || (!h->d.nd.on && !h->d.ix.on && h->d.ypart == nullptr)))
    return fail(h, AM_ERR_ARG,
                "the interface solve of this handle runs inside the local kernel (kernel 0)");
  DeviceState& d = h->d;
  const Structure& st = h->st;
  const LocalPlan& lp = h->lp;
  const int nr = pow2_at_least(nrhs);
  const double esz = d.prec == AM_FP64 ? 8 : (d.prec == AM_FP32 ? 4 : 2);
  const double isz = d.prec == AM_FP64 ? 8 : 4;
  double by = 0.0;
  if (kernel == 0) {
    for (int32_t s2 = 0; s2 < st.m; ++s2) {
      const double N = (double)(st.sub_ptr[s2 + 1] - st.sub_ptr[s2]);
      const double NP = (double)(lp.roff[s2 + 1] - lp.roff[s2]);
      const double ns = (double)(st.isub_ptr[s2 + 1] - st.isub_ptr[s2]);
      by += 2.0 * NP * lp.wp[s2] * esz + 2.0 * NP * isz + 2.0 * N * 8.0 * nr + ns * N * 8.0;
    }
    by += (double)d.NL * 8.0 * nr;
    // with the interface solve fused in, its operator S^{-1} (once) and the
    // interface partial right-hand sides
    if (d.fuse_eta) by += (double)d.NL * d.NL * 8.0 + 2.0 * d.NL * 8.0 * nr;
  } else if (kernel == 1 && d.nd.on) {
    // the block inverses (twice when there are top rows), C^{-1} once, the
    // coupling values and indices, the slots (read by both block passes and
    // the top product), y_B and the part sums written and read, eta
    const NdDevice& nd = d.nd;
    double blocks = 0.0;
    for (int b = 0; b < nd.nblk; ++b) {
      const double sb = (double)(nd.h_blk_off[b + 1] - nd.h_blk_off[b]);
      blocks += sb * sb * 8.0;
    }
    by = (nd.R > 0 ? 2.0 : 1.0) * blocks + (double)nd.R * nd.ldC * 8.0 +
         12.0 * (double)(nd.nt_pairs + nd.nb_pairs) + 3.0 * 2.0 * d.NL * 8.0 * nr +
         2.0 * (double)nd.nrows * 8.0 * nr + 2.0 * (double)nd.P * nd.ldC * 8.0 * nr +
         (double)d.NL * 8.0 * nr + 2.0 * nd.R * 8.0 * nr;
  } else if (kernel == 1 && d.ix.on) {
    // the inexact solve at its iteration cap: the first pass (slots, block
    // inverses, r, z, eta) and per inner iteration S (ELL values and
    // columns), the block inverses and the vectors it reads and writes
    const IxDevice& ix = d.ix;
    double blocks = 0.0;
    for (int b = 0; b < ix.nblk; ++b) {
      const double sb = (double)std::min<int64_t>(ix.bs, d.NL - (int64_t)b * ix.bs);
      blocks += sb * sb * 8.0;
    }
    const double vec = (double)d.NL * 8.0 * nr;
    by = blocks + 5.0 * vec + ix.maxit * (12.0 * ix.w * d.NL + blocks + 9.0 * vec);
  } else if (kernel == 1) {
    // S^{-1} once, the interface slots, the part sums written and read, eta
    by = (double)d.NL * d.NL * 8.0 + 3.0 * d.NL * 8.0 * nr +
         2.0 * d.op_parts * d.ldS * 8.0 * nr;
  } else if (kernel == 3) {
    // ELL values and columns, z and p read, p and q written
    by = (double)d.n * d.ell_w * 12.0 + 4.0 * d.n * 8.0 * nr;
  } else if (kernel == 4) {
    // x, p, r, q read, x and r written, MBFs read
    by = 6.0 * d.n * 8.0 * nr;
    for (int32_t s2 = 0; s2 < st.m; ++s2)
      by += (double)(st.isub_ptr[s2 + 1] - st.isub_ptr[s2]) * (st.sub_ptr[s2 + 1] - st.sub_ptr[s2]) * 8.0;
  } else {
    for (int32_t s2 = 0; s2 < st.m; ++s2) {
      const double N = (double)(st.sub_ptr[s2 + 1] - st.sub_ptr[s2]);
      const double ns = (double)(st.isub_ptr[s2 + 1] - st.isub_ptr[s2]);
      by += ns * N * 8.0 + N * 8.0 * nr;
    }
    by += 2.0 * d.NL * 8.0 * nr;
  }
  HCHK(hipSetDevice(d.device));
  hipStream_t st0 = h->own;
  if (kernel >= 3) {  // PCG kernels: run them on a live (not stopped) state
    HCHK(launch_pcg_init(d, nr, 1e-300, 1 << 30, d.prec != AM_FP64 ? 1 : 0, st0));
  }
  auto launch = [&]() -> hipError_t {
    if (kernel == 0) return launch_local_sweep(d, d.r, d.z, d.eta, nr, 1, st0);
    if (kernel == 1) return launch_iface_gemv(d, nr, 0, 0, st0);
    if (kernel == 3) return launch_pcg_spmv(d, nr, 0, st0);
    if (kernel == 4) return launch_pcg_update(d, nr, 0, st0);
    return launch_bpart(d, d.r, nr, st0);
  };
  HCHK(launch());  // warm-up
  HCHK(hipEventRecord(h->ev0, st0));
  for (int i = 0; i < reps; ++i) HCHK(launch());
  HCHK(hipEventRecord(h->ev1, st0));
  HCHK(hipEventSynchronize(h->ev1));
  float ms = 0.f;
  HCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  *avg_ms = ms / reps;
  *bytes = by;
  return AM_OK;
}

// ---------------------------------------------------------------------------
am_status am_tpfa_create(const am_faces* f, int64_t n, int32_t device, am_tpfa* out,
                         int64_t* nnz) {
  if (!f || !out || n <= 0 || f->n_faces < 0 || (f->n_faces > 0 && (!f->k || !f->l || !f->gk || !f->gl || !f->pD)))
    return fail(nullptr, AM_ERR_ARG, "bad face list");
  *out = nullptr;
  const int64_t nf = f->n_faces;
  for (int64_t i = 0; i < nf; ++i) {
    if (f->k[i] < 0 || f->k[i] >= n || f->l[i] < -1 || f->l[i] >= n || f->l[i] == f->k[i])
      return fail(nullptr, AM_ERR_ARG, "face " + std::to_string(i) + " has a bad cell index");
    if (!(f->gk[i] > 0) || (f->l[i] >= 0 && !(f->gl[i] > 0)))
      return fail(nullptr, AM_ERR_ARG, "face " + std::to_string(i) + " has a nonpositive factor");
  }
  am_tpfa t = new am_tpfa_s();
  TpfaDevice& T = t->t;
  T.device = device;
  T.n = n;
  T.nf = nf;
  // pattern: diagonal + the other cell of every interior face, columns ascending
  std::vector<std::vector<int64_t>> cols((size_t)n);
  for (int64_t c = 0; c < n; ++c) cols[c].push_back(c);
  for (int64_t i = 0; i < nf; ++i)
    if (f->l[i] >= 0) {
      cols[f->k[i]].push_back(f->l[i]);
      cols[f->l[i]].push_back(f->k[i]);
    }
  T.h_rp.assign(n + 1, 0);
  for (int64_t c = 0; c < n; ++c) {
    std::sort(cols[c].begin(), cols[c].end());
    if (std::adjacent_find(cols[c].begin(), cols[c].end()) != cols[c].end()) {
      delete t;
      return fail(nullptr, AM_ERR_ARG, "two faces join the same pair of cells");
    }
    T.h_rp[c + 1] = T.h_rp[c] + (int64_t)cols[c].size();
  }
  T.nnz = T.h_rp[n];
  T.h_ci.resize((size_t)T.nnz);
  for (int64_t c = 0; c < n; ++c)
    for (size_t q = 0; q < cols[c].size(); ++q) T.h_ci[T.h_rp[c] + q] = (int32_t)cols[c][q];
  auto slot = [&](int64_t r, int64_t c) {
    const int32_t* b = T.h_ci.data() + T.h_rp[r];
    const int32_t* e = T.h_ci.data() + T.h_rp[r + 1];
    return T.h_rp[r] + (std::lower_bound(b, e, (int32_t)c) - b);
  };
  std::vector<int64_t> skk(n), skl(nf, 0), slk(nf, 0), cf_ptr(n + 1, 0);
  for (int64_t c = 0; c < n; ++c) skk[c] = slot(c, c);
  for (int64_t i = 0; i < nf; ++i) {
    cf_ptr[f->k[i] + 1]++;
    if (f->l[i] >= 0) {
      skl[i] = slot(f->k[i], f->l[i]);
      slk[i] = slot(f->l[i], f->k[i]);
      cf_ptr[f->l[i] + 1]++;
    }
  }
  for (int64_t c = 0; c < n; ++c) cf_ptr[c + 1] += cf_ptr[c];
  std::vector<int32_t> cf_face(cf_ptr[n]);
  {
    std::vector<int64_t> fill(cf_ptr.begin(), cf_ptr.end() - 1);
    for (int64_t i = 0; i < nf; ++i) {
      cf_face[fill[f->k[i]]++] = (int32_t)i;
      if (f->l[i] >= 0) cf_face[fill[f->l[i]]++] = (int32_t)i;
    }
  }
  am_handle h = nullptr;
  auto bail = [&](hipError_t e, const char* what) {
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    am_tpfa_destroy(t);
    return fail(nullptr, e == hipErrorOutOfMemory ? AM_ERR_OOM : AM_ERR_HIP, msg);
  };
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return bail(e, "hipSetDevice");
  std::vector<int64_t> fk(f->k, f->k + nf), fl(f->l, f->l + nf);
  std::vector<double> gk(f->gk, f->gk + nf), gl(f->gl, f->gl + nf), pD(f->pD, f->pD + nf);
  hipStream_t s0 = nullptr;
#define TUP(p, v)                         \
  do {                                    \
    e = upload(T.allocs, &p, v, s0);      \
    if (e != hipSuccess) return bail(e, #p); \
  } while (0)
  TUP(T.fk, fk);
  TUP(T.fl, fl);
  TUP(T.gk, gk);
  TUP(T.gl, gl);
  TUP(T.pD, pD);
  TUP(T.slot_kk, skk);
  TUP(T.slot_kl, skl);
  TUP(T.slot_lk, slk);
  TUP(T.cf_ptr, cf_ptr);
  TUP(T.cf_face, cf_face);
#undef TUP
  (void)h;
  if (nnz) *nnz = T.nnz;
  *out = t;
  return AM_OK;
}

am_status am_tpfa_pattern(am_tpfa t, int64_t* row_ptr, int32_t* col_idx) {
  if (!t) return fail(nullptr, AM_ERR_ARG, "null tpfa handle");
  if (row_ptr) std::copy(t->t.h_rp.begin(), t->t.h_rp.end(), row_ptr);
  if (col_idx) std::copy(t->t.h_ci.begin(), t->t.h_ci.end(), col_idx);
  return AM_OK;
}

am_status am_tpfa_assemble(am_tpfa t, const double* logK, double* val, double* f, void* stream) {
  if (!t || !logK || !val) return fail(nullptr, AM_ERR_ARG, "bad argument");
  am_handle h = nullptr;
  HCHK(hipSetDevice(t->t.device));
  HCHK(launch_tpfa_assemble(t->t, logK, val, f, (hipStream_t)stream));
  return AM_OK;
}

am_status am_tpfa_face_grad(am_tpfa t, const double* logK, const double* p, const double* lambda,
                            double* grad, void* stream) {
  if (!t || !logK || !p || !lambda || !grad) return fail(nullptr, AM_ERR_ARG, "bad argument");
  am_handle h = nullptr;
  HCHK(hipSetDevice(t->t.device));
  HCHK(launch_face_grad(t->t, logK, p, lambda, grad, (hipStream_t)stream));
  return AM_OK;
}

am_status am_tpfa_destroy(am_tpfa t) {
  if (!t) return AM_OK;
  (void)hipSetDevice(t->t.device);
  for (void* p : t->t.allocs) (void)hipFree(p);
  delete t;
  return AM_OK;
}

am_status algmortar_adjoint_grad(am_handle h, am_tpfa t, const double* logK, const double* p,
                                 const double* dJdp, double tol, int32_t maxit, double* lambda,
                                 double* grad, am_info* info, void* stream) {
  if (!h || !t || !logK || !p || !dJdp || !lambda || !grad)
    return fail(h, AM_ERR_ARG, "bad argument");
  if (t->t.n != h->d.n) return fail(h, AM_ERR_ARG, "face list and handle sizes differ");
  am_status s = algmortar_pcg(h, dJdp, lambda, 1, h->d.n, tol, maxit, info, stream);
  if (s != AM_OK) return s;
  HCHK(launch_face_grad(t->t, logK, p, lambda, grad, h->own));
  HCHK(hipStreamSynchronize(h->own));
  return AM_OK;
}

}  // extern "C"
