// Device-side state of an AlgMortar handle and the launchers of the gfx950
// kernels.  Internal header (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "am_host.h"

namespace am {

constexpr int kMaxNRHS = 16;
constexpr int kMaxWp = 128;   // widest band window the LDS factor kernel holds
constexpr int kTile = 64;     // dense interface-matrix tile
// size of the static scratch of algmortar_apply_static (48 MiB of doubles)
constexpr int64_t kStaticScratchDoubles = (int64_t)48 * 1024 * 1024 / 8;

// PCG scalars of one right-hand side, device resident.
struct PcgScalars {
  double rzv[2];  // (r, z), by iteration parity (written and read in different launches)
  double rz;      // (r, z) of the last iteration (reporting)
  double pq;      // (p, A p)
  double alpha;
  double beta;
  double rr;      // ||r||^2
  double bb;      // ||b||^2
  double tol2;    // tol^2
  double qz;      // (q, z_new), for the flexible beta
  int32_t it;     // iterations done
  int32_t done;   // 1 once converged / stopped
  int32_t status; // am_status of this column
  int32_t conv;   // 1 if converged
};

struct PcgShared {
  int32_t maxit;
  int32_t nrhs;
  int32_t flexible;  // Polak-Ribiere beta
  int32_t all_done;
};

// Per-block partial sums of the PCG dots.  With up to four columns the
// kernel that needs a scalar folds the producer's partials itself, in block
// order, identically in every workgroup (deterministic, no fences or
// atomics), and workgroup 0 stores the scalars for later launches; with 8-16
// columns a one-workgroup-per-column launch folds them once into coef.
struct Reduce {
  double* pa = nullptr;         // (p, Ap) per SpMV block (1-4 columns) or subdomain (8-16)
  double* pb = nullptr;         // ||r||^2 per subdomain            [m][NR]
  double* pd = nullptr;         // (r, z), (q, z) per subdomain     [m][2 NR]
  double* coef = nullptr;       // beta, alpha of 8-16 columns      [2][kMaxNRHS]
  double* partial = nullptr;    // true-residual partials
  unsigned* counter = nullptr;
  int spmv_blocks = 0;
  int max_blocks = 0;
};

// Nested-dissection interface solve (kernels_nd.hip, layout from
// build_iface_nd): device arrays, owned through DeviceState::allocs.
struct NdDevice {
  int32_t on = 0;          // the interface solve uses this form
  int32_t nblk = 0;
  int64_t nrows = 0;       // rows in blocks
  int32_t R = 0;           // top rows
  int32_t ldC = 0;         // leading dimension of C^{-1} (R rounded up to 64)
  int32_t ldp = 0;         // padded dimension of the reordered S
  int32_t nwg = 0;         // workgroups of k_nd_blocks
  int64_t smax = 0;        // rows of the largest block
  int32_t P = 1, per = 1;  // row parts of k_nd_top and rows per part
  int64_t nt_pairs = 0, nb_pairs = 0;
  std::vector<int64_t> h_blk_off, h_pad_off;  // host copies
  std::vector<int32_t> h_src;
  int32_t* ord = nullptr;      // [NL] ND position -> basis function (top rows last)
  int32_t* src = nullptr;      // [ldp] padded position -> basis function, -1 on padding
  int64_t* blk_off = nullptr;  // [nblk+1]
  int64_t* pad_off = nullptr;  // [nblk+1]
  int64_t* inv_off = nullptr;  // [nblk+1] offsets of the block inverses (full squares)
  int32_t* wg_blk = nullptr;   // [nwg] block of each workgroup ..
  int32_t* wg_row0 = nullptr;  // .. and its first row
  double* binv = nullptr;      // block inverses
  double* cinv = nullptr;      // [R][ldC] C^{-1}
  int64_t* t_ptr = nullptr;    // [R+1] top row -> couplings to block rows
  int32_t* t_pos = nullptr;    //   ND positions of those rows
  double* t_val = nullptr;     //   S values
  int32_t *t_ri = nullptr, *t_ci = nullptr;  // (row, column) of each value in S (set-up)
  int64_t* b_ptr = nullptr;    // [nrows+1] block row -> couplings to top rows
  int32_t* b_top = nullptr;    //   top indices
  double* b_val = nullptr;
  int32_t *b_ri = nullptr, *b_ci = nullptr;
  double* y1 = nullptr;        // [nrows][max_nrhs]
  double* eta2 = nullptr;      // [R][max_nrhs]
  double* ypart = nullptr;     // [P][ldC][max_nrhs]
};

// Inexact interface solve (kernels_inexact.hip): per-column state of the
// inner PCG, by iteration parity where one launch reads what the next writes
struct IxScalars {
  double rzs[2];     // (r, z) of the inner iteration
  double bb;         // ||b||^2
  int32_t done[2];   // inner solve stopped
  int32_t iters;     // inner iterations of the last solve
  int32_t pad_;
};

struct IxDevice {
  int32_t on = 0;
  int32_t bs = 64;         // block-Jacobi block rows (multiple of 64, at most 256)
  int32_t nblk = 0;
  int32_t maxit = 50;
  int32_t w = 0;           // ELL width of S
  double rtol = 1e-2;
  int64_t* inv_off = nullptr;  // [nblk+1]
  double* binv = nullptr;      // block inverses, full squares
  int32_t* scol = nullptr;     // [w][NL] ELL columns of S (padding: the row itself)
  int8_t* pad = nullptr;       // [w][NL] 1 on padding entries
  double* sval = nullptr;      // [w][NL]
  double *r = nullptr, *z = nullptr, *q = nullptr;
  double* p[2] = {nullptr, nullptr};
  double* pa = nullptr;                 // [nblk][max_nrhs] (p, q) partials
  double* pb[2] = {nullptr, nullptr};   // [nblk][2 max_nrhs] (r, z), (r, r) partials
  IxScalars* sc = nullptr;              // [kMaxNRHS]
};

struct DeviceState {
  int device = 0;
  int prec = AM_FP64;
  int64_t n = 0;
  int32_t m = 0;
  int64_t NL = 0, NE = 0;
  int32_t ldS = 0;  // padded interface dimension (multiple of kTile)
  int32_t fuse_eta = 0;  // local kernel computes its own rows of eta = S^{-1} b
  int32_t plain = 0;     // factors are the plain diagonal blocks A_ii (block Jacobi)
  int32_t bf16_ops = 0;  // 16-RHS matrix-core sweeps: BF16 x BF16 products (AM_FLAG_BF16_PRODUCTS)
  int32_t max_nrhs = 1;
  int32_t max_np = 0;       // largest padded subdomain row count
  // wave layout of the tile kernel chosen by the autotuner per right-hand-side
  // count (slot log2 nrhs), -1 until tuned; the timed average per candidate
  int32_t tile_cand[5] = {-1, -1, -1, -1, -1};
  float tile_us[5][4] = {};
  // profiled solves: events that the first and the last launch of the next
  // operation carry (am_launch), and whether they were attached
  hipEvent_t prof_ev[2] = {nullptr, nullptr};
  bool prof_used[2] = {false, false};
  // second stream (default priority) and the events of the fork and join
  // that run the two window buckets of the local kernel side by side
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  // device ordering and permuted matrix
  int32_t* dperm = nullptr;    // [n] device position -> original index
  int32_t ell_w = 0;
  int32_t* ell_col = nullptr;  // [ell_w * n] column-major, device positions
  double* ell_val = nullptr;
  int64_t* prp = nullptr;      // permuted CSR (rows/cols in device positions)
  int32_t* pci = nullptr;
  double* pv = nullptr;

  // subdomains
  int64_t* sub_ptr = nullptr;  // [m+1]
  int32_t* wp = nullptr;       // [m]
  int64_t* roff = nullptr;     // [m+1] padded row offsets of the factor blocks
  int64_t* fac_off = nullptr;  // [m+1] element offsets of the factor blocks
  void* Lc = nullptr;          // band factor, column layout (precision dependent)
  void* Lr = nullptr;          // band factor, row layout (set-up only; freed after)
  void* invd = nullptr;        // [n] 1/L_jj (double for FP64, float otherwise)
  std::vector<int32_t> bucket_sub[2];  // host: subdomain ids per window width 64/128
  int32_t* d_bucket_sub[2] = {nullptr, nullptr};
  std::vector<int32_t> bucket_pair[2]; // host: (subdomain, slot) pairs per window width
  int32_t* d_bucket_pair[2] = {nullptr, nullptr};
  int32_t* fail = nullptr;     // [4]: failing subdomain and pivot of A_i; failing row of S (device)

  // mortar structure
  int64_t* isub_ptr = nullptr;   // [m+1]
  int32_t* isub_list = nullptr;  // [2 NL]
  int64_t* mbf_off = nullptr;    // [m+1] offsets of P^_s blocks ([n_s][N_s])
  double* mbf = nullptr;
  int64_t* bw_ptr = nullptr;     // [2 NL + 1] boundary weights per (subdomain, slot)
  int32_t* bw_row = nullptr;     // local row (device order inside the subdomain)
  double* bw_val = nullptr;      // -2 * sum a_e  (= -B_s psi_n)
  int32_t* mbf_pair_sub = nullptr;  // [2 NL] subdomain of each (s, slot) pair
  int32_t* mbf_pair_q = nullptr;    // [2 NL] slot
  int64_t* iface_ptr = nullptr;  // [NL+1]
  int32_t* iface_ij = nullptr;   // [2 NL]
  int32_t* e_kloc = nullptr;     // [NE] local row of k in subdomain i
  int32_t* e_lloc = nullptr;     // [NE] local row of l in subdomain j
  double* e_a = nullptr;         // [NE]
  int64_t* bdst = nullptr;       // [2 NL] (subdomain, slot) pair -> slot 2n + side of bpart
  double* S = nullptr;           // [ldS * ldS] symmetrised interface matrix
  double* Sinv = nullptr;        // [ldS * ldS]
  int32_t op_parts = 1;          // row parts of the interface product (k_iface_op)
  double* ypart = nullptr;       // [op_parts][ldS][max_nrhs] part sums of eta
  NdDevice nd;                   // nested-dissection interface solve (nd.on)
  IxDevice ix;                   // inexact interface solve (ix.on)

  // work vectors in device order, row-interleaved [n][nrhs]
  double* x = nullptr;
  double* r = nullptr;
  double* z = nullptr;
  double* p[2] = {nullptr, nullptr};
  double* q = nullptr;
  double* bpart = nullptr;  // [2 NL][nrhs], slot 2n + side
  double* eta = nullptr;    // [ldS][nrhs]
  PcgScalars* sc = nullptr; // [kMaxNRHS]
  PcgShared* shared = nullptr;
  int32_t* h_flags = nullptr;  // pinned host mirror of shared
  PcgScalars* h_sc = nullptr;  // pinned host copies of sc, two slots of kMaxNRHS
  Reduce red;

  // captured PCG chunks of 8 iterations (graph) and of 2, 4, 6 (graph_short)
  hipGraphExec_t graph = nullptr;
  hipGraphExec_t graph_short[3] = {nullptr, nullptr, nullptr};
  hipStream_t graph_stream = nullptr;
  int graph_nrhs = 0;
  const void* graph_key = nullptr;
  std::vector<void*> allocs;
};

// ---- static scratch (static_scratch.hip) ----
// address of the device's copy of the static scratch array, looked up once
// per device with `device` current (hipGetSymbolAddress)
hipError_t static_scratch_init(int device);
// that address, or null before static_scratch_init succeeded on `device`
double* static_scratch_ptr(int device);

// ---- launchers (kernels_local.hip) ----
hipError_t launch_band_factor(DeviceState& d, hipStream_t s);
hipError_t launch_mbf(DeviceState& d, hipStream_t s);
inline int tile_slot(int nrhs) { return nrhs <= 1 ? 0 : nrhs <= 2 ? 1 : nrhs <= 4 ? 2 : nrhs <= 8 ? 3 : 4; }
// number of tile-kernel wave layouts the autotuner times for nrhs
int tile_candidates(int nrhs);
// replaces the 64 x 64 diagonal blocks of the column layout by their inverses
hipError_t launch_invert_diag(DeviceState& d, hipStream_t s);
// z = A_i^{-1} r (+ prolongation with eta when eta != nullptr); dots when dot_out
hipError_t launch_local_sweep(DeviceState& d, const double* r, double* z, const double* eta,
                              int nrhs, int mode, hipStream_t s);
hipError_t launch_bpart(DeviceState& d, const double* r, int nrhs, hipStream_t s);

// ---- launchers (kernels_iface.hip) ----
hipError_t launch_assemble_S(DeviceState& d, hipStream_t s);
// S^{-1} through the tiled Cholesky factor L and its inverse Linv (both
// ldS x ldS scratch); part: trtri_part_tiles(ldS / 64) tiles of 64 x 64
// scratch for the split launches of the inverse (may be null if that is 0)
int64_t trtri_part_tiles(int T);
hipError_t dense_cholesky_inverse(DeviceState& d, double* L, double* Linv, double* part,
                                  hipStream_t s);
// eta = S^{-1} b; in PCG mode (pcg != 0) the launch first applies the stop
// test to the ||r||^2 partials (init: records ||b||^2)
hipError_t launch_iface_gemv(DeviceState& d, int nrhs, int pcg, int init, hipStream_t s);
// out = Li^T Li over a T x T tile block (Li lower triangular, leading
// dimension ld; both pointers at the block's first entry)
hipError_t launch_lauum(const double* Li, double* out, int ld, int T, hipStream_t s);

// ---- launchers (kernels_nd.hip) ----
// largest block (rows) the nested-dissection kernels take for nr_max columns
int64_t nd_max_rows(int nr_max);
// eta = S^{-1} b by the nested-dissection block elimination (same contract
// as launch_iface_gemv)
hipError_t launch_nd_solve(DeviceState& d, int nrhs, int pcg, int init, hipStream_t s);
// set-up: block inverses, C^{-1} and coupling values from d.S (see kernels_nd.hip)
hipError_t nd_numeric(DeviceState& d, double* Sp, double* L, double* Li, double* part,
                      hipStream_t s);

// ---- launchers (kernels_inexact.hip) ----
// eta ~ S^{-1} b by block-Jacobi PCG (same contract as launch_iface_gemv)
hipError_t launch_ix_solve(DeviceState& d, int nrhs, int pcg, int init, hipStream_t s);
// set-up: block inverses and the ELL values of S (see kernels_inexact.hip)
hipError_t ix_numeric(DeviceState& d, double* Sbd, double* L, double* Li, double* part,
                      hipStream_t s);

// ---- launchers (kernels_pcg.hip) ----
hipError_t launch_permute_in(const int32_t* dperm, int64_t n, const double* src, int64_t ld,
                             double* dst, int nrhs, hipStream_t s);
hipError_t launch_permute_out(const int32_t* dperm, int64_t n, const double* src, double* dst,
                              int64_t ld, int nrhs, hipStream_t s);
hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t s);
hipError_t launch_pcg_init(DeviceState& d, int nrhs, double tol, int maxit, int flexible,
                           hipStream_t s);
hipError_t launch_pcg_iteration(DeviceState& d, int nrhs, int parity, hipStream_t s);
hipError_t launch_pcg_start(DeviceState& d, int nrhs, hipStream_t s);
hipError_t launch_pcg_spmv(DeviceState& d, int nrhs, int parity, hipStream_t s);
hipError_t launch_pcg_update(DeviceState& d, int nrhs, int parity, hipStream_t s);
hipError_t launch_true_residual(DeviceState& d, const double* bperm, int nrhs, double* out2,
                                hipStream_t s);

hipError_t launch_pcg_rr0(DeviceState& d, int nrhs, hipStream_t s);  // ||r_0||^2 partials, b(r_0)
// the stop test on the ||r||^2 partials of the last update (kernels_local.hip)
hipError_t launch_stop_test(DeviceState& d, int nrhs, int init, hipStream_t s);

// ---- new values on an existing handle (kernels_values.hip) ----
// Index maps from the caller's CSR order (built at the first update; owned
// by the handle through `allocs`).
struct ValueMaps {
  bool built = false;
  int64_t nnz = 0, nbw = 0;
  int64_t* vpos = nullptr;   // [nnz] caller position of device-order CSR entry q
  int64_t* code = nullptr;   // [nnz] -2 diagonal, -1 no transpose, else transpose position
  int8_t* cross = nullptr;   // [nnz] 0 inside a subdomain, 1 interface edge, 2 zero between subdomains
  int64_t* epos = nullptr;   // [NE] caller position of interface edge e
  int64_t* bw_ptr = nullptr; // [nbw + 1] edges of boundary-weight entry t ..
  int32_t* bw_src = nullptr; // [2 NE] .. in the set-up's summation order
  double* vals = nullptr;    // [nnz] device copy of host-resident new values
  unsigned long long* bad = nullptr;  // lowest failing position of the checks
  std::vector<int64_t> code_h;  // host copies of code and cross (error messages)
  std::vector<int8_t> cross_h;
  std::vector<void*> allocs;
};
// *vm.bad = lowest position of v that fails the set-up's checks (else ~0)
hipError_t launch_check_values(const ValueMaps& vm, const double* v, hipStream_t s);
// d.pv, d.ell_val, d.e_a and d.bw_val from v
hipError_t launch_place_values(DeviceState& d, const ValueMaps& vm, const double* v, hipStream_t s);

// ---- block-Jacobi smoothing (kernels_smooth.hip) ----
struct SmoothDevice {
  DeviceState* bj = nullptr;        // band factors of the plain diagonal blocks
  int32_t steps = 0;                // steps before and after the correction
  const int32_t* to_bj = nullptr;   // [n] AlgMortar position of each block-Jacobi position
  const int32_t* to_am = nullptr;   // [n] block-Jacobi position of each AlgMortar position
  double* t_am = nullptr;           // [n * max_nrhs] correction input, AlgMortar order
  double* w_am = nullptr;           // [n * max_nrhs] correction output
};
// z_am = M^{-1} r_am (both in d's device order, node vectors of nr columns)
hipError_t launch_smoothed_apply(DeviceState& d, SmoothDevice& sm, const double* r_am,
                                 double* z_am, int nr, hipStream_t s);
// (r, z) and (q, z) partials of d's PCG vectors into d.red.pd (m workgroups)
hipError_t launch_smooth_dots(DeviceState& d, int nrhs, hipStream_t s);

// ---- launchers (kernels_tpfa.hip) ----
struct TpfaDevice {
  int device = 0;
  int64_t n = 0, nnz = 0, nf = 0;
  std::vector<int64_t> h_rp;
  std::vector<int32_t> h_ci;
  int64_t* fk = nullptr;   // [nf]
  int64_t* fl = nullptr;
  double* gk = nullptr;
  double* gl = nullptr;
  double* pD = nullptr;
  int64_t* slot_kk = nullptr;  // CSR slots touched by each face
  int64_t* slot_ll = nullptr;
  int64_t* slot_kl = nullptr;
  int64_t* slot_lk = nullptr;
  int64_t* cf_ptr = nullptr;   // cell -> faces CSR
  int32_t* cf_face = nullptr;
  std::vector<void*> allocs;
};
hipError_t launch_tpfa_assemble(TpfaDevice& t, const double* logK, double* val, double* f,
                                hipStream_t s);
hipError_t launch_face_grad(TpfaDevice& t, const double* logK, const double* p,
                            const double* lam, double* grad, hipStream_t s);

}  // namespace am
