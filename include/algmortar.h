/*
 * algmortar.h -- C-ABI of the MI355X (gfx950) AlgMortar-PCG library.
 *
 * AlgMortar (Santos, Sousa, Ausas, Guiraldello, Pereira: "AlgMortar: a fully
 * algebraic multiscale mortar preconditioner") preconditions the conjugate
 * gradient solve of A p = f, A SPD with nonpositive off-diagonals
 * (Sec. 3, eq. linear-system).  The library partitions the graph of A
 * (Sec. 3.1), builds the diagonal-modified local operators
 * A_i = A_ii - sum_j D_ij (eq. Dij-def, eq. A_i), factors them, computes the
 * multiscale basis functions (eq. def-phat-local) and the interface matrix S
 * (eq. interface-problem-alg, Corollary eq. k-schur), and applies
 * z = Mcal^{-1} r (Algorithm 2) inside a PCG loop (Sec. 5, Sec. 7 set-up).
 *
 * Conventions for every entry point:
 *  - Status codes, never aborts; algmortar_last_error() gives the text.
 *  - Arguments are validated on the host before any device work.
 *  - Pointers documented as "host" are read (or written) during the call
 *    only and are never retained.  Pointers documented as "device" must be
 *    HIP device (or managed) memory of the GPU the handle was created on.
 *  - Vectors passed to the solver are in ORIGINAL ordering; the library
 *    permutes internally (Sec. 5.3: permute once, map back at the end).
 *  - Multi-RHS vectors are column-major: column c of an n x nrhs block starts
 *    at ptr + c*ld, ld >= n.
 *  - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *    algmortar_apply is asynchronous on that stream (except its first call
 *    for a right-hand-side count, which runs the tile autotuner and
 *    synchronizes); algmortar_pcg and algmortar_adjoint_grad block until the
 *    solve ends (they report am_info).  Calls that work on the library's own
 *    stream (set-up, update_values, pcg, adjoint_grad) first wait for the
 *    work already queued on `stream`, the null stream included.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef ALGMORTAR_H
#define ALGMORTAR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct am_handle_s* am_handle;
typedef struct am_tpfa_s* am_tpfa;

typedef enum {
  AM_OK = 0,
  AM_ERR_ARG = -1,               /* bad pointer, size, pattern or partition */
  AM_ERR_NOT_SYMMETRIC = -2,     /* a_kl != a_lk (bitwise) */
  AM_ERR_POSITIVE_COUPLING = -3, /* an off-diagonal > 0: W must be negative */
  AM_ERR_NOT_SPD = -4,           /* a Cholesky pivot <= 0 (A_i or S) */
  AM_ERR_NO_CONVERGENCE = -5,    /* maxit reached; x holds the last iterate */
  AM_ERR_BREAKDOWN = -6,         /* (p,Ap) <= 0 or (r,z) <= 0 in PCG */
  AM_ERR_HIP = -7,               /* a HIP runtime call failed */
  AM_ERR_OOM = -8,               /* device allocation failed */
  AM_ERR_UNSUPPORTED = -9        /* e.g. local bandwidth beyond the kernels */
} am_status;

/* Square sparse matrix, full (both triangles) CSR storage, columns strictly
 * ascending within each row.  row_ptr[n+1] and col_idx[nnz] are host
 * pointers; val[nnz] is host memory, or device memory when
 * values_on_device != 0.  Explicit zeros are allowed and are not couplings
 * (the graph of A has an edge iff a_kl != 0, Sec. 3.1). */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const double* val;
  int32_t values_on_device;
} am_csr;

/* Precision of the local factors and local solves.  FP64 is the method as
 * written; FP32 and BF16 (bf16 storage, fp32 arithmetic) are the reduced-
 * precision forms.  The interface solve, PCG vectors, dots and residuals are
 * always FP64. */
typedef enum { AM_FP64 = 0, AM_FP32 = 1, AM_BF16 = 2 } am_prec;

/* Mortar space (Sec. 5.4): one piecewise-constant basis function per
 * interface E_ij (the paper's choice), or one per interface edge
 * (Lambda = R^E, with which the preconditioner equals A^{-1}, Sec. 3.3). */
typedef enum { AM_MORTAR_PER_INTERFACE = 0, AM_MORTAR_PER_EDGE = 1 } am_mortar;

typedef struct {
  int32_t local_prec; /* am_prec */
  int32_t mortar;     /* am_mortar */
  int32_t max_nrhs;   /* largest nrhs later passed to apply/pcg (1..16) */
  int32_t device;     /* HIP device ordinal */
  uint32_t flags;     /* AM_FLAG_* */
} am_options;

#define AM_FLAG_NO_GRAPH 1u /* run the PCG loop with plain launches, no hipGraph */
/* apply eta = S^{-1} b as its own launches (row-part products, then their sum)
 * even where S^{-1} is small enough to be applied inside the local kernel */
#define AM_FLAG_SEPARATE_IFACE 2u
/* where eta = S^{-1} b is its own launches: multiply by the dense explicit
 * S^{-1} instead of the nested-dissection block elimination (the default:
 * explicit inverses of the uncoupled diagonal blocks of S in a nested-
 * dissection order of the interfaces and of the Schur complement on the
 * separators above them; Sec. 4, Corollary cor-schur-eta) */
#define AM_FLAG_DENSE_IFACE 4u
/* solve the interface system inexactly, by PCG with a block-Jacobi
 * preconditioner on S stopped at a relative residual (the iterative option of
 * Sec. 6, used with tolerance 1e-2 in Sec. 7): zero initial guess, blocks of
 * 64 consecutive basis functions (lexicographic (i, j) numbering) solved
 * exactly; defaults rtol 1e-2 and at most 50 inner iterations, see
 * algmortar_set_inexact.  The outer PCG then uses the flexible Polak-Ribiere
 * beta (the preconditioner depends on its argument). */
#define AM_FLAG_INEXACT_IFACE 8u
/* precision form with BF16 factors (local_prec AM_BF16), the interface
 * solve as its own launches, and either 16 right-hand sides (where the local
 * solves run on the matrix cores) or one right-hand side with every
 * subdomain's band within 64 rows: multiply the BF16 factor tiles by the
 * block vectors rounded to BF16 (round to nearest even), BF16 x BF16
 * products with FP32 accumulation on the matrix cores
 * (v_mfma_f32_16x16x16bf16_1k; one right-hand side takes column 0 of each
 * 16-column tile), instead of the default FP32 x FP32 products of the
 * widened factors (matrix cores with 16 right-hand sides, vector units with
 * one).  The preconditioner then carries 8-bit block vectors into every
 * factor product; the outer PCG is the flexible one, as for every reduced
 * precision.  Ignored in every other case. */
#define AM_FLAG_BF16_PRODUCTS 16u

typedef struct {
  int32_t iterations;  /* PCG iterations (matrix products) performed */
  int32_t converged;   /* 1 if ||r||_2 <= tol ||b||_2 was reached */
  double rel_res;      /* recursive residual norm / ||b|| at exit */
  double true_rel_res; /* ||b - A x||_2 / ||b||_2 recomputed at exit */
  double solve_ms;     /* wall time of the device loop */
} am_info;

/* TPFA face list (host pointers): interior face f joins cells k[f] and l[f];
 * l[f] = -1 marks a Dirichlet face with boundary value pD[f].  Half-
 * transmissibilities are t_k = exp(logK[k]) * gk[f], t_l = exp(logK[l]) * gl[f];
 * an interior face has transmissibility T = t_k t_l / (t_k + t_l). */
typedef struct {
  int64_t n_faces;
  const int64_t* k;
  const int64_t* l;
  const double* gk;
  const double* gl;
  const double* pD;
} am_faces;

/* ---- host-only entry points (no device work; usable without a GPU) ---- */

/* Block partition of an nx*ny*nz grid, cell (i,j,k) at index i+nx*(j+ny*k),
 * part = i/bx + (nx/bx)*(j/by + (ny/by)*(k/bz)).  The paper uses a graph
 * partitioner (Sec. 3.1); blocks are the deterministic choice for Cartesian
 * grids.  part: host int32[nx*ny*nz] (out); nparts: host (out).
 * AM_ERR_ARG if a block size does not divide its grid size. */
am_status am_partition_blocks(int32_t nx, int32_t ny, int32_t nz, int32_t bx, int32_t by,
                              int32_t bz, int32_t* part, int32_t* nparts);

/* Recursive double-BFS bisection of the graph of A (Sec. 3.1 with a
 * deterministic integer rule in place of METIS): sets of at most hi cells
 * become parts; larger sets are ordered by d_u - d_v (u, v the ends of a
 * double BFS, ties to the smallest index, other components last) and cut at
 * clamp(n*rho/100, lo, n-lo), rho = 40 + splitmix64(seed ^ node) % 21.
 * Needs hi >= 2*lo.  part: host int32[n] (out). */
am_status am_partition_bisect(const am_csr* A, int32_t lo, int32_t hi, uint64_t seed,
                              int32_t* part, int32_t* nparts);

/* Sizes of the interface structure of (A, part) (Sec. 3.1, eq. Eij, eq. E):
 * number of mortar basis functions and of interface edges.  Validates A
 * (symmetry, sign of the couplings, finiteness) and the partition. */
am_status am_structure_sizes(const am_csr* A, const int32_t* part, int32_t nparts,
                             int32_t mortar, int64_t* n_iface, int64_t* n_edges);

/* The interface structure itself, all host outputs:
 *  perm[n]            perm[new] = old: unknowns ordered by subdomain, ascending
 *                     original index inside each (the permutation P, eq.
 *                     linear-system-perm);
 *  sub_ptr[nparts+1]  subdomain i occupies new positions [sub_ptr[i], sub_ptr[i+1]);
 *  iface_ptr[NL+1]    edges of basis function n are [iface_ptr[n], iface_ptr[n+1]);
 *  iface_ij[2*NL]     the subdomain pair (i < j) of each basis function;
 *  edge_k[|E|], edge_l[|E|]  original indices of each edge, k in the lower-
 *                     numbered subdomain; edges sorted by (part k, part l, k, l). */
am_status am_structure(const am_csr* A, const int32_t* part, int32_t nparts, int32_t mortar,
                       int32_t* perm, int64_t* sub_ptr, int64_t* iface_ptr, int32_t* iface_ij,
                       int32_t* edge_k, int32_t* edge_l);

/* The nested-dissection order of the interface system that the interface
 * solve uses when it runs as its own launches (host only; Sec. 4: S is
 * coupled exactly where two basis functions share a subdomain, so cutting
 * the subdomain graph splits the basis functions into two uncoupled sets and
 * a separator).  order[NL] (host, out): ND position -> basis function, the
 * rows of the nblk mutually uncoupled diagonal blocks first, then the ntop
 * separator rows above them; blk_off (host, out, NL + 1 entries): the
 * blocks' first positions and the end of the last block.  max_nrhs as at
 * set-up (it bounds the block size).  AM_ERR_UNSUPPORTED when no dissection
 * depth fits the kernels (the set-up then uses the dense explicit S^{-1}). */
am_status am_interface_nd(const am_csr* A, const int32_t* part, int32_t nparts, int32_t max_nrhs,
                          int32_t* order, int64_t* blk_off, int32_t* nblk, int64_t* ntop);

/* ---- device entry points ---- */

/* Algorithm 1 (AlgMortarSetup): validate A and the partition, build the
 * permutation and interface structure, copy A to the device, factor every
 * A_i, compute the MBFs, assemble S and factor/invert it (FP64).
 * A: see am_csr; part: host int32[n] with ids in [0, nparts), none empty.
 * opt: host (NULL = defaults: FP64, per-interface mortar, 1 RHS, device 0).
 * On success *out owns all device memory until algmortar_destroy.
 * AM_ERR_NOT_SPD names the subdomain and pivot that failed.  The host part
 * (validation, local orderings, device-order rows) runs on up to 16 host
 * threads, or ALGMORTAR_HOST_THREADS if that is set; results do not depend on
 * the thread count, and an error names the lowest failing row or subdomain.
 * With ALGMORTAR_SETUP_TIMES set, the time of each set-up phase is printed
 * to stderr (phases with device work then end with a synchronization). */
am_status algmortar_setup(const am_csr* A, const int32_t* part, int32_t nparts,
                          const am_options* opt, void* stream, am_handle* out);

/* New values for the matrix of an existing handle: Algorithm 1's numeric
 * part (local operators and factors, MBFs, S and S^{-1}) is redone on the
 * device, the structure, partition, local orderings and layout are kept
 * (for a sequence of permeabilities on one grid, as in the differentiation
 * form).  A: row_ptr and col_idx (host) must equal the set-up's; val holds
 * the new values in the same order, on the host or (values_on_device) on the
 * handle's device.  The
 * values must pass the set-up's checks (finite, positive diagonal, bitwise
 * symmetric, couplings not positive), and a coupling between two subdomains
 * must be nonzero exactly where it was at set-up (the interfaces are kept).
 * The factors, MBFs, S and S^{-1} equal, bit for bit, those of a handle set
 * up from scratch on the new values with the same options (and so do its
 * results, given the same wave layout of the local kernel: see
 * algmortar_tile_choice).  The first call builds index maps of the
 * pattern on the device (about 17 bytes per stored entry, kept until
 * algmortar_destroy).  Synchronizes `stream` and the handle's work first.
 * Errors: AM_ERR_ARG (pattern differs, non-finite value, a changed
 * interface coupling), AM_ERR_NOT_SYMMETRIC, AM_ERR_POSITIVE_COUPLING,
 * AM_ERR_NOT_SPD (diagonal, or a pivot of A_i or S), AM_ERR_UNSUPPORTED
 * while a smoother is set, AM_ERR_HIP / AM_ERR_OOM.  When a check fails the
 * handle keeps its previous values; when the factorization fails, apply, PCG
 * and local solves return AM_ERR_NOT_SPD until an update succeeds. */
am_status algmortar_update_values(am_handle h, const am_csr* A, void* stream);

/* Tolerance and iteration cap of the inexact interface solve of a handle set
 * up with AM_FLAG_INEXACT_IFACE: the inner PCG stops when
 * ||b - S eta||_2 <= rtol ||b||_2 (recursive residual) or after maxit
 * iterations.  rtol in [0, 1) (0: always maxit iterations), maxit in
 * [1, 1000].  The next algmortar_pcg captures its iteration graphs again.
 * AM_ERR_ARG on other handles or values. */
am_status algmortar_set_inexact(am_handle h, double rtol, int32_t maxit);

/* Block-Jacobi pre- and post-smoothing around the AlgMortar correction
 * (Sec. 5.4).  After this call algmortar_apply and algmortar_pcg use
 *   z = 0;  nu times z += B^{-1} (r - A z);  z += Mcal^{-1} (r - A z);
 *   nu times z += B^{-1} (r - A z)
 * with B = blockdiag(A[K, K]) over the blocks K of `blocks`, each block
 * solved exactly (band Cholesky of the block as it is, in the handle's factor
 * precision; the paper names block Jacobi and the number of blocks only).
 * blocks: host int32[n], ids in [0, nblocks), none empty (typically unions of
 * several subdomains; each block's bandwidth in ascending index order or RCM
 * order must be at most 128).  steps: nu in [0, 1000]; 0 removes the smoother.
 * The block factors take device memory like the subdomain factors.  Replaces
 * any earlier smoother; synchronizes the device (work on any stream may
 * still use the earlier smoother), so `stream` needs no special handling.
 * algmortar_local_solve and algmortar_time_kernel are unaffected;
 * algmortar_pcg_profile returns AM_ERR_UNSUPPORTED while a smoother is set.
 * Errors: AM_ERR_ARG (partition), AM_ERR_UNSUPPORTED (bandwidth), AM_ERR_OOM;
 * after an error the handle has no smoother. */
am_status algmortar_set_smoother(am_handle h, const int32_t* blocks, int32_t nblocks,
                                 int32_t steps, void* stream);

/* Algorithm 2 (AlgMortarApply): z = Mcal^{-1} r for nrhs columns.
 * r, z: device, n x nrhs column-major with leading dimension ld (may not
 * alias).  Asynchronous on stream. */
am_status algmortar_apply(am_handle h, const double* r, double* z, int32_t nrhs, int64_t ld,
                          void* stream);

/* Allocation-free variant of algmortar_apply, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and result as
 * algmortar_apply (the same kernels: bitwise the same z), but its work
 * buffers -- the permuted r and z, the interface slots, eta and the row-part
 * sums of the interface product -- live in a static device array of
 * 48 MiB (6,291,456 doubles) per GPU instead of the handle's memory, and the
 * call allocates nothing.  The array is shared by every handle and every call
 * on one GPU and keeps the last call's contents: calls that overlap on one
 * GPU (other streams, other threads) race and must be ordered by the caller.
 * Needs 2 n nr + 2 NL nr + ldS nr doubles (plus, where the interface solve
 * is its own launches, its part sums and, in the dissection form, the block
 * and separator vectors), nr = nrhs rounded up to a power of two; AM_ERR_ARG
 * when that exceeds the array.  AM_ERR_UNSUPPORTED while a smoother is set
 * and on handles with the inexact interface solve.  Its
 * first call for a right-hand-side count on a handle whose local-kernel
 * layout is not yet chosen runs the autotuner and synchronizes (call
 * algmortar_tile_choice first to keep it asynchronous).  Asynchronous on
 * stream. */
am_status algmortar_apply_static(am_handle h, const double* r, double* z, int32_t nrhs, int64_t ld,
                                 void* stream);

/* The local particular solutions only: pbar_i = A_i^{-1} r_i on every
 * subdomain (eq. def-pbar-local).  r, pbar: device, original ordering,
 * single column.  Asynchronous. */
am_status algmortar_local_solve(am_handle h, const double* r, double* pbar, void* stream);

/* PCG on A x = b preconditioned by the handle (x0 = 0, stop when
 * ||r||_2 <= tol ||b||_2 on the recursive residual, Sec. 7).  Columns are
 * solved independently.  b, x: device, n x nrhs column-major, leading
 * dimension ld.  info: host am_info[nrhs] (may be NULL).  maxit <= 0 means
 * 10000.  Returns AM_ERR_NO_CONVERGENCE if a column did not converge (x then
 * holds the last iterate) and AM_ERR_BREAKDOWN on a nonpositive curvature.
 * FP64 local factors use the Fletcher-Reeves beta, reduced-precision ones
 * the Polak-Ribiere (flexible) beta. */
am_status algmortar_pcg(am_handle h, const double* b, double* x, int32_t nrhs, int64_t ld,
                        double tol, int32_t maxit, am_info* info, void* stream);

/* Copy the handle's structure to host buffers (same layout as am_structure). */
am_status algmortar_interfaces(am_handle h, int32_t* perm, int64_t* sub_ptr, int64_t* iface_ptr,
                               int32_t* iface_ij, int32_t* edge_k, int32_t* edge_l);

/* Sizes held by a handle: n, nparts, number of basis functions, edges. */
am_status algmortar_sizes(am_handle h, int64_t* n, int64_t* nparts, int64_t* n_iface,
                          int64_t* n_edges);

/* Copy the interface matrix S (dense FP64, n_iface x n_iface, row-major,
 * symmetrised) or its inverse to a host buffer.  which: 0 = S, 1 = S^{-1}. */
am_status algmortar_export_interface(am_handle h, int32_t which, double* out);

/* Copy the MBF values of basis function `iface` on subdomain `sub` (one of
 * its two subdomains) to host buffer out[N_sub], in the subdomain's
 * ascending-original-index order (eq. def-phat-local). */
am_status algmortar_export_mbf(am_handle h, int64_t iface, int32_t sub, double* out);

/* Measurement: `reps` back-to-back launches of one apply kernel on the
 * handle's internal stream, bracketed by HIP events (the buffers hold the
 * last call's data).  kernel: 0 = local solves + reconstruction (the band
 * sweeps of Algorithm 2), 1 = interface solve eta = S^{-1} b (row-part
 * products and their sum; AM_ERR_ARG on a handle whose interface solve runs
 * inside the local kernel),
 * 2 = interface partial right-hand sides, 3 = the PCG SpMV (p update, A p,
 * (p, Ap)), 4 = the PCG x/r update with the interface partials, 5 = the
 * block solves of the smoother set by algmortar_set_smoother (kernel 0 on the
 * block factors; AM_ERR_ARG without a smoother).  Timing 3 or 4 leaves the
 * handle's PCG scalars in an unspecified state (the next algmortar_pcg call
 * re-initialises them).  avg_ms: host (out), average launch
 * duration; bytes: host (out), the kernel's algorithmic HBM bytes per launch
 * (factor, vectors and operators it must read or write once). */
am_status algmortar_time_kernel(am_handle h, int32_t kernel, int32_t nrhs, int32_t reps,
                                double* avg_ms, double* bytes);

/* Batching form: the wave layout of the local kernel (groups of right-hand
 * sides x column splits of each block pass) is chosen per right-hand-side
 * count by an autotuner that times every candidate layout on this handle's
 * subdomains as a solve runs it (with the PCG dot products, on a freshly
 * initialised PCG state that the next algmortar_pcg initialises again; the
 * candidates take turns over three rounds).  It runs, and synchronizes, on
 * the first algmortar_apply or algmortar_pcg with that count (or here).
 * choice: host (out), index of the chosen candidate; ncand: host (out),
 * number of candidates; us: host (out, may be NULL), double[4], each
 * candidate's average launch time in us over its fastest round.
 * The layouts add the waves' partial vectors in different orders, so two
 * handles whose timings chose differently can differ in the last bits; with
 * the environment variable ALGMORTAR_TILE=c, candidate c (clamped to the
 * list) is used without timing (us then holds zeros), which makes results
 * reproducible across handles and processes.  With
 * ALGMORTAR_AUTOTUNE_CACHE=path, the choices are appended to that text file
 * (one line per tuned case: a key of the handle's sizes, window buckets,
 * factor precision, interface form and right-hand-side count, and the
 * choice) and read back by later handles and processes, which then use the
 * recorded layout without timing (us holds zeros): the same results as the
 * process that timed it.  16 right-hand sides with the interface solve as
 * its own launches, and one right-hand side under AM_FLAG_BF16_PRODUCTS
 * with every subdomain's band within 64 rows, run matrix-core kernels of a
 * single layout: choice 0, ncand 1, nothing timed. */
am_status algmortar_tile_choice(am_handle h, int32_t nrhs, int32_t* choice, int32_t* ncand,
                                double* us);

/* Measurement: algmortar_pcg with plain launches (no hipGraph), every launch
 * timed with HIP events on the handle's internal stream (attached to the
 * first and the last launch of each operation, hipExtLaunchKernelGGL, so
 * they hold the dispatches' own start and end) and the stop flag read after
 * each iteration, so the durations are those of the kernels inside
 * a real solve (same order, same data, same cache state).  Same arguments and
 * results as algmortar_pcg, plus kernel_ms[5] (host, out): summed launch
 * durations in ms, and launches[5] (host, out): launch counts, indexed by the
 * kernel numbers of algmortar_time_kernel (2 stays zero: the PCG path computes
 * the interface partials inside kernel 4).  Launches of iterations that began
 * after convergence are not counted. */
am_status algmortar_pcg_profile(am_handle h, const double* b, double* x, int32_t nrhs, int64_t ld,
                                double tol, int32_t maxit, am_info* info, double* kernel_ms,
                                int64_t* launches, void* stream);

am_status algmortar_destroy(am_handle h);

/* Text of the last error on handle h, or of the calling thread's last error
 * when h is NULL.  Valid until the next call on that handle/thread. */
const char* algmortar_last_error(am_handle h);

/* ---- differentiation form (no paper analogue) ---- */

/* Create the TPFA assembler for a face list over n cells: builds the CSR
 * pattern of A on the host and the face -> CSR-slot maps on the device.
 * faces: host.  row_ptr[n+1], col_idx[nnz] (host, out, may be NULL) receive
 * the pattern; *nnz receives its size. */
am_status am_tpfa_create(const am_faces* faces, int64_t n, int32_t device, am_tpfa* out,
                         int64_t* nnz);
am_status am_tpfa_pattern(am_tpfa t, int64_t* row_ptr, int32_t* col_idx);

/* Assemble A's values and the Dirichlet part of f from logK on the device:
 * logK[n], val[nnz], f[n] all device.  Asynchronous. */
am_status am_tpfa_assemble(am_tpfa t, const double* logK, double* val, double* f, void* stream);

/* Adjoint gradient of J(p(theta)) for theta = log K: solves A lambda = dJdp
 * by PCG with the handle's preconditioner (A symmetric), then scatters
 *   grad_c = -sum_{faces f at c} dT_f/dtheta_c (lambda_k - lambda_l)(p_k - p_l)
 *            - sum_{Dirichlet faces of c} t_c lambda_c (p_c - pD)
 * per cell (deterministic cell-centric gather).  logK, p, dJdp, lambda, grad:
 * device, original ordering, single column.  info: host (may be NULL). */
am_status algmortar_adjoint_grad(am_handle h, am_tpfa t, const double* logK, const double* p,
                                 const double* dJdp, double tol, int32_t maxit, double* lambda,
                                 double* grad, am_info* info, void* stream);

/* Only the face scatter above, for given p and lambda (device). */
am_status am_tpfa_face_grad(am_tpfa t, const double* logK, const double* p, const double* lambda,
                            double* grad, void* stream);

am_status am_tpfa_destroy(am_tpfa t);

#ifdef __cplusplus
}
#endif

#endif /* ALGMORTAR_H */
