// PCG kernels for gfx950 (Sec. 5: AlgMortar as the CG preconditioner; Sec. 7:
// x0 = 0, relative residual stop).  One iteration is, in order:
//   SpMV     : beta from (r, z); p = z + beta p (ping-pong buffers), q = A p, (p, q)
//              (k_spmv_p with 1-4 columns, k_pcg_coef + k_spmv_sub with 8-16)
//   update   : alpha = (r, z)/(p, q); x += alpha p, r -= alpha q, ||r||^2; the
//              interface partial right-hand sides 1/4 phat^T r per (subdomain, slot)
//              (k_update_xr with 1-4 columns, k_pcg_coef + k_update_rows with 8-16)
//   interface: stop test on ||r||; eta = S^{-1} b, where it is its own launches
//              (kernels_nd.hip, kernels_iface.hip, kernels_inexact.hip)
//   local    : z = A_i^{-1} r + sum eta_m phat^(m), (r, z), (q, z) (local_kernels.h)
// Scalars stay on the device.  With up to four columns a launch that needs a
// scalar folds the per-block partial sums of the launch that produced them,
// in block order and identically in every workgroup (deterministic, no
// fences, no atomics), and workgroup 0 stores the scalars; with 8 or 16
// columns a small launch before the SpMV and the update folds them once
// (k_pcg_coef).  Every launch returns at once when all columns have stopped,
// so a captured chunk of iterations can run past convergence harmlessly.
#include <type_traits>

#include "am_common.h"

namespace am {

template <int NR>
__global__ __launch_bounds__(256) void k_permute_in(const int32_t* __restrict__ dperm, int64_t n,
                                                    const double* __restrict__ src, int64_t ld,
                                                    int nrhs, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o = dperm[i];
#pragma unroll
  for (int k = 0; k < NR; ++k) dst[vix<NR>(n, i, k)] = k < nrhs ? src[k * ld + o] : 0.0;
}

template <int NR>
__global__ __launch_bounds__(256) void k_permute_out(const int32_t* __restrict__ dperm, int64_t n,
                                                     const double* __restrict__ src, int nrhs,
                                                     double* __restrict__ dst, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o = dperm[i];
#pragma unroll
  for (int k = 0; k < NR; ++k)
    if (k < nrhs) dst[k * ld + o] = src[vix<NR>(n, i, k)];
}

__global__ __launch_bounds__(256) void k_fill(double* p, int64_t cnt, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) p[i] = v;
}

__global__ void k_init_scalars(PcgScalars* sc, PcgShared* sh, int nr, int nrhs, double tol2,
                               int maxit, int flexible) {
  const int k = threadIdx.x;
  if (k < nr) {
    PcgScalars& S = sc[k];
    S.rzv[0] = S.rzv[1] = 0.0;
    S.rz = S.pq = S.alpha = S.beta = S.rr = S.bb = S.qz = 0.0;
    S.tol2 = tol2;
    S.it = 0;
    S.done = 0;
    S.status = 0;
    S.conv = 0;
  }
  if (k == 0) {
    sh->maxit = maxit;
    sh->nrhs = nr;
    sh->flexible = flexible;
    sh->all_done = 0;
  }
  (void)nrhs;
}

// Right-hand sides per workgroup of the PCG kernels: a workgroup takes the
// group of KG columns given by blockIdx.x % (NT/KG) (the vector layout keeps
// a group contiguous; see vix), so the groups of the same rows run together.

// p_new = z + beta p_old; q = A p_new (ELL, column-major, device positions).
// beta comes from the (r, z), (q, z) partials of the previous local launch,
// folded by every workgroup in block order; the first workgroup of each group
// stores rz and beta.  Every load that does not depend on another one is
// issued first (the stop flag, the scalars, the partials to fold, the ELL
// rows), then the gathers; the stop decision and the fold are taken once they
// are in flight, so the launch costs two memory round trips.  Grid-stride over
// rows with a fixed grid, one (p, q) partial per workgroup and column.
template <int NT, int MAXW>
__global__ __launch_bounds__(256) void k_spmv_p(int64_t n, int w, const int32_t* __restrict__ ec,
                                                const double* __restrict__ ev,
                                                const double* __restrict__ z,
                                                const double* __restrict__ pold,
                                                double* __restrict__ pnew, double* __restrict__ q,
                                                const double* __restrict__ pd, int npd,
                                                double* __restrict__ pa, PcgScalars* sc,
                                                PcgShared* sh, int parity) {
  static_assert(NT <= 4, "8 and 16 columns: k_spmv_sub");
  constexpr int KG = KGroup<NT>::v, TR = NT / KG;
  __shared__ double lds[8 * KG];
  const int blk = blockIdx.x / TR, g = blockIdx.x % TR, k0 = g * KG;
  const int nblk = gridDim.x / TR;
  auto vi = [&](int64_t row, int k) { return ((size_t)g * n + row) * KG + k; };  // vix<NT>(n, row, k0 + k)
  const int done_flag = *(volatile const int32_t*)&sh->all_done;
  const int nrhs = sh->nrhs, flexible = sh->flexible;
  double rzo[KG], alph[KG];
  int sdone[KG], sit[KG];
#pragma unroll
  for (int k = 0; k < KG; ++k) {
    rzo[k] = sc[k0 + k].rzv[1 - parity];
    alph[k] = sc[k0 + k].alpha;
    sdone[k] = sc[k0 + k].done;
    sit[k] = sc[k0 + k].it;
  }
  double rzq[2 * KG];
#pragma unroll
  for (int k = 0; k < 2 * KG; ++k) rzq[k] = 0.0;
  static_assert(TR == 1, "one group of columns");
  fold_rows<2 * NT>(pd, npd, threadIdx.x, blockDim.x, rzq);  // rows of pd: (r, z) then (q, z)
  double pq[KG];
#pragma unroll
  for (int k = 0; k < KG; ++k) pq[k] = 0.0;
  double beta[KG];
  // beta from the folded partials; the first workgroup of each group stores
  // the scalars
  auto set_beta = [&]() {
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      beta[k] = 0.0;
      if (k0 + k >= nrhs || sdone[k]) continue;
      const double rzn = rzq[k];
      int done = 0;
      if (!(rzn > 0.0)) {
        done = 1;
      } else if (sit[k] > 0) {
        beta[k] = flexible ? -alph[k] * rzq[KG + k] / rzo[k] : rzn / rzo[k];
      }
      if (blk == 0 && threadIdx.x == 0) {
        PcgScalars& S = sc[k0 + k];
        S.rzv[parity] = rzn;
        S.rz = rzn;
        S.qz = rzq[KG + k];
        S.beta = beta[k];
        if (done) {
          S.done = 1;
          S.status = AM_ERR_BREAKDOWN;
        }
      }
    }
  };
  // p_new and q of row i from its ELL row (v), own values and gathers
  auto finish_row = [&](int64_t i, const double (&v)[MAXW], const double (&zi)[KG],
                        const double (&pi)[KG], const double (&zc)[MAXW][KG],
                        const double (&pc)[MAXW][KG]) {
    double acc[KG];
#pragma unroll
    for (int k = 0; k < KG; ++k) acc[k] = 0.0;
#pragma unroll
    for (int c = 0; c < MAXW; ++c)
#pragma unroll
      for (int k = 0; k < KG; ++k) acc[k] = fma(v[c], fma(beta[k], pc[c][k], zc[c][k]), acc[k]);
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      const double pn = fma(beta[k], pi[k], zi[k]);
      pnew[vi(i, k)] = pn;
      q[vi(i, k)] = acc[k];
      pq[k] = fma(pn, acc[k], pq[k]);
    }
  };
  const int64_t stride = (int64_t)nblk * blockDim.x;
  if constexpr (KG <= 2 && MAXW <= 8) {
    // Software pipeline over the rows of this thread: the ELL row and the
    // own values of the next row are loaded while the gathers of the current
    // row are in flight, so a row costs one memory round trip, not two.
    // (With 4 columns per row the extra registers cost more than this saves.)
    int32_t coln[MAXW];
    double vn[MAXW], zin[KG], pin[KG];
    auto load_row = [&](int64_t row) {
      const bool okr = row < n;
#pragma unroll
      for (int c = 0; c < MAXW; ++c) {
        coln[c] = (okr && c < w) ? ec[(int64_t)c * n + row] : 0;
        vn[c] = (okr && c < w) ? ev[(int64_t)c * n + row] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < KG; ++k) {
        zin[k] = okr ? z[vi(row, k)] : 0.0;
        pin[k] = okr ? pold[vi(row, k)] : 0.0;
      }
    };
    load_row((int64_t)blk * blockDim.x + threadIdx.x);
    block_sum<2 * KG>(rzq, lds);  // with the first row in flight
    if (done_flag) return;        // uniform: every thread read the same flag
    set_beta();
    for (int64_t i0 = (int64_t)blk * blockDim.x; i0 < n; i0 += stride) {
      const int64_t i = i0 + threadIdx.x;
      int32_t col[MAXW];
      double v[MAXW], zi[KG], pi[KG];
#pragma unroll
      for (int c = 0; c < MAXW; ++c) {
        col[c] = coln[c];
        v[c] = vn[c];
      }
#pragma unroll
      for (int k = 0; k < KG; ++k) {
        zi[k] = zin[k];
        pi[k] = pin[k];
      }
      double zc[MAXW][KG], pc[MAXW][KG];
#pragma unroll
      for (int c = 0; c < MAXW; ++c)
#pragma unroll
        for (int k = 0; k < KG; ++k) {
          zc[c][k] = (c < w) ? z[vi(col[c], k)] : 0.0;
          pc[c][k] = (c < w) ? pold[vi(col[c], k)] : 0.0;
        }
      if (i0 + stride < n) load_row(i + stride);
      if (i < n) finish_row(i, v, zi, pi, zc, pc);
    }
  } else {
    bool first = true;
    for (int64_t i0 = (int64_t)blk * blockDim.x; i0 < n; i0 += stride) {
      const int64_t i = i0 + threadIdx.x;
      const bool ok = i < n;
      int64_t col[MAXW];
      double v[MAXW];
#pragma unroll
      for (int c = 0; c < MAXW; ++c) {
        col[c] = (ok && c < w) ? ec[(int64_t)c * n + i] : 0;
        v[c] = (ok && c < w) ? ev[(int64_t)c * n + i] : 0.0;
      }
      double zc[MAXW][KG], pc[MAXW][KG], zi[KG], pi[KG];
#pragma unroll
      for (int k = 0; k < KG; ++k) {
        zi[k] = ok ? z[vi(i, k)] : 0.0;
        pi[k] = ok ? pold[vi(i, k)] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < MAXW; ++c)
#pragma unroll
        for (int k = 0; k < KG; ++k) {
          zc[c][k] = (c < w) ? z[vi(col[c], k)] : 0.0;
          pc[c][k] = (c < w) ? pold[vi(col[c], k)] : 0.0;
        }
      if (first) {  // fold the (r, z), (q, z) partials while the gathers are in flight
        first = false;
        block_sum<2 * KG>(rzq, lds);
        if (done_flag) return;  // uniform: every thread read the same flag
        set_beta();
      }
      if (ok) finish_row(i, v, zi, pi, zc, pc);
    }
    if (first) {  // a workgroup with no rows still folds (and may be the writer)
      block_sum<2 * KG>(rzq, lds);
      if (done_flag) return;
    }
  }
  block_sum<KG>(pq, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < KG; ++k) pa[(size_t)blk * NT + k0 + k] = pq[k];
}

// Interface partial right-hand sides of subdomain s for the KG columns
// k0 .. k0+KG-1 of vectors with NT values per row (see bpart_sub).
template <int NT, int KG>
__device__ __forceinline__ void bpart_sub_g(int s, int k0, int64_t n, const int64_t* __restrict__ sub_ptr,
                                            const int64_t* __restrict__ isub_ptr,
                                            const int64_t* __restrict__ mbf_off,
                                            const double* __restrict__ mbf,
                                            const int64_t* __restrict__ bdst, const double* r,
                                            double* bpart, double* lds) {
  // MBF slots per round: six cover a box subdomain (one interface per face)
  // in one round, with fewer registers than eight
  constexpr int QB = KG <= 2 ? 6 : 4;
  const int64_t base = sub_ptr[s];
  const int N = (int)(sub_ptr[s + 1] - base);
  const int64_t i0 = isub_ptr[s];
  const int ns = (int)(isub_ptr[s + 1] - i0);
  const double* P = mbf + mbf_off[s];
  for (int q0 = 0; q0 < ns; q0 += QB) {
    double v[QB * KG];
#pragma unroll
    for (int t = 0; t < QB * KG; ++t) v[t] = 0.0;
#pragma unroll 2
    for (int row = threadIdx.x; row < N; row += blockDim.x) {
      double rv[KG];
#pragma unroll
      for (int k = 0; k < KG; ++k) rv[k] = r[vix<NT>(n, base + row, k0 + k)];
#pragma unroll
      for (int qq = 0; qq < QB; ++qq) {
        const double ph = (q0 + qq < ns) ? P[(size_t)(q0 + qq) * N + row] : 0.0;
#pragma unroll
        for (int k = 0; k < KG; ++k) v[qq * KG + k] = fma(ph, rv[k], v[qq * KG + k]);
      }
    }
    block_sum<QB * KG>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
      for (int qq = 0; qq < QB; ++qq)
        if (q0 + qq < ns)
#pragma unroll
          for (int k = 0; k < KG; ++k)
            bpart[(size_t)bdst[i0 + q0 + qq] * NT + k0 + k] = 0.25 * v[qq * KG + k];
  }
}

// x += alpha p, r -= alpha q on one subdomain and column group per
// workgroup, its ||r||^2 partial, and the interface partial right-hand sides
//   bpart[2n + side] = 1/4 phat^(n)_s . r_s
// from the updated r held in registers.  alpha = (r, z) / (p, Ap) from the
// SpMV partials, folded in every workgroup; the first subdomain's workgroup
// of each group stores alpha and counts the iteration.  The stop flag,
// scalars and partials are loaded before the rows, the decisions taken once
// the rows are in flight.  Rows per thread: up to RPT.
template <int NT>
__global__ __launch_bounds__(256) void k_update_xr(
    int64_t n, const int64_t* __restrict__ sub_ptr, const int64_t* __restrict__ isub_ptr,
    const int64_t* __restrict__ mbf_off, const double* __restrict__ mbf,
    const int64_t* __restrict__ bdst, const double* __restrict__ p, const double* __restrict__ q,
    double* __restrict__ x, double* r, double* bpart, const double* __restrict__ pa, int npa,
    double* __restrict__ pb, PcgScalars* sc, PcgShared* sh, int init, int parity) {
  static_assert(NT <= 4, "8 and 16 columns: k_update_rows");
  constexpr int KG = KGroup<NT>::v, TR = NT / KG;
  // two rows per thread cover a 512-cell subdomain in one pass with half the
  // registers of four (more workgroups resident where there are many)
  constexpr int RPT = 2;
  // MBF slots per round as in bpart_sub_g (six: one round for a box
  // subdomain; 91 -> 84 registers with one column)
  constexpr int QB = KG <= 2 ? 6 : 4;
  __shared__ double lds[4 * 32];
  const int s = blockIdx.x / TR, g = blockIdx.x % TR, k0 = g * KG;
  const int done_flag = *(volatile const int32_t*)&sh->all_done;
  const int nrhs = sh->nrhs;
  double rzc[KG];
  int sdone[KG], sit[KG];
#pragma unroll
  for (int k = 0; k < KG; ++k) {
    rzc[k] = sc[k0 + k].rzv[parity];
    sdone[k] = sc[k0 + k].done;
    sit[k] = sc[k0 + k].it;
  }
  double pqs[KG];
#pragma unroll
  for (int k = 0; k < KG; ++k) pqs[k] = 0.0;
  static_assert(TR == 1, "one group of columns");
  if (!init) fold_rows<NT>(pa, npa, threadIdx.x, blockDim.x, pqs);
  const int64_t base = sub_ptr[s];
  const int N = (int)(sub_ptr[s + 1] - base);
  const int64_t i0 = isub_ptr[s];
  const int ns = (int)(isub_ptr[s + 1] - i0);
  const double* P = mbf + mbf_off[s];
  const int tid = threadIdx.x;
  double rr[KG];
#pragma unroll
  for (int k = 0; k < KG; ++k) rr[k] = 0.0;
  double alpha[KG];
#pragma unroll
  for (int k = 0; k < KG; ++k) alpha[k] = 0.0;
  bool have_alpha = false;
  for (int r0 = 0; r0 < N; r0 += RPT * 256) {
    double xv[RPT][KG], pv[RPT][KG], rv[RPT][KG], qv[RPT][KG], ph[RPT][QB];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int row = r0 + tid + 256 * u;
      const bool ok = row < N;
#pragma unroll
      for (int k = 0; k < KG; ++k) {
        const size_t o = vix<NT>(n, base + row, k0 + k);
        rv[u][k] = ok ? r[o] : 0.0;
        xv[u][k] = (ok && !init) ? x[o] : 0.0;
        pv[u][k] = (ok && !init) ? p[o] : 0.0;
        qv[u][k] = (ok && !init) ? q[o] : 0.0;
      }
#pragma unroll
      for (int qq = 0; qq < QB; ++qq)
        ph[u][qq] = (ok && qq < ns) ? P[(size_t)qq * N + row] : 0.0;
    }
    if (!have_alpha) {
      have_alpha = true;
      if (!init) block_sum<KG>(pqs, lds);
      if (done_flag) return;  // uniform
      if (!init) {
#pragma unroll
        for (int k = 0; k < KG; ++k) {
          if (k0 + k >= nrhs || sdone[k]) continue;
          int done = 0;
          if (!(pqs[k] > 0.0))
            done = 1;
          else
            alpha[k] = rzc[k] / pqs[k];
          if (s == 0 && tid == 0) {
            PcgScalars& S = sc[k0 + k];
            S.pq = pqs[k];
            S.alpha = alpha[k];
            if (done) {
              S.done = 1;
              S.status = AM_ERR_BREAKDOWN;
            } else {
              S.it = sit[k] + 1;
            }
          }
        }
      }
    }
    double vb[QB * KG];
#pragma unroll
    for (int t = 0; t < QB * KG; ++t) vb[t] = 0.0;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int row = r0 + tid + 256 * u;
      if (row >= N) continue;
#pragma unroll
      for (int k = 0; k < KG; ++k) {
        const size_t o = vix<NT>(n, base + row, k0 + k);
        double rn = rv[u][k];
        if (!init) {
          x[o] = fma(alpha[k], pv[u][k], xv[u][k]);
          rn = fma(-alpha[k], qv[u][k], rn);
          r[o] = rn;
        }
        rr[k] = fma(rn, rn, rr[k]);
        rv[u][k] = rn;
#pragma unroll
        for (int qq = 0; qq < QB; ++qq) vb[qq * KG + k] = fma(ph[u][qq], rn, vb[qq * KG + k]);
      }
    }
    if (N <= RPT * 256) {
      // single pass: the first QB slots from registers, the rest re-read
      block_sum<QB * KG>(vb, lds);
      if (tid == 0)
#pragma unroll
        for (int qq = 0; qq < QB; ++qq)
          if (qq < ns)
#pragma unroll
            for (int k = 0; k < KG; ++k) bpart[(size_t)bdst[i0 + qq] * NT + k0 + k] = 0.25 * vb[qq * KG + k];
      for (int q0 = QB; q0 < ns; q0 += QB) {
        double vc[QB * KG];
#pragma unroll
        for (int t = 0; t < QB * KG; ++t) vc[t] = 0.0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int row = tid + 256 * u;
          if (row >= N) continue;
#pragma unroll
          for (int qq = 0; qq < QB; ++qq) {
            const double phv = (q0 + qq < ns) ? P[(size_t)(q0 + qq) * N + row] : 0.0;
#pragma unroll
            for (int k = 0; k < KG; ++k) vc[qq * KG + k] = fma(phv, rv[u][k], vc[qq * KG + k]);
          }
        }
        block_sum<QB * KG>(vc, lds);
        if (tid == 0)
#pragma unroll
          for (int qq = 0; qq < QB; ++qq)
            if (q0 + qq < ns)
#pragma unroll
              for (int k = 0; k < KG; ++k)
                bpart[(size_t)bdst[i0 + q0 + qq] * NT + k0 + k] = 0.25 * vc[qq * KG + k];
      }
    }
  }
  if (N > RPT * 256) {
    __syncthreads();
    bpart_sub_g<NT, KG>(s, k0, n, sub_ptr, isub_ptr, mbf_off, mbf, bdst, r, bpart, lds);
  }
  block_sum<KG>(rr, lds);
  if (tid == 0)
#pragma unroll
    for (int k = 0; k < KG; ++k) pb[(size_t)s * NT + k0 + k] = rr[k];
}

// ---------------------------------------------------------------------------
// 8 and 16 right-hand sides.  A row's NT values are contiguous (vix) and the
// TR = NT / 4 threads of a row are neighbouring lanes, each with a group of
// four columns: the lanes of a row load the same ELL entries (one request
// per wave) and together one line of each vector per row and per gathered
// neighbour, so the matrix, the basis functions and every vector line are
// fetched once for all columns.

// Workgroup sums of NT (8 or 16) columns held as groups of four per thread
// (group g = threadIdx.x % (NT / 4)): the lanes of a group are summed with
// shuffles, then the four waves in order; out[c] for c < NT.
template <int NT>
__device__ __forceinline__ void group_sum(double (&v)[4], double* lds, double* out) {
  constexpr int TR = NT / 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int off = TR; off < 64; off <<= 1) v[k] += __shfl_xor(v[k], off, 64);
  if (lane < TR)
#pragma unroll
    for (int k = 0; k < 4; ++k) lds[wv * NT + lane * 4 + k] = v[k];
  __syncthreads();
  if (threadIdx.x < NT) {
    const int c = threadIdx.x;
    out[c] = ((lds[c] + lds[NT + c]) + lds[2 * NT + c]) + lds[3 * NT + c];
  }
}

// The step coefficients of NT (8 or 16) columns, once per launch instead of
// in every workgroup of the kernel that uses them: one workgroup per column
// sums that column's partials (thread t the rows t, t + 1024, ... in order,
// then the threads in wave order, the same on every run) and takes the
// decision workgroup 0 takes for fewer columns.
//   kind 0: beta from the (r, z), (q, z) partials of the preconditioner
//           launch, part = [nb][2 NT]; coef[c] = beta (Fletcher-Reeves, or
//           the flexible Polak-Ribiere form), 0 for a stopped column;
//   kind 1: alpha = (r, z) / (p, A p) from the SpMV partials,
//           part = [nb][NT]; coef[kMaxNRHS + c] = alpha, 0 for a stopped
//           column; counts the iteration.
// A breakdown ((r, z) or (p, A p) not positive) stops the column with
// AM_ERR_BREAKDOWN and gives it coefficient 0.
template <int NT>
__global__ __launch_bounds__(1024) void k_pcg_coef(int kind, const double* __restrict__ part, int nb,
                                                   double* __restrict__ coef, PcgScalars* sc,
                                                   PcgShared* sh, int parity) {
  __shared__ double lds[16 * 2];
  if (*(volatile const int32_t*)&sh->all_done) return;  // uniform
  const int c = blockIdx.x;
  const int stride = kind == 0 ? 2 * NT : NT;
  double v[2] = {0.0, 0.0};
  for (int b0 = threadIdx.x; b0 < nb; b0 += 4 * blockDim.x) {  // four rows' loads together
    double a[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = min(b0 + u * (int)blockDim.x, nb - 1);
      a[u][0] = part[(size_t)b * stride + c];
      a[u][1] = kind == 0 ? part[(size_t)b * stride + NT + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (b0 + u * (int)blockDim.x < nb) {
        v[0] += a[u][0];
        v[1] += a[u][1];
      }
  }
  block_sum<2>(v, lds);
  if (threadIdx.x != 0) return;
  PcgScalars& S = sc[c];
  double cf = 0.0;
  if (c < sh->nrhs && !S.done) {
    if (kind == 0) {
      const double rzn = v[0];
      int done = 0;
      if (!(rzn > 0.0))
        done = 1;
      else if (S.it > 0)
        cf = sh->flexible ? -S.alpha * v[1] / S.rzv[1 - parity] : rzn / S.rzv[1 - parity];
      S.rzv[parity] = rzn;
      S.rz = rzn;
      S.qz = v[1];
      S.beta = cf;
      if (done) {
        S.done = 1;
        S.status = AM_ERR_BREAKDOWN;
      }
    } else {
      const double pq = v[0];
      S.pq = pq;
      if (!(pq > 0.0)) {
        S.alpha = 0.0;
        S.done = 1;
        S.status = AM_ERR_BREAKDOWN;
      } else {
        cf = S.rzv[parity] / pq;
        S.alpha = cf;
        S.it = S.it + 1;
      }
    }
  }
  coef[(kind == 0 ? 0 : kMaxNRHS) + c] = cf;
}

// p_new = z + beta p_old, q = A p_new and the (p, q) partials for NT (8 or
// 16) columns, one workgroup per subdomain, beta from k_pcg_coef.  The gathers
// of A p_new dominate this product's traffic through the vector memory
// path (seven neighbours, two vectors each, with p_new formed on the fly), so
// the workgroup first forms p_new on its own rows and keeps the first
// SubCap<NT> of them (all rows of a subdomain of up to 1024 cells with 16
// columns) in LDS; a neighbour inside that range is then read from
// LDS, any other one (another subdomain, or beyond the cap) from z and p_old
// as before.  The NT / 4 lanes of a row are neighbours, each with four
// columns.  The ELL rows of the product are loaded one pass ahead: the first
// pass's before p_new is formed, the next pass's while the current one is
// multiplied.
template <int NT> struct SubCap { static constexpr int v = 16384 / NT; };  // 128 KB of p_new
constexpr int kSpmvSubThreads = 1024;
template <int NT, int MAXW>
__global__ __launch_bounds__(kSpmvSubThreads) void k_spmv_sub(
    int64_t n, int w, const int32_t* __restrict__ ec, const double* __restrict__ ev,
    const double* __restrict__ z, const double* __restrict__ pold, double* __restrict__ pnew,
    double* __restrict__ q, const int64_t* __restrict__ sub_ptr, const double* __restrict__ coef,
    double* __restrict__ pa, PcgShared* sh) {
  static_assert(NT == 8 || NT == 16, "k_spmv_sub: 8 or 16 columns");
  constexpr int KG = 4, TR = NT / KG, NTHR = kSpmvSubThreads, RW = NTHR / TR;
  constexpr int CAP = SubCap<NT>::v;
  constexpr int RPA = CAP / RW;  // rows per thread forming p_new: the LDS rows in one pass
  __shared__ double ps[CAP * NT];
  __shared__ double lds[(NTHR / 64) * NT];
  if (*(volatile const int32_t*)&sh->all_done) return;  // uniform
  const int s = blockIdx.x;
  const int g = threadIdx.x % TR, k0 = g * KG, rsub = threadIdx.x / TR;
  const int64_t base = sub_ptr[s];
  const int N = (int)(sub_ptr[s + 1] - base);
  const int NL = min(N, CAP);  // rows held in LDS
  double beta[KG];
#pragma unroll
  for (int k = 0; k < KG; ++k) beta[k] = coef[k0 + k];
  // ELL row of the product (row index clamped into the subdomain)
  int32_t col[MAXW];
  double v[MAXW];
  auto load_ell = [&](int r) {
    const int64_t i = base + min(r, N - 1);
#pragma unroll
    for (int c = 0; c < MAXW; ++c) {
      col[c] = c < w ? ec[(int64_t)c * n + i] : 0;
      v[c] = c < w ? ev[(int64_t)c * n + i] : 0.0;
    }
  };
  load_ell(rsub);
  // p_new on the subdomain's rows
  const double* zs = z + (size_t)base * NT + k0;
  const double* ps_old = pold + (size_t)base * NT + k0;
  for (int r0 = rsub; r0 < N; r0 += RPA * RW) {
    double zi[RPA][KG], pi[RPA][KG];
#pragma unroll
    for (int u = 0; u < RPA; ++u) {
      const int r = min(r0 + u * RW, N - 1);
#pragma unroll
      for (int k = 0; k < KG; ++k) {
        zi[u][k] = zs[(size_t)r * NT + k];
        pi[u][k] = ps_old[(size_t)r * NT + k];
      }
    }
#pragma unroll
    for (int u = 0; u < RPA; ++u) {
      const int r = r0 + u * RW;
      if (r >= N) continue;
#pragma unroll
      for (int k = 0; k < KG; ++k) {
        const double pn = fma(beta[k], pi[u][k], zi[u][k]);
        pnew[(size_t)(base + r) * NT + k0 + k] = pn;
        if (r < NL) ps[r * NT + k0 + k] = pn;
      }
    }
  }
  __syncthreads();
  // q = A p_new on the subdomain's rows
  double pq[KG];
#pragma unroll
  for (int k = 0; k < KG; ++k) pq[k] = 0.0;
  for (int r = rsub; r < N; r += RW) {
    int32_t cc[MAXW];
    double vv[MAXW];
#pragma unroll
    for (int c = 0; c < MAXW; ++c) {
      cc[c] = col[c];
      vv[c] = v[c];
    }
    if (r + RW < N) load_ell(r + RW);  // the next pass's row, in flight meanwhile
    double acc[KG];
#pragma unroll
    for (int k = 0; k < KG; ++k) acc[k] = 0.0;
#pragma unroll
    for (int c = 0; c < MAXW; ++c) {
      if (c >= w) break;
      const int64_t j = (int64_t)cc[c] - base;
      double pv[KG];
      if (j >= 0 && j < NL) {
#pragma unroll
        for (int k = 0; k < KG; ++k) pv[k] = ps[(int)j * NT + k0 + k];
      } else {
        const size_t o = (size_t)cc[c] * NT + k0;
#pragma unroll
        for (int k = 0; k < KG; ++k) pv[k] = fma(beta[k], pold[o + k], z[o + k]);
      }
#pragma unroll
      for (int k = 0; k < KG; ++k) acc[k] = fma(vv[c], pv[k], acc[k]);
    }
    double pn[KG];
    if (r < NL) {
#pragma unroll
      for (int k = 0; k < KG; ++k) pn[k] = ps[r * NT + k0 + k];
    } else {
      const size_t o = (size_t)(base + r) * NT + k0;
#pragma unroll
      for (int k = 0; k < KG; ++k) pn[k] = fma(beta[k], pold[o + k], z[o + k]);
    }
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      q[(size_t)(base + r) * NT + k0 + k] = acc[k];
      pq[k] = fma(pn[k], acc[k], pq[k]);
    }
  }
  // (p, q) partial of this subdomain: lanes of a group, then the waves in order
  {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < KG; ++k)
#pragma unroll
      for (int off = TR; off < 64; off <<= 1) pq[k] += __shfl_xor(pq[k], off, 64);
    if (lane < TR)
#pragma unroll
      for (int k = 0; k < KG; ++k) lds[wv * NT + lane * KG + k] = pq[k];
    __syncthreads();
    if (threadIdx.x < NT) {
      double t = 0.0;
#pragma unroll
      for (int u = 0; u < NTHR / 64; ++u) t += lds[u * NT + threadIdx.x];
      pa[(size_t)s * NT + threadIdx.x] = t;
    }
  }
}

// x += alpha p, r -= alpha q, ||r||^2 partials and the interface partial
// right-hand sides bpart[2n + side] = 1/4 phat^(n)_s . r_s (as k_update_xr),
// one workgroup per subdomain for all NT (8 or 16) columns, alpha from
// k_pcg_coef.  Lane l of a wave holds column l % 16 of row 4 j + l / 16 of its
// row steps j: that is the B operand of v_mfma_f64_16x16x4f64 (lane l holds
// B[l / 16][l % 16]), and with A = 16 slots of the subdomain's basis
// functions at the same four rows (lane l holds A[l % 16][l / 16]) the slot
// sums are accumulated from the updated r in registers (D[l / 16 + 4 v][l % 16]
// in element v), one tile of 16 slots per accumulator.  Slots beyond
// kTiles * 16 are formed afterwards from r re-read.  Every value of P and of
// the four vectors is read once.
template <int NT, bool INIT>
__global__ __launch_bounds__(256) void k_update_rows(
    int64_t n, const int64_t* __restrict__ sub_ptr, const int64_t* __restrict__ isub_ptr,
    const int64_t* __restrict__ mbf_off, const double* __restrict__ mbf,
    const int64_t* __restrict__ bdst, const double* __restrict__ p, const double* __restrict__ q,
    double* __restrict__ x, double* r, double* bpart, const double* __restrict__ coef,
    double* __restrict__ pb, PcgShared* sh) {
  static_assert(NT == 8 || NT == 16, "k_update_rows: 8 or 16 columns");
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int RS = 4;      // row steps of four rows per wave and pass
  constexpr int kTiles = 2;  // tiles of 16 slots accumulated in registers
  constexpr int PASS = 4 * 4 * RS;
  __shared__ double part[4][16][16];  // [wave][slot][column]
  __shared__ double lds_rr[4][16];
  if (*(volatile const int32_t*)&sh->all_done) return;  // uniform
  const int s = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, li = lane % 16, lk = lane / 16;
  const bool colok = li < NT;
  const int64_t base = sub_ptr[s];
  const int N = (int)(sub_ptr[s + 1] - base);
  const int64_t i0 = isub_ptr[s];
  const int ns = (int)(isub_ptr[s + 1] - i0);
  const int nreg = ns < 16 * kTiles ? (ns + 15) / 16 : kTiles;  // uniform
  const double* P = mbf + mbf_off[s];
  const double alpha = (INIT || !colok) ? 0.0 : coef[kMaxNRHS + li];
  d4 acc[kTiles];
#pragma unroll
  for (int t = 0; t < kTiles; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  double rr = 0.0;
  // this subdomain's rows (uniform bases, 32-bit lane offsets from here on)
  const size_t sb = (size_t)base * NT;
  double* __restrict__ xs = x + sb;
  double* rs = r + sb;
  const double* __restrict__ ps = p + sb;
  const double* __restrict__ qs = q + sb;
  // loads use clamped indices (always in bounds) and zero what lies outside
  const int lic = colok ? li : NT - 1;
  int qo[kTiles];
  bool qok[kTiles];
#pragma unroll
  for (int t = 0; t < kTiles; ++t) {
    const int qq = 16 * t + li;
    qok[t] = t < nreg && qq < ns;
    qo[t] = (qok[t] ? qq : 0) * N;
  }
  // the rows of a wave's next pass are loaded while the current pass is
  // multiplied (four row steps per pass: eight without the overlap measured
  // 209 against 202 us at the 16-RHS grid)
  double rvn[RS], xvn[RS], pvn[RS], qvn[RS], avn[kTiles][RS];
  auto load_pass = [&](int r0) {
#pragma unroll
    for (int j = 0; j < RS; ++j) {
      const int row = r0 + 4 * j + lk;
      const int o = min(row, N - 1) * NT + lic;
      rvn[j] = rs[o];
      if (!INIT) {
        xvn[j] = xs[o];
        pvn[j] = ps[o];
        qvn[j] = qs[o];
      } else {
        xvn[j] = pvn[j] = qvn[j] = 0.0;  // unused
      }
#pragma unroll
      for (int t = 0; t < kTiles; ++t) avn[t][j] = P[qo[t] + min(row, N - 1)];
    }
  };
  if (wv * 4 * RS < N) load_pass(wv * 4 * RS);
  for (int r0 = wv * 4 * RS; r0 < N; r0 += PASS) {  // uniform in the wave
    double rv[RS], xv[RS], pv[RS], qv[RS], av[kTiles][RS];
#pragma unroll
    for (int j = 0; j < RS; ++j) {
      rv[j] = rvn[j];
      xv[j] = xvn[j];
      pv[j] = pvn[j];
      qv[j] = qvn[j];
#pragma unroll
      for (int t = 0; t < kTiles; ++t) av[t][j] = avn[t][j];
    }
    if (r0 + PASS < N) load_pass(r0 + PASS);
#pragma unroll
    for (int j = 0; j < RS; ++j) {
      const int row = r0 + 4 * j + lk;
      const bool ok = row < N && colok;
      const int o = row * NT + li;
      double rn = rv[j];
      if (!INIT) {
        rn = fma(-alpha, qv[j], rn);
        if (ok) {
          xs[o] = fma(alpha, pv[j], xv[j]);
          rs[o] = rn;
        }
      }
      rn = ok ? rn : 0.0;
      rr = fma(rn, rn, rr);
#pragma unroll
      for (int t = 0; t < kTiles; ++t)
        if (t < nreg)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(qok[t] ? av[t][j] : 0.0, rn, acc[t], 0, 0, 0);
    }
  }
  // ||r||^2: lanes of one column, then the waves in order
  rr += __shfl_xor(rr, 16, 64);
  rr += __shfl_xor(rr, 32, 64);
  if (lane < 16) lds_rr[wv][lane] = rr;
  __syncthreads();
  if (tid < NT) pb[(size_t)s * NT + tid] = ((lds_rr[0][tid] + lds_rr[1][tid]) + lds_rr[2][tid]) + lds_rr[3][tid];
  // the register tiles: the four waves' partial products added in wave order
  for (int t = 0; t < nreg; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) part[wv][lk + 4 * v][li] = acc[0][v];
    __syncthreads();
    {
      const int qi = tid / 16, k = tid % 16;
      if (16 * t + qi < ns && k < NT) {
        const double sum = ((part[0][qi][k] + part[1][qi][k]) + part[2][qi][k]) + part[3][qi][k];
        bpart[(size_t)bdst[i0 + 16 * t + qi] * NT + k] = 0.25 * sum;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u + 1 < kTiles; ++u) acc[u] = acc[u + 1];  // the next tile into acc[0]
  }
  // slots beyond the register tiles, from the updated r
  for (int q0 = 16 * kTiles; q0 < ns; q0 += 16) {
    d4 a4 = {0.0, 0.0, 0.0, 0.0};
    const int qq = q0 + li;
    for (int row0 = 4 * wv; row0 < N; row0 += 16) {
      const int row = row0 + lk;
      const double a = (row < N && qq < ns) ? P[(size_t)qq * N + row] : 0.0;
      const double b = (row < N && colok) ? r[(size_t)(base + row) * NT + li] : 0.0;
      a4 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, a4, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) part[wv][lk + 4 * v][li] = a4[v];
    __syncthreads();
    {
      const int qi = tid / 16, k = tid % 16;
      if (q0 + qi < ns && k < NT) {
        const double sum = ((part[0][qi][k] + part[1][qi][k]) + part[2][qi][k]) + part[3][qi][k];
        bpart[(size_t)bdst[i0 + q0 + qi] * NT + k] = 0.25 * sum;
      }
    }
    __syncthreads();
  }
}

// ||b - A x||^2 per column (device positions).
template <int NR>
__global__ __launch_bounds__(256) void k_true_res(int64_t n, int w, const int32_t* __restrict__ ec,
                                                  const double* __restrict__ ev,
                                                  const double* __restrict__ b,
                                                  const double* __restrict__ x, double* partial,
                                                  unsigned* counter, double* out) {
  __shared__ double lds[4 * NR];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) v[k] = 0.0;
  if (i < n) {
    double acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = b[vix<NR>(n, i, k)];
    for (int c = 0; c < w; ++c) {
      const int64_t col = ec[(int64_t)c * n + i];
      const double a = ev[(int64_t)c * n + i];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] = fma(-a, x[vix<NR>(n, col, k)], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) v[k] = acc[k] * acc[k];
  }
  block_sum<NR>(v, lds);
  if (!publish_partial<NR>(v, partial, counter, gridDim.x)) return;
  double tot[NR];
  reduce_partials<NR>(tot, partial, gridDim.x, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NR; ++k) out[k] = tot[k];
    *counter = 0u;
    __threadfence();
  }
}

// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

#define AM_NR_SWITCH(nr, CALL)          \
  switch (nr) {                         \
    case 1: { constexpr int NR = 1; CALL; } break;   \
    case 2: { constexpr int NR = 2; CALL; } break;   \
    case 4: { constexpr int NR = 4; CALL; } break;   \
    case 8: { constexpr int NR = 8; CALL; } break;   \
    case 16: { constexpr int NR = 16; CALL; } break; \
    default: return hipErrorInvalidValue;            \
  }

hipError_t launch_permute_in(const int32_t* dperm, int64_t n, const double* src, int64_t ld,
                             double* dst, int nrhs, hipStream_t s) {
  int nr = 1;
  while (nr < nrhs) nr *= 2;
  AM_NR_SWITCH(nr, hipLaunchKernelGGL(k_permute_in<NR>, dim3(nblk(n)), dim3(256), 0, s, dperm, n,
                                      src, ld, nrhs, dst));
  return hipGetLastError();
}

hipError_t launch_permute_out(const int32_t* dperm, int64_t n, const double* src, double* dst,
                              int64_t ld, int nrhs, hipStream_t s) {
  int nr = 1;
  while (nr < nrhs) nr *= 2;
  AM_NR_SWITCH(nr, hipLaunchKernelGGL(k_permute_out<NR>, dim3(nblk(n)), dim3(256), 0, s, dperm,
                                       n, src, nrhs, dst, ld));
  return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(nblk(count)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t launch_pcg_init(DeviceState& d, int nr, double tol, int maxit, int flexible,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, s, d.sc, d.shared, nr, nr, tol * tol,
                     maxit, flexible);
  return hipGetLastError();
}

// SpMV workgroups with up to four columns (and so (p, Ap) partials per
// column): at most 1024, one round of resident workgroups.  Every workgroup
// of the SpMV and update launches folds the partials it needs itself.  (With
// 8-16 columns the SpMV has one workgroup per subdomain and k_pcg_coef folds
// the partials once per launch.)
template <int NR>
static int spmv_grid(const DeviceState& d) {
  return std::max(1, d.red.spmv_blocks);
}

static hipError_t update_xr(DeviceState& d, int nr, int parity, int init, hipStream_t s) {
  const double* pn = d.p[1 - parity];
  AM_NR_SWITCH(nr, if constexpr (NR >= 8) {
    if (!init)  // (p, Ap) partials: one per subdomain (k_spmv_sub)
      am_launch(d, true, false, k_pcg_coef<NR>, dim3(NR), dim3(1024), s, 1, d.red.pa, d.m,
                d.red.coef, d.sc, d.shared, parity);
    auto kern = (init ? &k_update_rows<NR, true> : &k_update_rows<NR, false>);
    am_launch(d, init != 0, true, kern, dim3(d.m), dim3(256), s, d.n, d.sub_ptr, d.isub_ptr,
              d.mbf_off, d.mbf, d.bdst, pn, d.q, d.x, d.r, d.bpart, d.red.coef, d.red.pb,
              d.shared);
  } else {
    am_launch(d, true, true, k_update_xr<NR>, dim3(d.m), dim3(256), s, d.n, d.sub_ptr,
              d.isub_ptr, d.mbf_off, d.mbf, d.bdst, pn, d.q, d.x, d.r, d.bpart, d.red.pa,
              spmv_grid<NR>(d), d.red.pb, d.sc, d.shared, init, parity);
  });
  return hipGetLastError();
}

hipError_t launch_pcg_start(DeviceState& d, int nr, hipStream_t s) {
  hipError_t e = update_xr(d, nr, 0, 1, s);
  if (e != hipSuccess) return e;
  if (!d.fuse_eta) {
    e = launch_iface_gemv(d, nr, 1, 1, s);
    if (e != hipSuccess) return e;
  }
  return launch_local_sweep(d, d.r, d.z, d.eta, nr, 12, s);
}

hipError_t launch_pcg_rr0(DeviceState& d, int nr, hipStream_t s) {
  return update_xr(d, nr, 0, 1, s);
}

hipError_t launch_pcg_spmv(DeviceState& d, int nr, int parity, hipStream_t s) {
  const double* po = d.p[parity];
  double* pn = d.p[1 - parity];
  auto go = [&](auto maxw) -> hipError_t {
    constexpr int MW = decltype(maxw)::value;
    AM_NR_SWITCH(nr, if constexpr (NR >= 8) {
      am_launch(d, true, false, k_pcg_coef<NR>, dim3(NR), dim3(1024), s, 0, d.red.pd, d.m,
                d.red.coef, d.sc, d.shared, parity);
      am_launch(d, false, true, k_spmv_sub<NR, MW>, dim3(d.m), dim3(kSpmvSubThreads), s, d.n, d.ell_w,
                d.ell_col, d.ell_val, d.z, po, pn, d.q, d.sub_ptr, d.red.coef, d.red.pa, d.shared);
    } else {
      am_launch(d, true, true, k_spmv_p<NR, MW>, dim3(spmv_grid<NR>(d)), dim3(256), s, d.n,
                d.ell_w, d.ell_col, d.ell_val, d.z, po, pn, d.q, d.red.pd, d.m, d.red.pa, d.sc,
                d.shared, parity);
    });
    return hipSuccess;
  };
  hipError_t e = d.ell_w <= 8 ? go(std::integral_constant<int, 8>{})
                              : go(std::integral_constant<int, 32>{});
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_pcg_update(DeviceState& d, int nr, int parity, hipStream_t s) {
  return update_xr(d, nr, parity, 0, s);
}

hipError_t launch_pcg_iteration(DeviceState& d, int nr, int parity, hipStream_t s) {
  hipError_t e = launch_pcg_spmv(d, nr, parity, s);
  if (e != hipSuccess) return e;
  e = update_xr(d, nr, parity, 0, s);
  if (e != hipSuccess) return e;
  if (!d.fuse_eta) {
    e = launch_iface_gemv(d, nr, 1, 0, s);
    if (e != hipSuccess) return e;
  }
  return launch_local_sweep(d, d.r, d.z, d.eta, nr, 2, s);
}

hipError_t launch_true_residual(DeviceState& d, const double* bperm, int nr, double* out2,
                                hipStream_t s) {
  AM_NR_SWITCH(nr, hipLaunchKernelGGL(k_true_res<NR>, dim3(nblk(d.n)), dim3(256), 0, s, d.n,
                                      d.ell_w, d.ell_col, d.ell_val, bperm, d.x, d.red.partial,
                                      d.red.counter + 3, out2));
  return hipGetLastError();
}

}  // namespace am
