// PCG kernels for gfx950 (Sec. 5: AlgMortar as the CG preconditioner; Sec. 7:
// x0 = 0, relative residual stop).  One iteration is four launches:
//   spmv_p   : beta from (r, z); p = z + beta p (ping-pong buffers), q = A p, (p, q)
//   update_xr: alpha = (r, z)/(p, q); x += alpha p, r -= alpha q, ||r||^2; the
//              interface partial right-hand sides 1/4 phat^T r per (subdomain, slot)
//   gemv     : stop test on ||r||; eta = S^{-1} b      (kernels_iface.hip)
//   local    : z = A_i^{-1} r + sum eta_m phat^(m), (r, z), (q, z) (kernels_local.hip)
// Scalars stay on the device.  A launch that needs a scalar folds the per-
// block partial sums of the launch that produced them, in block order and
// identically in every workgroup (deterministic, no fences, no atomics);
// workgroup 0 stores the scalars.  Every launch returns at once when all
// columns have stopped, so a captured chunk of iterations can run past
// convergence harmlessly.
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
  for (int k = 0; k < NR; ++k) dst[i * NR + k] = k < nrhs ? src[k * ld + o] : 0.0;
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
    if (k < nrhs) dst[k * ld + o] = src[i * NR + k];
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

// p_new = z + beta p_old; q = A p_new (ELL, column-major, device positions).
// beta comes from the (r, z), (q, z) partials of the previous local launch,
// folded by every workgroup in block order; workgroup 0 stores rz and beta.
// Every load that does not depend on another one is issued first (the stop
// flag, the scalars, the partials to fold, the ELL rows), then the gathers;
// the stop decision and the fold are taken once they are in flight, so the
// launch costs two memory round trips.  Grid-stride over rows with a fixed
// grid, one (p, q) partial per workgroup.
template <int NR, int MAXW>
__global__ __launch_bounds__(256) void k_spmv_p(int64_t n, int w, const int32_t* __restrict__ ec,
                                                const double* __restrict__ ev,
                                                const double* __restrict__ z,
                                                const double* __restrict__ pold,
                                                double* __restrict__ pnew, double* __restrict__ q,
                                                const double* __restrict__ pd, int npd,
                                                double* __restrict__ pa, PcgScalars* sc,
                                                PcgShared* sh, int parity) {
  __shared__ double lds[8 * NR];
  const int done_flag = *(volatile const int32_t*)&sh->all_done;
  const int nrhs = sh->nrhs, flexible = sh->flexible;
  double rzo[NR], alph[NR];
  int sdone[NR], sit[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    rzo[k] = sc[k].rzv[1 - parity];
    alph[k] = sc[k].alpha;
    sdone[k] = sc[k].done;
    sit[k] = sc[k].it;
  }
  double rzq[2 * NR];
#pragma unroll
  for (int k = 0; k < 2 * NR; ++k) rzq[k] = 0.0;
  for (int bb = threadIdx.x; bb < npd; bb += blockDim.x)
#pragma unroll
    for (int k = 0; k < 2 * NR; ++k) rzq[k] += pd[(size_t)bb * 2 * NR + k];
  double pq[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) pq[k] = 0.0;
  bool first = true;
  double beta[NR];
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    const bool ok = i < n;
    int64_t col[MAXW];
    double v[MAXW];
#pragma unroll
    for (int c = 0; c < MAXW; ++c) {
      col[c] = (ok && c < w) ? ec[(int64_t)c * n + i] : 0;
      v[c] = (ok && c < w) ? ev[(int64_t)c * n + i] : 0.0;
    }
    double zc[MAXW][NR], pc[MAXW][NR], zi[NR], pi[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      zi[k] = ok ? z[i * NR + k] : 0.0;
      pi[k] = ok ? pold[i * NR + k] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < MAXW; ++c)
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        zc[c][k] = (c < w) ? z[col[c] * NR + k] : 0.0;
        pc[c][k] = (c < w) ? pold[col[c] * NR + k] : 0.0;
      }
    if (first) {  // fold the (r, z), (q, z) partials while the gathers are in flight
      first = false;
      block_sum<2 * NR>(rzq, lds);
      if (done_flag) return;  // uniform: every thread read the same flag
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        beta[k] = 0.0;
        if (k >= nrhs || sdone[k]) continue;
        const double rzn = rzq[k];
        int done = 0;
        if (!(rzn > 0.0)) {
          done = 1;
        } else if (sit[k] > 0) {
          beta[k] = flexible ? -alph[k] * rzq[NR + k] / rzo[k] : rzn / rzo[k];
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          sc[k].rzv[parity] = rzn;
          sc[k].rz = rzn;
          sc[k].qz = rzq[NR + k];
          sc[k].beta = beta[k];
          if (done) {
            sc[k].done = 1;
            sc[k].status = AM_ERR_BREAKDOWN;
          }
        }
      }
    }
    if (ok) {
      double acc[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] = 0.0;
#pragma unroll
      for (int c = 0; c < MAXW; ++c)
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = fma(v[c], fma(beta[k], pc[c][k], zc[c][k]), acc[k]);
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const double pn = fma(beta[k], pi[k], zi[k]);
        pnew[i * NR + k] = pn;
        q[i * NR + k] = acc[k];
        pq[k] = fma(pn, acc[k], pq[k]);
      }
    }
  }
  if (first) {  // a workgroup with no rows still folds (and may be workgroup 0)
    block_sum<2 * NR>(rzq, lds);
    if (done_flag) return;
  }
  block_sum<NR>(pq, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NR; ++k) pa[(size_t)blockIdx.x * NR + k] = pq[k];
}

// x += alpha p, r -= alpha q on one subdomain per workgroup, its ||r||^2
// partial, and the interface partial right-hand sides
//   bpart[2n + side] = 1/4 phat^(n)_s . r_s
// from the updated r held in registers.  alpha = (r, z) / (p, Ap) from the
// SpMV partials, folded in every workgroup; workgroup 0 stores alpha and
// counts the iteration.  The row vectors and the MBF values are loaded before
// the fold (one memory round trip).  Rows per thread: up to RPT.
template <int NR>
__global__ __launch_bounds__(256) void k_update_xr(
    const int64_t* __restrict__ sub_ptr, const int64_t* __restrict__ isub_ptr,
    const int64_t* __restrict__ mbf_off, const double* __restrict__ mbf,
    const int64_t* __restrict__ bdst, const double* __restrict__ p, const double* __restrict__ q,
    double* __restrict__ x, double* r, double* bpart, const double* __restrict__ pa, int npa,
    double* __restrict__ pb, PcgScalars* sc, PcgShared* sh, int init, int parity) {
  constexpr int RPT = 4;
  constexpr int QB = NR <= 2 ? 8 : (NR <= 4 ? 4 : (NR <= 8 ? 2 : 1));
  __shared__ double lds[4 * 16];
  // stop flag, scalars and the (p, Ap) partials are loaded before the rows
  // (all independent), the decisions taken once the rows are in flight
  const int done_flag = *(volatile const int32_t*)&sh->all_done;
  const int nrhs = sh->nrhs;
  double rzc[NR];
  int sdone[NR], sit[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    rzc[k] = sc[k].rzv[parity];
    sdone[k] = sc[k].done;
    sit[k] = sc[k].it;
  }
  double pqs[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) pqs[k] = 0.0;
  if (!init)
    for (int bb = threadIdx.x; bb < npa; bb += blockDim.x)
#pragma unroll
      for (int k = 0; k < NR; ++k) pqs[k] += pa[(size_t)bb * NR + k];
  const int s = blockIdx.x;
  const int64_t base = sub_ptr[s];
  const int N = (int)(sub_ptr[s + 1] - base);
  const int64_t i0 = isub_ptr[s];
  const int ns = (int)(isub_ptr[s + 1] - i0);
  const double* P = mbf + mbf_off[s];
  const int tid = threadIdx.x;
  // rows tid + 256 u, u < RPT (subdomains up to 1024 cells; larger ones loop)
  double rr[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) rr[k] = 0.0;
  double alpha[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) alpha[k] = 0.0;
  bool have_alpha = false;
  for (int r0 = 0; r0 < N; r0 += RPT * 256) {
    double xv[RPT][NR], pv[RPT][NR], rv[RPT][NR], qv[RPT][NR], ph[RPT][QB];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int row = r0 + tid + 256 * u;
      const bool ok = row < N;
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const int64_t o = (base + row) * NR + k;
        rv[u][k] = ok ? r[o] : 0.0;
        xv[u][k] = (ok && !init) ? x[o] : 0.0;
        pv[u][k] = (ok && !init) ? p[o] : 0.0;
        qv[u][k] = (ok && !init) ? q[o] : 0.0;
      }
#pragma unroll
      for (int qq = 0; qq < QB; ++qq) ph[u][qq] = (ok && qq < ns) ? P[(size_t)qq * N + row] : 0.0;
    }
    if (!have_alpha) {
      have_alpha = true;
      if (!init) block_sum<NR>(pqs, lds);
      if (done_flag) return;  // uniform
      if (!init) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          if (k >= nrhs || sdone[k]) continue;
          int done = 0;
          if (!(pqs[k] > 0.0))
            done = 1;
          else
            alpha[k] = rzc[k] / pqs[k];
          if (blockIdx.x == 0 && tid == 0) {
            sc[k].pq = pqs[k];
            sc[k].alpha = alpha[k];
            if (done) {
              sc[k].done = 1;
              sc[k].status = AM_ERR_BREAKDOWN;
            } else {
              sc[k].it = sit[k] + 1;
            }
          }
        }
      }
    }
    double vb[QB * NR];
#pragma unroll
    for (int t = 0; t < QB * NR; ++t) vb[t] = 0.0;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int row = r0 + tid + 256 * u;
      if (row >= N) continue;
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const int64_t o = (base + row) * NR + k;
        double rn = rv[u][k];
        if (!init) {
          x[o] = fma(alpha[k], pv[u][k], xv[u][k]);
          rn = fma(-alpha[k], qv[u][k], rn);
          r[o] = rn;
        }
        rr[k] = fma(rn, rn, rr[k]);
        rv[u][k] = rn;
#pragma unroll
        for (int qq = 0; qq < QB; ++qq) vb[qq * NR + k] = fma(ph[u][qq], rn, vb[qq * NR + k]);
      }
    }
    if (N <= RPT * 256) {
      // single pass: the first QB slots from registers, the rest re-read
      block_sum<QB * NR>(vb, lds);
      if (tid == 0)
#pragma unroll
        for (int qq = 0; qq < QB; ++qq)
          if (qq < ns)
#pragma unroll
            for (int k = 0; k < NR; ++k) bpart[(size_t)bdst[i0 + qq] * NR + k] = 0.25 * vb[qq * NR + k];
      for (int q0 = QB; q0 < ns; q0 += QB) {
        double vc[QB * NR];
#pragma unroll
        for (int t = 0; t < QB * NR; ++t) vc[t] = 0.0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int row = tid + 256 * u;
          if (row >= N) continue;
#pragma unroll
          for (int qq = 0; qq < QB; ++qq) {
            const double phv = (q0 + qq < ns) ? P[(size_t)(q0 + qq) * N + row] : 0.0;
#pragma unroll
            for (int k = 0; k < NR; ++k) vc[qq * NR + k] = fma(phv, rv[u][k], vc[qq * NR + k]);
          }
        }
        block_sum<QB * NR>(vc, lds);
        if (tid == 0)
#pragma unroll
          for (int qq = 0; qq < QB; ++qq)
            if (q0 + qq < ns)
#pragma unroll
              for (int k = 0; k < NR; ++k)
                bpart[(size_t)bdst[i0 + q0 + qq] * NR + k] = 0.25 * vc[qq * NR + k];
      }
    }
  }
  if (N > RPT * 256) {
    __syncthreads();
    bpart_sub<NR>(s, sub_ptr, isub_ptr, mbf_off, mbf, bdst, r, bpart, lds);
  }
  block_sum<NR>(rr, lds);
  if (tid == 0)
#pragma unroll
    for (int k = 0; k < NR; ++k) pb[(size_t)s * NR + k] = rr[k];
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
    for (int k = 0; k < NR; ++k) acc[k] = b[i * NR + k];
    for (int c = 0; c < w; ++c) {
      const int64_t col = ec[(int64_t)c * n + i];
      const double a = ev[(int64_t)c * n + i];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] = fma(-a, x[col * NR + k], acc[k]);
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

static hipError_t update_xr(DeviceState& d, int nr, int parity, int init, hipStream_t s) {
  const double* pn = d.p[1 - parity];
  AM_NR_SWITCH(nr, hipLaunchKernelGGL(k_update_xr<NR>, dim3(d.m), dim3(256), 0, s, d.sub_ptr,
                                      d.isub_ptr, d.mbf_off, d.mbf, d.bdst, pn, d.q, d.x, d.r,
                                      d.bpart, d.red.pa, d.red.spmv_blocks, d.red.pb, d.sc,
                                      d.shared, init, parity));
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

hipError_t launch_pcg_spmv(DeviceState& d, int nr, int parity, hipStream_t s) {
  const double* po = d.p[parity];
  double* pn = d.p[1 - parity];
  if (d.ell_w <= 8) {
    AM_NR_SWITCH(nr, hipLaunchKernelGGL((k_spmv_p<NR, 8>), dim3(d.red.spmv_blocks), dim3(256), 0, s,
                                        d.n, d.ell_w, d.ell_col, d.ell_val, d.z, po, pn, d.q,
                                        d.red.pd, d.m, d.red.pa, d.sc, d.shared, parity));
  } else {
    AM_NR_SWITCH(nr, hipLaunchKernelGGL((k_spmv_p<NR, 32>), dim3(d.red.spmv_blocks), dim3(256), 0, s,
                                        d.n, d.ell_w, d.ell_col, d.ell_val, d.z, po, pn, d.q,
                                        d.red.pd, d.m, d.red.pa, d.sc, d.shared, parity));
  }
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
