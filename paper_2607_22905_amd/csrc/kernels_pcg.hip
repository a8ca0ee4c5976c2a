// PCG kernels for gfx950 (Sec. 5: AlgMortar as the CG preconditioner; Sec. 7:
// x0 = 0, relative residual stop).  One iteration is four launches:
//   spmv_p   : p = z + beta p (ping-pong buffers), q = A p, (p, q) -> alpha
//   update_xr: x += alpha p, r -= alpha q, ||r||^2 -> stop test; interface
//              partial right-hand sides 1/4 phat^T r per (subdomain, slot)
//   gemv     : eta = S^{-1} b                         (kernels_iface.hip)
//   local    : z = A_i^{-1} r + sum eta_m phat^(m), (r, z) -> beta (kernels_local.hip)
// Scalars stay on the device; every reducing launch folds its per-block
// partial sums in its last block, in block order (deterministic).  Every
// launch returns at once when all columns have stopped, so a captured chunk
// of iterations can run past convergence harmlessly.
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

// p_new = z + beta p_old; q = A p_new (ELL, column-major, device positions);
// the last block turns (p, q) into alpha.
template <int NR>
__global__ __launch_bounds__(256) void k_spmv_p(int64_t n, int w, const int32_t* __restrict__ ec,
                                                const double* __restrict__ ev,
                                                const double* __restrict__ z,
                                                const double* __restrict__ pold,
                                                double* __restrict__ pnew, double* __restrict__ q,
                                                double* partial, unsigned* counter,
                                                PcgScalars* sc, PcgShared* sh) {
  if (all_done(sh)) return;
  __shared__ double lds[4 * NR];
  double beta[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) beta[k] = sc[k].beta;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double pq[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) pq[k] = 0.0;
  if (i < n) {
    double acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = 0.0;
    for (int c = 0; c < w; ++c) {
      const int64_t col = ec[(int64_t)c * n + i];
      const double v = ev[(int64_t)c * n + i];
#pragma unroll
      for (int k = 0; k < NR; ++k)
        acc[k] = fma(v, fma(beta[k], pold[col * NR + k], z[col * NR + k]), acc[k]);
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const double pn = fma(beta[k], pold[i * NR + k], z[i * NR + k]);
      pnew[i * NR + k] = pn;
      q[i * NR + k] = acc[k];
      pq[k] = pn * acc[k];
    }
  }
  block_sum<NR>(pq, lds);
  if (!publish_partial<NR>(pq, partial, counter, gridDim.x)) return;
  double tot[NR];
  reduce_partials<NR>(tot, partial, gridDim.x, lds);
  if (threadIdx.x == 0) {
    for (int k = 0; k < sh->nrhs; ++k) {
      PcgScalars& S = sc[k];
      if (S.done) continue;
      S.pq = tot[k];
      if (!(tot[k] > 0.0)) {
        S.status = AM_ERR_BREAKDOWN;
        S.done = 1;
        S.alpha = 0.0;
      } else {
        S.alpha = S.rz / tot[k];
        S.it += 1;
      }
    }
    *counter = 0u;
    __threadfence();
  }
}

// x += alpha p, r -= alpha q on one subdomain per block, ||r||^2, then the
// interface partial right-hand sides from the updated r.  The last block
// applies the stop test ||r|| <= tol ||b|| (init: records ||b||^2).
template <int NR>
__global__ __launch_bounds__(256) void k_update_xr(
    const int64_t* __restrict__ sub_ptr, const int64_t* __restrict__ isub_ptr,
    const int64_t* __restrict__ mbf_off, const double* __restrict__ mbf,
    const double* __restrict__ p, const double* __restrict__ q, double* __restrict__ x, double* r,
    double* bpart, double* partial, unsigned* counter, PcgScalars* sc, PcgShared* sh, int init) {
  if (all_done(sh)) return;
  __shared__ double lds[4 * NR];
  const int s = blockIdx.x;
  double alpha[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) alpha[k] = (init || sc[k].done) ? 0.0 : sc[k].alpha;
  const int64_t b0 = sub_ptr[s], b1 = sub_ptr[s + 1];
  double rr[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) rr[k] = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int64_t o = i * NR + k;
      if (!init) {
        x[o] = fma(alpha[k], p[o], x[o]);
        r[o] = fma(-alpha[k], q[o], r[o]);
      }
      rr[k] = fma(r[o], r[o], rr[k]);
    }
  }
  __syncthreads();
  bpart_sub<NR>(s, sub_ptr, isub_ptr, mbf_off, mbf, r, bpart, lds);
  block_sum<NR>(rr, lds);
  if (!publish_partial<NR>(rr, partial, counter, gridDim.x)) return;
  double tot[NR];
  reduce_partials<NR>(tot, partial, gridDim.x, lds);
  if (threadIdx.x == 0) {
    int alld = 1;
    for (int k = 0; k < sh->nrhs; ++k) {
      PcgScalars& S = sc[k];
      if (!S.done) {
        S.rr = tot[k];
        if (init) {
          S.bb = tot[k];
          if (tot[k] == 0.0) {
            S.conv = 1;
            S.done = 1;
          }
        } else if (tot[k] <= S.tol2 * S.bb) {
          S.conv = 1;
          S.done = 1;
        } else if (S.it >= sh->maxit) {
          S.status = AM_ERR_NO_CONVERGENCE;
          S.done = 1;
        }
      }
      alld &= S.done;
    }
    sh->all_done = alld;
    *counter = 0u;
    __threadfence();
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
                                      d.isub_ptr, d.mbf_off, d.mbf, pn, d.q, d.x, d.r, d.bpart,
                                      d.red.partial, d.red.counter + 1, d.sc, d.shared, init));
  return hipGetLastError();
}

hipError_t launch_pcg_start(DeviceState& d, int nr, hipStream_t s) {
  hipError_t e = update_xr(d, nr, 0, 1, s);
  if (e != hipSuccess) return e;
  e = launch_iface_gemv(d, -nr, s);
  if (e != hipSuccess) return e;
  return launch_local_sweep(d, d.r, d.z, d.eta, nr, 12, s);
}

hipError_t launch_pcg_iteration(DeviceState& d, int nr, int parity, hipStream_t s) {
  const double* po = d.p[parity];
  double* pn = d.p[1 - parity];
  AM_NR_SWITCH(nr, hipLaunchKernelGGL(k_spmv_p<NR>, dim3(nblk(d.n)), dim3(256), 0, s, d.n,
                                      d.ell_w, d.ell_col, d.ell_val, d.z, po, pn, d.q,
                                      d.red.partial, d.red.counter + 0, d.sc, d.shared));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = update_xr(d, nr, parity, 0, s);
  if (e != hipSuccess) return e;
  e = launch_iface_gemv(d, -nr, s);
  if (e != hipSuccess) return e;
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
