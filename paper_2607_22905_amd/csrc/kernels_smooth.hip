// Block-Jacobi pre- and post-smoothing around the AlgMortar correction
// (Sec. 5.4), for gfx950.  The smoother's block solves run on a second set
// of band factors, those of the plain diagonal blocks A[K, K] of a coarser
// partition, laid out in that partition's own device order; the AlgMortar
// correction runs in the AlgMortar device order.  Vectors cross between the
// two orders by gathers.  One application z = M^{-1} r, from z = 0:
//   nu times      z <- z + B^{-1} (r - A z)
//   once          z <- z + Mcal^{-1} (r - A z)
//   nu times      z <- z + B^{-1} (r - A z)
// Every "z <- z + w" is folded into the next residual launch, which reads z
// and w and writes both z + w and r - A (z + w).
#include <utility>

#include "am_common.h"

namespace am {

// dst[i] = a[map[i]] (+ b[map[i]]) for the NT values of node i
template <int NT>
__global__ __launch_bounds__(256) void k_gather(int64_t n, const int32_t* __restrict__ map,
                                                const double* __restrict__ a,
                                                const double* __restrict__ b,
                                                double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = map[i];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    double v = a[vix<NT>(n, j, k)];
    if (b) v += b[vix<NT>(n, j, k)];
    dst[vix<NT>(n, i, k)] = v;
  }
}

// u = zin (+ win); zout[i] = u[i] when zout is set; t[i] = r[i] - (A u)[i]
// (ELL, column-major, padded entries point at the row itself with value 0)
template <int NT, int MAXW>
__global__ __launch_bounds__(256) void k_sres(int64_t n, int w, const int32_t* __restrict__ ec,
                                              const double* __restrict__ ev,
                                              const double* __restrict__ r,
                                              const double* __restrict__ zin,
                                              const double* __restrict__ win,
                                              double* __restrict__ zout, double* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t col[MAXW];
  double v[MAXW];
#pragma unroll
  for (int c = 0; c < MAXW; ++c) {
    col[c] = c < w ? ec[(int64_t)c * n + i] : i;
    v[c] = c < w ? ev[(int64_t)c * n + i] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const size_t o = vix<NT>(n, i, k);
    double acc = r[o];
#pragma unroll
    for (int c = 0; c < MAXW; ++c) {
      if (c >= w) break;
      const size_t oc = vix<NT>(n, col[c], k);
      double u = zin[oc];
      if (win) u += win[oc];
      acc = fma(-v[c], u, acc);
    }
    if (zout) {
      double u = zin[o];
      if (win) u += win[o];
      zout[o] = u;
    }
    t[o] = acc;
  }
}

// (r, z) and (q, z) partials of workgroup b over rows [b n / m, (b+1) n / m),
// in the layout the PCG SpMV launch folds: pd[b][0..NT) and pd[b][NT..2NT).
template <int NT>
__global__ __launch_bounds__(256) void k_dots(int64_t n, int m, const double* __restrict__ r,
                                              const double* __restrict__ z,
                                              const double* __restrict__ q,
                                              double* __restrict__ pd) {
  __shared__ double lds[4 * 2 * NT];
  const int b = blockIdx.x;
  const int64_t r0 = n * b / m, r1 = n * (b + 1) / m;
  double v[2 * NT];
#pragma unroll
  for (int t = 0; t < 2 * NT; ++t) v[t] = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x)
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      const size_t o = vix<NT>(n, i, k);
      const double zv = z[o];
      v[k] = fma(r[o], zv, v[k]);
      v[NT + k] = fma(q[o], zv, v[NT + k]);
    }
  block_sum<2 * NT>(v, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int t = 0; t < 2 * NT; ++t) pd[(size_t)b * 2 * NT + t] = v[t];
}

// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

#define AM_NR_SWITCH(nr, CALL)                       \
  switch (nr) {                                      \
    case 1: { constexpr int NR = 1; CALL; } break;   \
    case 2: { constexpr int NR = 2; CALL; } break;   \
    case 4: { constexpr int NR = 4; CALL; } break;   \
    case 8: { constexpr int NR = 8; CALL; } break;   \
    case 16: { constexpr int NR = 16; CALL; } break; \
    default: return hipErrorInvalidValue;            \
  }

static hipError_t gather(int64_t n, const int32_t* map, const double* a, const double* b,
                         double* dst, int nr, hipStream_t s) {
  AM_NR_SWITCH(nr, hipLaunchKernelGGL(k_gather<NR>, dim3(nblk(n)), dim3(256), 0, s, n, map, a, b, dst));
  return hipGetLastError();
}

static hipError_t sres(const DeviceState& D, const double* r, const double* zin, const double* win,
                       double* zout, double* t, int nr, hipStream_t s) {
  if (D.ell_w <= 8) {
    AM_NR_SWITCH(nr, hipLaunchKernelGGL((k_sres<NR, 8>), dim3(nblk(D.n)), dim3(256), 0, s, D.n,
                                        D.ell_w, D.ell_col, D.ell_val, r, zin, win, zout, t));
  } else {
    AM_NR_SWITCH(nr, hipLaunchKernelGGL((k_sres<NR, 32>), dim3(nblk(D.n)), dim3(256), 0, s, D.n,
                                        D.ell_w, D.ell_col, D.ell_val, r, zin, win, zout, t));
  }
  return hipGetLastError();
}

#define SM_TRY(expr)                    \
  do {                                  \
    hipError_t e_ = (expr);             \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

hipError_t launch_smoothed_apply(DeviceState& d, SmoothDevice& sm, const double* r_am,
                                 double* z_am, int nr, hipStream_t s) {
  DeviceState& D = *sm.bj;
  if (sm.steps < 1 || D.n != d.n || nr > D.max_nrhs || nr > d.max_nrhs)
    return hipErrorInvalidValue;
  const int64_t n = d.n;
  double* rb = D.r;   // r in the block-Jacobi order
  double* zc = D.z;   // current z
  double* zn = D.p[0];
  double* w = D.p[1];  // pending correction, folded into the next residual
  double* t = D.q;     // residual r - A z
  const double* pend = nullptr;
  SM_TRY(gather(n, sm.to_bj, r_am, nullptr, rb, nr, s));
  // pre-smoothing; the first step from z = 0 is z = B^{-1} r
  SM_TRY(launch_local_sweep(D, rb, zc, D.eta, nr, 0, s));
  for (int j = 1; j < sm.steps; ++j) {
    SM_TRY(sres(D, rb, zc, pend, zn, t, nr, s));
    std::swap(zc, zn);
    SM_TRY(launch_local_sweep(D, t, w, D.eta, nr, 0, s));
    pend = w;
  }
  // the AlgMortar correction of r - A z, in its own device order
  SM_TRY(sres(D, rb, zc, pend, zn, t, nr, s));
  std::swap(zc, zn);
  SM_TRY(gather(n, sm.to_am, t, nullptr, sm.t_am, nr, s));
  if (d.NL > 0) {
    SM_TRY(launch_bpart(d, sm.t_am, nr, s));
    if (!d.fuse_eta) SM_TRY(launch_iface_gemv(d, nr, 0, 0, s));
  }
  SM_TRY(launch_local_sweep(d, sm.t_am, sm.w_am, d.eta, nr, 1, s));
  SM_TRY(gather(n, sm.to_bj, sm.w_am, nullptr, w, nr, s));
  pend = w;
  // post-smoothing
  for (int j = 0; j < sm.steps; ++j) {
    SM_TRY(sres(D, rb, zc, pend, zn, t, nr, s));
    std::swap(zc, zn);
    SM_TRY(launch_local_sweep(D, t, w, D.eta, nr, 0, s));
    pend = w;
  }
  return gather(n, sm.to_am, zc, pend, z_am, nr, s);
}

hipError_t launch_smooth_dots(DeviceState& d, int nr, hipStream_t s) {
  if (d.m < 1) return hipErrorInvalidValue;
  AM_NR_SWITCH(nr, hipLaunchKernelGGL(k_dots<NR>, dim3((unsigned)d.m), dim3(256), 0, s, d.n, d.m,
                                      d.r, d.z, d.q, d.red.pd));
  return hipGetLastError();
}

}  // namespace am
