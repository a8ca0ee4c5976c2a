// TPFA kernels of the differentiation form (no paper analogue): assembly of
// A's values and of the Dirichlet part of f from log K on the device, and the
// per-cell gather of the adjoint sensitivity
//   dJ/dtheta_c = -sum_{faces f at c} dT_f/dtheta_c (lambda_k - lambda_l)(p_k - p_l)
//                 - sum_{Dirichlet faces of c} t_c lambda_c (p_c - pD),
// with T = t_k t_l / (t_k + t_l), t_c = exp(theta_c) g_c,
// dT/dtheta_k = T t_l / (t_k + t_l).  Both kernels are cell-centric gathers
// over a cell -> faces list, so results do not depend on scheduling.
#include "am_common.h"

namespace am {

__global__ __launch_bounds__(256) void k_tpfa_offdiag(int64_t nf, const int64_t* __restrict__ fk,
                                                      const int64_t* __restrict__ fl,
                                                      const double* __restrict__ gk,
                                                      const double* __restrict__ gl,
                                                      const double* __restrict__ logK,
                                                      const int64_t* __restrict__ skl,
                                                      const int64_t* __restrict__ slk,
                                                      double* __restrict__ val) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int64_t l = fl[f];
  if (l < 0) return;
  const double tk = exp(logK[fk[f]]) * gk[f];
  const double tl = exp(logK[l]) * gl[f];
  const double T = tk * tl / (tk + tl);
  val[skl[f]] = -T;
  val[slk[f]] = -T;
}

__global__ __launch_bounds__(256) void k_tpfa_diag(int64_t n, const int64_t* __restrict__ cf_ptr,
                                                   const int32_t* __restrict__ cf_face,
                                                   const int64_t* __restrict__ fk,
                                                   const int64_t* __restrict__ fl,
                                                   const double* __restrict__ gk,
                                                   const double* __restrict__ gl,
                                                   const double* __restrict__ pD,
                                                   const double* __restrict__ logK,
                                                   const int64_t* __restrict__ sdiag,
                                                   double* __restrict__ val,
                                                   double* __restrict__ rhs) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double d = 0.0, fsum = 0.0;
  for (int64_t p = cf_ptr[c]; p < cf_ptr[c + 1]; ++p) {
    const int64_t f = cf_face[p];
    const int64_t l = fl[f];
    const double tk = exp(logK[fk[f]]) * gk[f];
    if (l >= 0) {
      const double tl = exp(logK[l]) * gl[f];
      d += tk * tl / (tk + tl);
    } else {
      d += tk;
      fsum += tk * pD[f];
    }
  }
  val[sdiag[c]] = d;
  if (rhs) rhs[c] = fsum;
}

__global__ __launch_bounds__(256) void k_face_grad(int64_t n, const int64_t* __restrict__ cf_ptr,
                                                   const int32_t* __restrict__ cf_face,
                                                   const int64_t* __restrict__ fk,
                                                   const int64_t* __restrict__ fl,
                                                   const double* __restrict__ gk,
                                                   const double* __restrict__ gl,
                                                   const double* __restrict__ pD,
                                                   const double* __restrict__ logK,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ lam,
                                                   double* __restrict__ grad) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double g = 0.0;
  for (int64_t q = cf_ptr[c]; q < cf_ptr[c + 1]; ++q) {
    const int64_t f = cf_face[q];
    const int64_t k = fk[f], l = fl[f];
    const double tk = exp(logK[k]) * gk[f];
    if (l >= 0) {
      const double tl = exp(logK[l]) * gl[f];
      const double T = tk * tl / (tk + tl);
      const double dT = (c == k) ? T * tl / (tk + tl) : T * tk / (tk + tl);
      g -= dT * (lam[k] - lam[l]) * (p[k] - p[l]);
    } else {
      g -= tk * lam[k] * (p[k] - pD[f]);
    }
  }
  grad[c] = g;
}

hipError_t launch_tpfa_assemble(TpfaDevice& t, const double* logK, double* val, double* f,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_tpfa_offdiag, dim3((unsigned)((t.nf + 255) / 256)), dim3(256), 0, s, t.nf,
                     t.fk, t.fl, t.gk, t.gl, logK, t.slot_kl, t.slot_lk, val);
  hipLaunchKernelGGL(k_tpfa_diag, dim3((unsigned)((t.n + 255) / 256)), dim3(256), 0, s, t.n,
                     t.cf_ptr, t.cf_face, t.fk, t.fl, t.gk, t.gl, t.pD, logK, t.slot_kk, val, f);
  return hipGetLastError();
}

hipError_t launch_face_grad(TpfaDevice& t, const double* logK, const double* p,
                            const double* lam, double* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_face_grad, dim3((unsigned)((t.n + 255) / 256)), dim3(256), 0, s, t.n,
                     t.cf_ptr, t.cf_face, t.fk, t.fl, t.gk, t.gl, t.pD, logK, p, lam, grad);
  return hipGetLastError();
}

}  // namespace am
