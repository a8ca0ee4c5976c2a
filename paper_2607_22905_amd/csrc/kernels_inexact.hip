// Inexact interface solve for gfx950 (the iterative option of Sec. 6, used
// with relative tolerance 1e-2 in Sec. 7): eta ~ S^{-1} b by PCG on S with a
// block-Jacobi preconditioner, stopped when ||b - S eta||_2 <= rtol ||b||_2
// (recursive residual) or after maxit iterations; zero initial guess,
// Fletcher-Reeves beta.  The blocks are contiguous ranges of the basis
// functions (in their lexicographic numbering), each solved exactly with its
// explicit inverse.  S is held sparse (ELL, column-major: a basis function
// couples to those sharing one of its subdomains).
//
// One workgroup per block.  The solve is 1 + 2 maxit launches, captured with
// the rest of a PCG iteration:
//   k_ix_init  r = b, eta = 0, z = B^{-1} r, partials (r, z), (r, r)
//   k_ix_a(k)  fold (r, z), (r, r) of the previous launch; stop test; beta;
//              p = z + beta p_old (own rows); q = S p, where the p of other
//              rows is formed from their z and p_old; partials (p, q)
//   k_ix_b(k)  fold (p, q); alpha; eta += alpha p, r -= alpha q; z = B^{-1} r;
//              partials (r, z), (r, r)
// Every workgroup folds the partials of all blocks in block order (the same
// sums everywhere); workgroup 0 stores the per-column state, by iteration
// parity where a later launch reads it while the next one writes it.  A
// column that has stopped stays stopped (its flag is carried forward), and a
// launch in which every column has stopped returns after the fold.  In PCG
// mode k_ix_init also takes the outer stop decision (its wave 0 of workgroup
// 0), and every launch returns at once once the outer solve has stopped.
#include <algorithm>

#include "am_common.h"
#include "iface_products.h"

namespace am {

// folds per-block partials part[b][c], c < NC, over nb blocks (block order,
// then the fixed tree of block_sum); every thread gets the totals
template <int NC>
__device__ __forceinline__ void ix_fold(const double* __restrict__ part, int nb, double (&tot)[NC],
                                        double* lds) {
#pragma unroll
  for (int c = 0; c < NC; ++c) tot[c] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
    for (int c = 0; c < NC; ++c) tot[c] += part[(size_t)b * NC + c];
  block_sum<NC>(tot, lds);
}

__device__ __forceinline__ bool ix_skip(int pcg, int init, const PcgShared* sh, int* flag) {
  if (threadIdx.x == 0) *flag = (pcg && !init && all_done(sh)) ? 1 : 0;
  __syncthreads();
  return *flag != 0;
}

// z = B_b^{-1} r over the rows of block b (r in LDS [bs][NR]); the wave w
// takes output rows 64 w ..; writes z and the partials (r, z), (r, r)
template <int NR>
__device__ __forceinline__ void ix_precond(const double* __restrict__ inv, int s, const double* rl,
                                           int64_t row0, double* __restrict__ z,
                                           double* __restrict__ pb_out, double* red) {
  const int w = threadIdx.x >> 6;
  nd_d4 acc[4];
  nd_wave_product<NR, false>(inv, s, 64 * w, s, 0, s, rl, 0, acc);
  double part[2 * NR];
#pragma unroll
  for (int c = 0; c < 2 * NR; ++c) part[c] = 0.0;
  nd_wave_each<NR>(acc, [&](int l, int k, double v) {
    const int r = 64 * w + l;
    if (r < s) {
      z[(size_t)(row0 + r) * NR + k] = v;
      const double rv = rl[r * NR + k];
#pragma unroll
      for (int c = 0; c < NR; ++c)
        if (c == k) {
          part[c] = fma(rv, v, part[c]);
          part[NR + c] = fma(rv, rv, part[NR + c]);
        }
    }
  });
  block_sum<2 * NR>(part, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < 2 * NR; ++c) pb_out[c] = part[c];
}

template <int NR>
__global__ __launch_bounds__(256) void k_ix_init(
    int NL, int bs, const int64_t* __restrict__ inv_off, const double* __restrict__ binv,
    const double* __restrict__ bpart, double* __restrict__ r, double* __restrict__ z,
    double* __restrict__ eta, double* __restrict__ pb, int pcg, int init,
    const double* __restrict__ opb, int npb, PcgScalars* sc, PcgShared* sh) {
  __shared__ double rl[256 * NR];
  __shared__ double red[4 * 2 * NR];
  __shared__ int skip;
  if (ix_skip(pcg, init, sh, &skip)) return;
  if (pcg && blockIdx.x == 0 && threadIdx.x < 64) stop_test<NR>(opb, npb, init, sc, sh);
  const int b = blockIdx.x;
  const int64_t row0 = (int64_t)b * bs;
  const int s = (int)min((int64_t)bs, (int64_t)NL - row0);
  for (int t = threadIdx.x; t < s * NR; t += blockDim.x) {
    const int j = t / NR, k = t % NR;
    const int64_t n = row0 + j;
    const double v = bpart[(size_t)(2 * n) * NR + k] + bpart[(size_t)(2 * n + 1) * NR + k];
    rl[t] = v;
    r[(size_t)n * NR + k] = v;
    eta[(size_t)n * NR + k] = 0.0;
  }
  __syncthreads();
  ix_precond<NR>(binv + inv_off[b], s, rl, row0, z, pb + (size_t)b * 2 * NR, red);
}

template <int NR>
__global__ __launch_bounds__(256) void k_ix_a(
    int k_it, int NL, int bs, int nb, int w, const int32_t* __restrict__ scol,
    const double* __restrict__ sval, const double* __restrict__ z, const double* __restrict__ pold,
    double* __restrict__ pnew, double* __restrict__ q, const double* __restrict__ pb_prev,
    double* __restrict__ pa, IxScalars* ixs, double rtol2, int pcg, const PcgShared* sh) {
  __shared__ double red[4 * 2 * NR];
  __shared__ int skip;
  if (ix_skip(pcg, 0, sh, &skip)) return;
  const int par = k_it & 1;
  double tot[2 * NR];
  ix_fold<2 * NR>(pb_prev, nb, tot, red);
  double beta[NR];
  bool done[NR];
  bool any = false;
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    const double rz = tot[c], rr = tot[NR + c];
    const bool prev = k_it > 1 && ixs[c].done[1 - par] != 0;
    const double bb = k_it == 1 ? rr : ixs[c].bb;
    done[c] = prev || !(rr > rtol2 * bb) || !(rz > 0.0);
    beta[c] = (k_it == 1 || done[c]) ? 0.0 : rz / ixs[c].rzs[1 - par];
    any |= !done[c];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ixs[c].done[par] = done[c] ? 1 : 0;
      ixs[c].rzs[par] = rz;
      if (k_it == 1) ixs[c].bb = rr;
      if (done[c] && !prev) ixs[c].iters = k_it - 1;
      if (!done[c]) ixs[c].iters = k_it;
    }
  }
  if (!any) return;
  const int64_t row0 = (int64_t)blockIdx.x * bs;
  const int s = (int)min((int64_t)bs, (int64_t)NL - row0);
  double pq[NR];
#pragma unroll
  for (int c = 0; c < NR; ++c) pq[c] = 0.0;
  for (int t = threadIdx.x; t < s; t += blockDim.x) {
    const int64_t j = row0 + t;
    // p_new = z + beta p_old, at any row (p_old is not read on the first
    // iteration, where it holds no values)
    auto pn = [&](int64_t row, int c) {
      return k_it == 1 ? z[row * NR + c] : fma(beta[c], pold[row * NR + c], z[row * NR + c]);
    };
    double acc[NR], pj[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      acc[c] = 0.0;
      pj[c] = pn(j, c);
    }
    for (int e = 0; e < w; ++e) {
      const int64_t col = scol[(size_t)e * NL + j];
      const double a = sval[(size_t)e * NL + j];
#pragma unroll
      for (int c = 0; c < NR; ++c) acc[c] = fma(a, pn(col, c), acc[c]);
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      if (done[c]) continue;
      pnew[j * NR + c] = pj[c];
      q[j * NR + c] = acc[c];
      pq[c] = fma(pj[c], acc[c], pq[c]);
    }
  }
  block_sum<NR>(pq, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < NR; ++c) pa[(size_t)blockIdx.x * NR + c] = pq[c];
}

template <int NR>
__global__ __launch_bounds__(256) void k_ix_b(
    int k_it, int NL, int bs, int nb, const int64_t* __restrict__ inv_off,
    const double* __restrict__ binv, const double* __restrict__ p, const double* __restrict__ q,
    double* __restrict__ r, double* __restrict__ z, double* __restrict__ eta,
    const double* __restrict__ pa, double* __restrict__ pb_out, const IxScalars* ixs, int pcg,
    const PcgShared* sh) {
  __shared__ double rl[256 * NR];
  __shared__ double red[4 * 2 * NR];
  __shared__ int skip;
  if (ix_skip(pcg, 0, sh, &skip)) return;
  const int par = k_it & 1;
  double pq[NR];
  ix_fold<NR>(pa, nb, pq, red);
  double alpha[NR];
  bool done[NR];
  bool any = false;
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    done[c] = ixs[c].done[par] != 0 || !(pq[c] > 0.0);
    alpha[c] = done[c] ? 0.0 : ixs[c].rzs[par] / pq[c];
    any |= !done[c];
  }
  if (!any) return;
  const int b = blockIdx.x;
  const int64_t row0 = (int64_t)b * bs;
  const int s = (int)min((int64_t)bs, (int64_t)NL - row0);
  for (int t = threadIdx.x; t < s * NR; t += blockDim.x) {
    const int j = t / NR, c = t % NR;
    const int64_t n = row0 + j;
    double rv = r[(size_t)n * NR + c];
    if (!done[c]) {
      eta[(size_t)n * NR + c] = fma(alpha[c], p[(size_t)n * NR + c], eta[(size_t)n * NR + c]);
      rv = fma(-alpha[c], q[(size_t)n * NR + c], rv);
      r[(size_t)n * NR + c] = rv;
    }
    rl[t] = rv;
  }
  __syncthreads();
  ix_precond<NR>(binv + inv_off[b], s, rl, row0, z, pb_out + (size_t)b * 2 * NR, red);
}

template <int NR>
static void ix_solve_t(DeviceState& d, hipStream_t st, int pcg, int init) {
  IxDevice& ix = d.ix;
  const int nb = ix.nblk, NL = (int)d.NL;
  am_launch(d, true, ix.maxit == 0, k_ix_init<NR>, dim3(nb), dim3(256), st, NL, ix.bs, ix.inv_off,
            ix.binv, d.bpart, ix.r, ix.z, d.eta, ix.pb[0], pcg, init, d.red.pb, d.m, d.sc,
            d.shared);
  for (int k = 1; k <= ix.maxit; ++k) {
    am_launch(d, false, false, k_ix_a<NR>, dim3(nb), dim3(256), st, k, NL, ix.bs, nb, ix.w,
              ix.scol, ix.sval, ix.z, ix.p[(k - 1) & 1], ix.p[k & 1], ix.q, ix.pb[(k - 1) & 1],
              ix.pa, ix.sc, ix.rtol * ix.rtol, pcg, d.shared);
    am_launch(d, false, k == ix.maxit, k_ix_b<NR>, dim3(nb), dim3(256), st, k, NL, ix.bs, nb,
              ix.inv_off, ix.binv, ix.p[k & 1], ix.q, ix.r, ix.z, d.eta, ix.pa, ix.pb[k & 1],
              ix.sc, pcg, d.shared);
  }
}

hipError_t launch_ix_solve(DeviceState& d, int nr, int pcg, int init, hipStream_t st) {
  if (nr > d.max_nrhs) return hipErrorInvalidValue;
  switch (nr) {
    case 1: ix_solve_t<1>(d, st, pcg, init); break;
    case 2: ix_solve_t<2>(d, st, pcg, init); break;
    case 4: ix_solve_t<4>(d, st, pcg, init); break;
    case 8: ix_solve_t<8>(d, st, pcg, init); break;
    case 16: ix_solve_t<16>(d, st, pcg, init); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---- set-up ----------------------------------------------------------------

// Sbd = the block-diagonal part of S (blocks of bs rows; identity padding)
__global__ __launch_bounds__(256) void k_ix_blockdiag(const double* __restrict__ S, int ldS, int NL,
                                                      int bs, double* __restrict__ Sbd) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)ldS * ldS) return;
  const int a = (int)(t / ldS), c = (int)(t % ldS);
  double v = 0.0;
  if (a >= NL || c >= NL)
    v = a == c ? 1.0 : 0.0;
  else if (a / bs == c / bs)
    v = S[t];
  Sbd[t] = v;
}

// block b's inverse as a full square from the diagonal block of X
__global__ __launch_bounds__(256) void k_ix_extract(const double* __restrict__ X, int ldS, int NL,
                                                    int bs, const int64_t* __restrict__ inv_off,
                                                    double* __restrict__ binv) {
  const int b = blockIdx.y;
  const int64_t a0 = (int64_t)b * bs, s = std::min<int64_t>(bs, NL - a0);
  double* out = binv + inv_off[b];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < s * s;
       t += (int64_t)gridDim.x * blockDim.x)
    out[t] = X[(size_t)(a0 + t / s) * ldS + a0 + t % s];
}

// ELL values of S: sval[e][j] = S[j][scol[e][j]] (padding entries: column j, 0)
__global__ __launch_bounds__(256) void k_ix_ell(const double* __restrict__ S, int ldS, int NL,
                                                int w, const int32_t* __restrict__ scol,
                                                const int8_t* __restrict__ pad,
                                                double* __restrict__ sval) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)w * NL) return;
  const int64_t j = t % NL;
  sval[t] = pad[t] ? 0.0 : S[(size_t)j * ldS + scol[t]];
}

// block inverses and the ELL values from the handle's S (original order).
// Sbd, L, Li: ldS x ldS scratch; part: trtri_part_tiles(ldS / 64) tiles.
hipError_t ix_numeric(DeviceState& d, double* Sbd, double* L, double* Li, double* part,
                      hipStream_t st) {
  IxDevice& ix = d.ix;
  const int64_t tot = (int64_t)d.ldS * d.ldS;
  hipLaunchKernelGGL(k_ix_blockdiag, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, d.S,
                     d.ldS, (int)d.NL, ix.bs, Sbd);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double* S0 = d.S;
  d.S = Sbd;
  e = dense_cholesky_inverse(d, L, Li, part, st);  // d.Sinv = Sbd^{-1}
  d.S = S0;
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ix_extract, dim3(64, ix.nblk), dim3(256), 0, st, d.Sinv, d.ldS, (int)d.NL,
                     ix.bs, ix.inv_off, ix.binv);
  const int64_t ne = (int64_t)ix.w * d.NL;
  hipLaunchKernelGGL(k_ix_ell, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, d.S, d.ldS,
                     (int)d.NL, ix.w, ix.scol, ix.pad, ix.sval);
  return hipGetLastError();
}

}  // namespace am
