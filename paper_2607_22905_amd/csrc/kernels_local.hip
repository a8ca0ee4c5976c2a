// Subdomain kernels for gfx950: the local operators A_i = A_ii - sum_j D_ij
// (eq. Dij-def, eq. A_i) factored as banded Cholesky A_i = L_i L_i^T
// (Algorithm 1), the local solves A_i pbar_i = r_i (eq. def-pbar-local,
// Algorithm 2), the multiscale basis functions A_i phat = -B_i psi
// (eq. def-phat-local) and the reconstruction z = pbar + sum eta_m phat^(m)
// (eq. p-decomposition-alg).
//
// Layout.  Inside subdomain s the rows are in the device order (a bandwidth-
// reducing order, see plan_local), padded to NP = 64*ceil(N/64) rows.  With a
// window width WP = 64*C >= bandwidth, the factor is stored twice:
//   Lc[j][slot] = L[row, j]  for the row in [j+1, j+WP] with row % WP == slot
//   Lr[j][slot] = L[j, col]  for the col in [j-WP, j-1] with col % WP == slot
// so that both the forward sweep (column j) and the backward sweep (row j)
// read one contiguous WP-vector per step: lane t of the wave owns slots
// t, t+64, ... and each step is one coalesced load, a broadcast of the pivot
// (readlane) and one FMA per slot.  invd[j] = 1/L_jj.  Padding rows have a
// zero factor and invd = 1.
#include "am_common.h"

namespace am {

template <typename FT> struct AccT { using T = float; };
template <> struct AccT<double> { using T = double; };

// prefetch distance (steps) of the rolling register ring; the sweeps run in
// fully unrolled chunks of RING steps (RING divides 64)
#ifndef ALGMORTAR_RING1
#define ALGMORTAR_RING1 32
#endif
template <int C, int NR> struct Ring {
  static constexpr int v = (C * NR <= 1) ? ALGMORTAR_RING1 : (C * NR <= 2) ? 32 : (C * NR <= 8) ? 16 : 8;
};

// ---------------------------------------------------------------------------
// Banded Cholesky of A_i in a (WP+1)^2 LDS window (right-looking).
template <typename FT, int WP>
__global__ __launch_bounds__(256) void k_band_factor(
    const int32_t* __restrict__ subs, const int64_t* __restrict__ sub_ptr,
    const int64_t* __restrict__ roff, const int64_t* __restrict__ fac_off,
    const int64_t* __restrict__ prp, const int32_t* __restrict__ pci,
    const double* __restrict__ pv, FT* __restrict__ Lc, FT* __restrict__ Lr,
    typename AccT<FT>::T* __restrict__ invd, int32_t* __restrict__ fail) {
  using IT = typename AccT<FT>::T;
  constexpr int WN = WP + 1;
  __shared__ double B[WN * WN];
  __shared__ double lcol[WN];
  const int s = subs[blockIdx.x];
  const int64_t base = sub_ptr[s];
  const int N = (int)(sub_ptr[s + 1] - base);
  const int64_t ro = roff[s];
  const int NP = (int)(roff[s + 1] - ro);
  FT* lc = Lc + fac_off[s];
  FT* lr = Lr + fac_off[s];
  IT* iv = invd + ro;
  const int tid = threadIdx.x;

  // row `row` of A_i: in-subdomain lower entries, minus the sum of the
  // couplings that leave the subdomain on the diagonal
  auto load_row = [&](int row) {
    const int64_t g = base + row;
    double dout = 0.0;
    double* Br = B + (row % WN) * WN;
    for (int64_t p = prp[g]; p < prp[g + 1]; ++p) {
      const int64_t c = pci[p];
      const double v = pv[p];
      if (c >= base && c < base + N) {
        const int lcn = (int)(c - base);
        if (lcn <= row && row - lcn <= WP) Br[lcn % WN] = v;
      } else {
        dout += v;
      }
    }
    Br[row % WN] -= dout;
  };

  for (int t = tid; t < WN * WN; t += blockDim.x) B[t] = 0.0;
  __syncthreads();
  for (int row = tid; row < min(WP + 1, N); row += blockDim.x) load_row(row);
  __syncthreads();

  for (int j = 0; j < N; ++j) {
    const int sj = j % WN;
    const double d = B[sj * WN + sj];
    const bool bad = !(d > 0.0) || !(d < 1.0e300);
    const double inv = bad ? 1.0 : 1.0 / sqrt(d);
    if (tid == 0) {
      if (bad && atomicCAS(fail, -1, s) == -1) fail[1] = j;
      iv[j] = (IT)inv;
    }
    for (int t = tid; t < WP; t += blockDim.x) {
      const int row = j + 1 + t;
      double l = 0.0;
      if (row < N) l = B[(row % WN) * WN + sj] * inv;
      lcol[row % WN] = l;
      st_fac(lc + (size_t)j * WP + (row % WP), l);
      if (row < N) st_fac(lr + (size_t)row * WP + (j % WP), l);
    }
    __syncthreads();
    const int nu = j + WP + 1;
    for (int t = tid; t < WP * WP; t += blockDim.x) {
      const int a = t / WP, b = t % WP;
      if (b <= a) {
        const int rho = j + 1 + a, kap = j + 1 + b;
        if (rho < N) B[(rho % WN) * WN + (kap % WN)] -= lcol[rho % WN] * lcol[kap % WN];
      }
    }
    if (nu < N)
      for (int t = tid; t < WN; t += blockDim.x) B[(nu % WN) * WN + t] = 0.0;
    __syncthreads();
    if (nu < N && tid == 0) load_row(nu);
    __syncthreads();
  }
  for (int j = N + tid; j < NP; j += blockDim.x) iv[j] = (IT)1.0;
}

// ---------------------------------------------------------------------------
// Forward sweep L y = r.  Window before step j: rows j..j+WP-1; the pivot of
// step j sits in slot j % WP, whose lane then takes row j+WP.
template <typename FT, int C, int NR>
__device__ __forceinline__ void fwd_sweep(const int N, const int NP, const FT* __restrict__ lc,
                                          const typename AccT<FT>::T* __restrict__ iv,
                                          const double* rin, double* yout) {
  using AT = typename AccT<FT>::T;
  constexpr int WP = 64 * C;
  constexpr int RING = Ring<C, NR>::v;
  const int lane = threadIdx.x & 63;
  AT acc[C][NR];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int row = 64 * c + lane;
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[c][k] = row < N ? (AT)rin[(size_t)row * NR + k] : (AT)0;
  }
  AT buf[RING][C];
#pragma unroll
  for (int t = 0; t < RING; ++t)
#pragma unroll
    for (int c = 0; c < C; ++c)
      buf[t][c] = ld_fac(lc + (size_t)min(t, NP - 1) * WP + 64 * c + lane);

  for (int b = 0; b < NP / 64; ++b) {
    const int j0 = 64 * b;
    const int cb = b % C;
    AT rn[NR];
    const int nrow = j0 + WP + lane;
#pragma unroll
    for (int k = 0; k < NR; ++k) rn[k] = nrow < N ? (AT)rin[(size_t)nrow * NR + k] : (AT)0;
    const AT ivl = iv[j0 + lane];
    AT yl[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) yl[k] = (AT)0;
#pragma unroll 1
    for (int ch = 0; ch < 64; ch += RING) {
#pragma unroll
      for (int tt = 0; tt < RING; ++tt) {
        const int t = ch + tt;
        const int j = j0 + t;
        AT l[C];
#pragma unroll
        for (int c = 0; c < C; ++c) l[c] = buf[tt][c];
        const int jn = min(j + RING, NP - 1);
#pragma unroll
        for (int c = 0; c < C; ++c) buf[tt][c] = ld_fac(lc + (size_t)jn * WP + 64 * c + lane);
        const AT inv = readlane(ivl, t);
        AT y[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          AT piv = acc[0][k];
#pragma unroll
          for (int c = 1; c < C; ++c) piv = (cb == c) ? acc[c][k] : piv;
          y[k] = readlane(piv, t) * inv;
        }
        const bool own = (lane == t);
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const bool take = own && (c == cb);
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            const AT a = take ? rn[k] : acc[c][k];
            acc[c][k] = fma(-l[c], y[k], a);
          }
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) yl[k] = own ? y[k] : yl[k];
      }
    }
    const int row = j0 + lane;
    if (row < N)
#pragma unroll
      for (int k = 0; k < NR; ++k) yout[(size_t)row * NR + k] = (double)yl[k];
  }
}

// Backward sweep L^T x = y (y read from and x written to yx).  Window before
// step j (descending): rows j-WP+1..j; slot j % WP then takes row j-WP.
// After each block of 64 steps, lane t holds x of row j0+t and calls
// epi(row, x[NR]).
template <typename FT, int C, int NR, class Epi>
__device__ __forceinline__ void bwd_sweep(const int N, const int NP, const FT* __restrict__ lr,
                                          const typename AccT<FT>::T* __restrict__ iv,
                                          const double* yx, Epi& epi) {
  using AT = typename AccT<FT>::T;
  constexpr int WP = 64 * C;
  constexpr int RING = Ring<C, NR>::v;
  const int lane = threadIdx.x & 63;
  AT acc[C][NR];
  const int wbase = NP - WP;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int slot = 64 * c + lane;
    const int row = wbase + ((((slot - wbase) % WP) + WP) % WP);
#pragma unroll
    for (int k = 0; k < NR; ++k)
      acc[c][k] = (row >= 0 && row < N) ? (AT)yx[(size_t)row * NR + k] : (AT)0;
  }
  // ring slot u holds the column consumed u steps (mod RING) after the start
  AT buf[RING][C];
#pragma unroll
  for (int u = 0; u < RING; ++u)
#pragma unroll
    for (int c = 0; c < C; ++c)
      buf[u][c] = ld_fac(lr + (size_t)max(NP - 1 - u, 0) * WP + 64 * c + lane);

  for (int b = NP / 64 - 1; b >= 0; --b) {
    const int j0 = 64 * b;
    const int cb = b % C;
    AT rn[NR];
    const int nrow = j0 + lane - WP;
#pragma unroll
    for (int k = 0; k < NR; ++k) rn[k] = nrow >= 0 ? (AT)yx[(size_t)nrow * NR + k] : (AT)0;
    const AT ivl = iv[j0 + lane];
    AT xl[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) xl[k] = (AT)0;
#pragma unroll 1
    for (int ch = 64 - RING; ch >= 0; ch -= RING) {
#pragma unroll
      for (int tt = RING - 1; tt >= 0; --tt) {
        const int t = ch + tt;
        const int j = j0 + t;
        constexpr int dummy = 0;
        (void)dummy;
        const int su = RING - 1 - tt;
        AT l[C];
#pragma unroll
        for (int c = 0; c < C; ++c) l[c] = buf[su][c];
        const int jn = max(j - RING, 0);
#pragma unroll
        for (int c = 0; c < C; ++c) buf[su][c] = ld_fac(lr + (size_t)jn * WP + 64 * c + lane);
        const AT inv = readlane(ivl, t);
        AT x[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          AT piv = acc[0][k];
#pragma unroll
          for (int c = 1; c < C; ++c) piv = (cb == c) ? acc[c][k] : piv;
          x[k] = readlane(piv, t) * inv;
        }
        const bool own = (lane == t);
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const bool take = own && (c == cb);
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            const AT a = take ? rn[k] : acc[c][k];
            acc[c][k] = fma(-l[c], x[k], a);
          }
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) xl[k] = own ? x[k] : xl[k];
      }
    }
    double xd[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) xd[k] = (double)xl[k];
    epi(j0 + lane, xd);
  }
}

// ---------------------------------------------------------------------------
// Local solve / apply kernel, one wave per subdomain.
//   mode 0: out = A_i^{-1} r                          (local particular solution)
//   mode 1: out = A_i^{-1} r + sum_q eta_q phat^(q)    (preconditioner apply)
//   mode 2: mode 1 plus (r, z) and (q, z) for PCG; the last block updates beta
constexpr int kMaxNiLds = 128;

template <typename FT, int C, int NR>
__global__ __launch_bounds__(64) void k_local(
    const int32_t* __restrict__ subs, const int64_t* __restrict__ sub_ptr,
    const int64_t* __restrict__ roff, const int64_t* __restrict__ fac_off,
    const FT* __restrict__ Lc, const FT* __restrict__ Lr,
    const typename AccT<FT>::T* __restrict__ invd, const double* rin, double* out, int mode,
    const int64_t* __restrict__ isub_ptr, const int32_t* __restrict__ isub_list,
    const int64_t* __restrict__ mbf_off, const double* __restrict__ mbf,
    const double* __restrict__ eta, const double* __restrict__ qv, double* partial,
    unsigned* counter, unsigned blk_off, unsigned nblk_total, PcgScalars* sc, PcgShared* sh,
    int init) {
  if (mode == 2 && all_done(sh)) return;
  __shared__ double eta_s[kMaxNiLds * NR];
  __shared__ double red[2 * NR];
  const int s = subs[blockIdx.x];
  const int64_t base = sub_ptr[s];
  const int N = (int)(sub_ptr[s + 1] - base);
  const int64_t ro = roff[s];
  const int NP = (int)(roff[s + 1] - ro);
  const FT* lc = Lc + fac_off[s];
  const FT* lr = Lr + fac_off[s];
  const auto* iv = invd + ro;
  const int lane = threadIdx.x;
  const int64_t i0 = isub_ptr[s];
  const int ns = (int)(isub_ptr[s + 1] - i0);
  const double* P = mbf + mbf_off[s];
  if (mode >= 1)
    for (int t = lane; t < ns * NR; t += 64)
      eta_s[t] = eta[(size_t)isub_list[i0 + t / NR] * NR + (t % NR)];

  fwd_sweep<FT, C, NR>(N, NP, lc, iv, rin + base * NR, out + base * NR);
  __syncthreads();

  double rz[NR], qz[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) rz[k] = qz[k] = 0.0;
  double* o = out + base * NR;
  const double* rr = rin + base * NR;
  const double* qq = qv ? qv + base * NR : nullptr;
  auto epi = [&](int row, double (&x)[NR]) {
    if (row >= N) return;
    if (mode >= 1)
      for (int q = 0; q < ns; ++q) {
        const double ph = P[(size_t)q * N + row];
#pragma unroll
        for (int k = 0; k < NR; ++k) x[k] = fma(ph, eta_s[q * NR + k], x[k]);
      }
#pragma unroll
    for (int k = 0; k < NR; ++k) o[(size_t)row * NR + k] = x[k];
    if (mode == 2) {
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        rz[k] = fma(rr[(size_t)row * NR + k], x[k], rz[k]);
        qz[k] = fma(qq[(size_t)row * NR + k], x[k], qz[k]);
      }
    }
  };
  bwd_sweep<FT, C, NR>(N, NP, lr, iv, out + base * NR, epi);

  if (mode != 2) return;
  double v[2 * NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    v[k] = wave_sum(rz[k]);
    v[NR + k] = wave_sum(qz[k]);
  }
  __shared__ int last;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 2 * NR; ++k) partial[(size_t)(blk_off + blockIdx.x) * 2 * NR + k] = v[k];
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    last = (prev == nblk_total - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double tot[2 * NR];
#pragma unroll
  for (int k = 0; k < 2 * NR; ++k) tot[k] = 0.0;
  for (unsigned b = lane; b < nblk_total; b += 64)
#pragma unroll
    for (int k = 0; k < 2 * NR; ++k) tot[k] += partial[(size_t)b * 2 * NR + k];
#pragma unroll
  for (int k = 0; k < 2 * NR; ++k) tot[k] = wave_sum(tot[k]);
  if (lane == 0) {
    int alld = 1;
    for (int k = 0; k < sh->nrhs; ++k) {
      PcgScalars& S = sc[k];
      if (!S.done) {
        const double rzn = tot[k];
        if (!(rzn > 0.0)) {
          S.status = AM_ERR_BREAKDOWN;
          S.done = 1;
        } else {
          if (init)
            S.beta = 0.0;
          else if (sh->flexible)
            S.beta = -S.alpha * tot[NR + k] / S.rz;
          else
            S.beta = rzn / S.rz;
          S.rz = rzn;
        }
      }
      alld &= S.done;
    }
    sh->all_done = alld;
    *counter = 0u;
    __threadfence();
  }
  (void)red;
}

// MBFs: one wave per (subdomain, slot): rhs = -B_s psi_n scattered from the
// boundary weights, then the two sweeps in place.
template <typename FT, int C>
__global__ __launch_bounds__(64) void k_mbf(
    const int32_t* __restrict__ pairs, const int32_t* __restrict__ pair_sub,
    const int32_t* __restrict__ pair_q, const int64_t* __restrict__ sub_ptr,
    const int64_t* __restrict__ roff, const int64_t* __restrict__ fac_off,
    const FT* __restrict__ Lc, const FT* __restrict__ Lr,
    const typename AccT<FT>::T* __restrict__ invd, const int64_t* __restrict__ mbf_off,
    double* mbf, const int64_t* __restrict__ bw_ptr, const int32_t* __restrict__ bw_row,
    const double* __restrict__ bw_val) {
  const int pi = pairs[blockIdx.x];
  const int s = pair_sub[pi], q = pair_q[pi];
  const int64_t base = sub_ptr[s];
  const int N = (int)(sub_ptr[s + 1] - base);
  const int64_t ro = roff[s];
  const int NP = (int)(roff[s + 1] - ro);
  double* col = mbf + mbf_off[s] + (size_t)q * N;
  const int lane = threadIdx.x;
  for (int row = lane; row < N; row += 64) col[row] = 0.0;
  __syncthreads();
  for (int64_t e = bw_ptr[pi] + lane; e < bw_ptr[pi + 1]; e += 64) col[bw_row[e]] = bw_val[e];
  __syncthreads();
  fwd_sweep<FT, C, 1>(N, NP, Lc + fac_off[s], invd + ro, col, col);
  __syncthreads();
  auto epi = [&](int row, double (&x)[1]) {
    if (row < N) col[row] = x[0];
  };
  bwd_sweep<FT, C, 1>(N, NP, Lr + fac_off[s], invd + ro, col, epi);
}

template <int NR>
__global__ __launch_bounds__(256) void k_bpart(const int64_t* __restrict__ sub_ptr,
                                               const int64_t* __restrict__ isub_ptr,
                                               const int64_t* __restrict__ mbf_off,
                                               const double* __restrict__ mbf,
                                               const double* __restrict__ r, double* bpart) {
  __shared__ double lds[4 * NR];
  bpart_sub<NR>(blockIdx.x, sub_ptr, isub_ptr, mbf_off, mbf, r, bpart, lds);
}


// ---------------------------------------------------------------------------
// launchers

template <typename FT>
static hipError_t band_factor_t(DeviceState& d, hipStream_t st) {
  using IT = typename AccT<FT>::T;
  for (int bk = 0; bk < 2; ++bk) {
    const int nb = (int)d.bucket_sub[bk].size();
    if (!nb) continue;
    if (bk == 0)
      hipLaunchKernelGGL((k_band_factor<FT, 64>), dim3(nb), dim3(256), 0, st,
                         d.d_bucket_sub[bk], d.sub_ptr, d.roff, d.fac_off, d.prp, d.pci, d.pv,
                         (FT*)d.Lc, (FT*)d.Lr, (IT*)d.invd, d.fail);
    else
      hipLaunchKernelGGL((k_band_factor<FT, 128>), dim3(nb), dim3(256), 0, st,
                         d.d_bucket_sub[bk], d.sub_ptr, d.roff, d.fac_off, d.prp, d.pci, d.pv,
                         (FT*)d.Lc, (FT*)d.Lr, (IT*)d.invd, d.fail);
  }
  return hipGetLastError();
}

hipError_t launch_band_factor(DeviceState& d, hipStream_t st) {
  switch (d.prec) {
    case AM_FP64: return band_factor_t<double>(d, st);
    case AM_FP32: return band_factor_t<float>(d, st);
    default: return band_factor_t<bf16_t>(d, st);
  }
}

template <typename FT>
static hipError_t mbf_t(DeviceState& d, hipStream_t st) {
  using IT = typename AccT<FT>::T;
  for (int bk = 0; bk < 2; ++bk) {
    const int nb = (int)d.bucket_pair[bk].size();
    if (!nb) continue;
    if (bk == 0)
      hipLaunchKernelGGL((k_mbf<FT, 1>), dim3(nb), dim3(64), 0, st, d.d_bucket_pair[bk],
                         d.mbf_pair_sub, d.mbf_pair_q, d.sub_ptr, d.roff, d.fac_off,
                         (const FT*)d.Lc, (const FT*)d.Lr, (const IT*)d.invd, d.mbf_off, d.mbf,
                         d.bw_ptr, d.bw_row, d.bw_val);
    else
      hipLaunchKernelGGL((k_mbf<FT, 2>), dim3(nb), dim3(64), 0, st, d.d_bucket_pair[bk],
                         d.mbf_pair_sub, d.mbf_pair_q, d.sub_ptr, d.roff, d.fac_off,
                         (const FT*)d.Lc, (const FT*)d.Lr, (const IT*)d.invd, d.mbf_off, d.mbf,
                         d.bw_ptr, d.bw_row, d.bw_val);
  }
  return hipGetLastError();
}

hipError_t launch_mbf(DeviceState& d, hipStream_t st) {
  switch (d.prec) {
    case AM_FP64: return mbf_t<double>(d, st);
    case AM_FP32: return mbf_t<float>(d, st);
    default: return mbf_t<bf16_t>(d, st);
  }
}

template <typename FT, int NR>
static hipError_t local_t(DeviceState& d, const double* r, double* z, const double* eta,
                          int mode, int init, hipStream_t st) {
  using IT = typename AccT<FT>::T;
  const unsigned total = (unsigned)(d.bucket_sub[0].size() + d.bucket_sub[1].size());
  unsigned off = 0;
  for (int bk = 0; bk < 2; ++bk) {
    const int nb = (int)d.bucket_sub[bk].size();
    if (!nb) continue;
    auto args = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(nb), dim3(64), 0, st, d.d_bucket_sub[bk], d.sub_ptr, d.roff,
                         d.fac_off, (const FT*)d.Lc, (const FT*)d.Lr, (const IT*)d.invd, r, z,
                         mode, d.isub_ptr, d.isub_list, d.mbf_off, d.mbf, eta, d.q,
                         d.red.partial, d.red.counter + 2, off, total, d.sc, d.shared, init);
    };
    if (bk == 0)
      args(k_local<FT, 1, NR>);
    else
      args(k_local<FT, 2, NR>);
    off += nb;
  }
  return hipGetLastError();
}

template <typename FT>
static hipError_t local_nr(DeviceState& d, const double* r, double* z, const double* eta,
                           int nrhs, int mode, int init, hipStream_t st) {
  switch (nrhs) {
    case 1: return local_t<FT, 1>(d, r, z, eta, mode, init, st);
    case 2: return local_t<FT, 2>(d, r, z, eta, mode, init, st);
    case 4: return local_t<FT, 4>(d, r, z, eta, mode, init, st);
    case 8: return local_t<FT, 8>(d, r, z, eta, mode, init, st);
    case 16: return local_t<FT, 16>(d, r, z, eta, mode, init, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_local_sweep(DeviceState& d, const double* r, double* z, const double* eta,
                              int nrhs, int mode, hipStream_t st) {
  // mode >= 10 encodes the PCG init pass (mode 2 with init = 1)
  const int init = mode >= 10 ? 1 : 0;
  const int m = mode % 10;
  switch (d.prec) {
    case AM_FP64: return local_nr<double>(d, r, z, eta, nrhs, m, init, st);
    case AM_FP32: return local_nr<float>(d, r, z, eta, nrhs, m, init, st);
    default: return local_nr<bf16_t>(d, r, z, eta, nrhs, m, init, st);
  }
}

hipError_t launch_bpart(DeviceState& d, const double* r, int nrhs, hipStream_t st) {
  const dim3 g(d.m), b(256);
  switch (nrhs) {
    case 1: hipLaunchKernelGGL(k_bpart<1>, g, b, 0, st, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, r, d.bpart); break;
    case 2: hipLaunchKernelGGL(k_bpart<2>, g, b, 0, st, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, r, d.bpart); break;
    case 4: hipLaunchKernelGGL(k_bpart<4>, g, b, 0, st, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, r, d.bpart); break;
    case 8: hipLaunchKernelGGL(k_bpart<8>, g, b, 0, st, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, r, d.bpart); break;
    case 16: hipLaunchKernelGGL(k_bpart<16>, g, b, 0, st, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, r, d.bpart); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace am
