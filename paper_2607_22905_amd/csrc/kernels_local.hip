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
// (readlane), one FMA per slot and one writelane.  The factor is kept in unit-diagonal form
// A_i = Lt D Lt^T (Lt = L diag(1/L_jj), D = diag(L_jj^2)): the sweeps then
// need no division per step; dinv[j] = 1/L_jj^2 scales w = Lt^{-1} r once
// per row between the two sweeps.  Padding rows have a zero factor and
// dinv = 1.
#include "am_common.h"

namespace am {

template <typename FT> struct AccT { using T = float; };
template <> struct AccT<double> { using T = double; };

// prefetch distance (steps) of the rolling register ring (RING divides 64);
// each block of 64 steps is fully unrolled so that the only loop back-edge
// (where the compiler merges outstanding-load counts) is once per block
#ifndef ALGMORTAR_RING1
#define ALGMORTAR_RING1 32
#endif
// One drain of the vector-memory counter before a sweep's main loop, so that
// the loads issued before the loop never force a full drain inside it.
__device__ __forceinline__ void wait_all_loads() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt, lgkmcnt untouched
}
// A copy of v the compiler cannot see through, so that per-step compares
// against it are evaluated in the step (and not kept live as 64 masks).
__device__ __forceinline__ int opaque(int v) {
  int r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
  return r;
}
// Keep each step's refill load where it is written (issued right after the
// slot is consumed): the scheduler may not move instructions across.
__device__ __forceinline__ void step_fence() { __builtin_amdgcn_sched_barrier(0); }

template <int C, int NR> struct Ring {
  static constexpr int v = (C * NR <= 1) ? ALGMORTAR_RING1 : (C * NR <= 2) ? 32 : (C * NR <= 8) ? 16 : 4;
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
      iv[j] = (IT)(inv * inv);
    }
    for (int t = tid; t < WP; t += blockDim.x) {
      const int row = j + 1 + t;
      double l = 0.0;
      if (row < N) l = B[(row % WN) * WN + sj] * inv;  // L[row, j]
      lcol[row % WN] = l;
      const double lt = l * inv;                        // Lt[row, j] = L[row, j] / L[j, j]
      st_fac(lc + (size_t)j * WP + (row % WP), lt);
      if (row < N) st_fac(lr + (size_t)row * WP + (j % WP), lt);
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
// Forward sweep Lt w = r, then v = dinv * w written to yout.  Window before
// step j: rows j..j+WP-1, row i held by lane (i % WP) % 64 in accumulator
// (i % WP) / 64.  At step j the pivot w_j is broadcast from lane t = j % 64
// (readlane), the owner lane's slot switches to row j+WP (its accumulator is
// replaced by r[j+WP]), every lane applies acc -= Lt[row, j] * w_j (one FMA)
// and w_j is recorded in lane t (writelane).  The owner's test is a compare
// against a per-block lane index, so no per-step masks are kept live.
// Per-block values consumed at a block's start (the rows entering the window)
// are loaded one block ahead, so no wait on them drains the factor prefetch
// ring.
template <typename FT, int C, int NR>
__device__ __forceinline__ void fwd_sweep(const int N, const int NP, const FT* __restrict__ lc,
                                          const typename AccT<FT>::T* __restrict__ dv,
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
  typename RawT<FT>::T buf[RING][C];
#pragma unroll
  for (int t = 0; t < RING; ++t) {
    const FT* colp = lc + (size_t)min(t, NP - 1) * WP;
#pragma unroll
    for (int c = 0; c < C; ++c) buf[t][c] = ld_raw(colp + 64 * c + lane);
  }
  AT rn[NR];
  {
    const int nrow = WP + lane;
#pragma unroll
    for (int k = 0; k < NR; ++k) rn[k] = nrow < N ? (AT)rin[(size_t)nrow * NR + k] : (AT)0;
  }
  wait_all_loads();

  for (int b = 0; b < NP / 64; ++b) {
    const int j0 = 64 * b;
    const int cb = b % C;
    AT rnx[NR];
    const int nrow = j0 + 64 + WP + lane;
#pragma unroll
    for (int k = 0; k < NR; ++k) rnx[k] = nrow < N ? (AT)rin[(size_t)nrow * NR + k] : (AT)0;
    const AT dvl = dv[j0 + lane];
    const int lane_j = opaque(j0 + lane);
    AT yl[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) yl[k] = (AT)0;
#pragma unroll
    for (int ch = 0; ch < 64; ch += RING) {
#pragma unroll
      for (int tt = 0; tt < RING; ++tt) {
        const int t = ch + tt;
        const int j = j0 + t;
        AT l[C];
#pragma unroll
        for (int c = 0; c < C; ++c) l[c] = widen(buf[tt][c]);
        const FT* colp = lc + (size_t)min(j + RING, NP - 1) * WP;
#pragma unroll
        for (int c = 0; c < C; ++c) buf[tt][c] = ld_raw(colp + 64 * c + lane);
        AT y[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          AT piv = acc[0][k];
#pragma unroll
          for (int c = 1; c < C; ++c) piv = (cb == c) ? acc[c][k] : piv;
          y[k] = readlane(piv, t);
        }
        const bool own = (lane_j == j);
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const bool take = own && (c == cb);
#pragma unroll
          for (int k = 0; k < NR; ++k) acc[c][k] = fma(-l[c], y[k], take ? rn[k] : acc[c][k]);
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) yl[k] = writelane(y[k], t, yl[k]);
        step_fence();
      }
    }
    const int row = j0 + lane;
    if (row < N)
#pragma unroll
      for (int k = 0; k < NR; ++k) yout[(size_t)row * NR + k] = (double)(yl[k] * dvl);
#pragma unroll
    for (int k = 0; k < NR; ++k) rn[k] = rnx[k];
  }
}

// Backward sweep Lt^T x = v (v read from and x written to yx).  Window before
// step j (descending): rows j-WP+1..j; the owner slot j % WP then takes row
// j-WP.  pre(row) is
// called at the start of each block of 64 steps (to issue the loads its
// epilogue needs early), post(row, x[NR]) at its end, when lane t holds x of
// row j0+t.
template <typename FT, int C, int NR, class Pre, class Post>
__device__ __forceinline__ void bwd_sweep(const int N, const int NP, const FT* __restrict__ lr,
                                          const double* yx, Pre& pre, Post& post) {
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
  // ring slot u holds the row consumed u steps (mod RING) after the start
  typename RawT<FT>::T buf[RING][C];
#pragma unroll
  for (int u = 0; u < RING; ++u) {
    const FT* rowp = lr + (size_t)max(NP - 1 - u, 0) * WP;
#pragma unroll
    for (int c = 0; c < C; ++c) buf[u][c] = ld_raw(rowp + 64 * c + lane);
  }
  const int nb = NP / 64;
  AT rn[NR];
  {
    const int nrow = 64 * (nb - 1) + lane - WP;
#pragma unroll
    for (int k = 0; k < NR; ++k) rn[k] = nrow >= 0 ? (AT)yx[(size_t)nrow * NR + k] : (AT)0;
  }
  wait_all_loads();

  for (int b = nb - 1; b >= 0; --b) {
    const int j0 = 64 * b;
    const int cb = b % C;
    AT rnx[NR];
    const int nrow = j0 - 64 + lane - WP;
#pragma unroll
    for (int k = 0; k < NR; ++k) rnx[k] = nrow >= 0 ? (AT)yx[(size_t)nrow * NR + k] : (AT)0;
    pre(j0 + lane);
    const int lane_j = opaque(j0 + lane);
    AT xl[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) xl[k] = (AT)0;
#pragma unroll
    for (int ch = 64 - RING; ch >= 0; ch -= RING) {
#pragma unroll
      for (int tt = RING - 1; tt >= 0; --tt) {
        const int t = ch + tt;
        const int j = j0 + t;
        const int su = RING - 1 - tt;
        AT l[C];
#pragma unroll
        for (int c = 0; c < C; ++c) l[c] = widen(buf[su][c]);
        const FT* rowp = lr + (size_t)max(j - RING, 0) * WP;
#pragma unroll
        for (int c = 0; c < C; ++c) buf[su][c] = ld_raw(rowp + 64 * c + lane);
        AT x[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          AT piv = acc[0][k];
#pragma unroll
          for (int c = 1; c < C; ++c) piv = (cb == c) ? acc[c][k] : piv;
          x[k] = readlane(piv, t);
        }
        const bool own = (lane_j == j);
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const bool take = own && (c == cb);
#pragma unroll
          for (int k = 0; k < NR; ++k) acc[c][k] = fma(-l[c], x[k], take ? rn[k] : acc[c][k]);
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) xl[k] = writelane(x[k], t, xl[k]);
        step_fence();
      }
    }
    double xd[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) xd[k] = (double)xl[k];
    post(j0 + lane, xd);
#pragma unroll
    for (int k = 0; k < NR; ++k) rn[k] = rnx[k];
  }
}

// ---------------------------------------------------------------------------
// Local solve / apply kernel, one subdomain per workgroup of two waves.
//   mode 0: out = A_i^{-1} r                          (local particular solution)
//   mode 1: out = A_i^{-1} r + sum_q eta_q phat^(q)    (preconditioner apply)
//   mode 2: mode 1 plus this block's (r, z) and (q, z) partial sums for PCG
// Wave 0 runs the two band sweeps.  Wave 1 gathers eta for the subdomain's
// basis functions while wave 0 runs the forward sweep: from the global eta
// (computed by the interface GEMV) or, when fuse_eta is set, as the
// subdomain's own rows of eta = S^{-1} b (so no separate interface launch is
// needed); in PCG mode with fuse_eta it also folds the ||r||^2 partials and
// applies the stop test ||r|| <= tol ||b|| (workgroup 0 stores the outcome).
constexpr int kMaxNiLds = 128;
constexpr int kPreQ = 8;  // MBF columns whose values are fetched a block ahead
constexpr int kEtaChunk = 24;  // interface columns per lane per chunk of the fused rows

template <int NR>
__device__ __forceinline__ bool stop_test(const double* __restrict__ pb, int npb, int init,
                                          PcgScalars* sc, PcgShared* sh) {
  // one wave: fold the ||r||^2 partials in block order (same order in every workgroup)
  const int lane = threadIdx.x & 63;
  double rr[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) rr[k] = 0.0;
  for (int b = lane; b < npb; b += 64)
#pragma unroll
    for (int k = 0; k < NR; ++k) rr[k] += pb[(size_t)b * NR + k];
#pragma unroll
  for (int k = 0; k < NR; ++k) rr[k] = wave_sum(rr[k]);
  int alld = 1;
  for (int k = 0; k < sh->nrhs; ++k) {
    const PcgScalars S = sc[k];
    int done = S.done, conv = S.conv, status = S.status;
    double bb = S.bb;
    if (!done) {
      if (init) {
        bb = rr[k];
        if (bb == 0.0) done = conv = 1;
      } else if (rr[k] <= S.tol2 * S.bb) {
        done = conv = 1;
      } else if (S.it >= sh->maxit) {
        done = 1;
        status = AM_ERR_NO_CONVERGENCE;
      }
    }
    alld &= done;
    if (blockIdx.x == 0 && lane == 0) {
      sc[k].rr = rr[k];
      sc[k].bb = bb;
      sc[k].done = done;
      sc[k].conv = conv;
      sc[k].status = status;
    }
  }
  if (blockIdx.x == 0 && lane == 0) sh->all_done = alld;
  return alld != 0;
}

template <typename FT, int C, int NR>
__global__ __launch_bounds__(128) void k_local(
    const int32_t* __restrict__ subs, const int64_t* __restrict__ sub_ptr,
    const int64_t* __restrict__ roff, const int64_t* __restrict__ fac_off,
    const FT* __restrict__ Lc, const FT* __restrict__ Lr,
    const typename AccT<FT>::T* __restrict__ dinv, const double* rin, double* out, int mode,
    const int64_t* __restrict__ isub_ptr, const int32_t* __restrict__ isub_list,
    const int64_t* __restrict__ mbf_off, const double* __restrict__ mbf,
    const double* __restrict__ eta, const double* __restrict__ qv, double* __restrict__ partial,
    unsigned blk_off, int fuse_eta, const double* __restrict__ Sinv, int NL, int ldS,
    const double* __restrict__ bpart, const double* __restrict__ pb, int npb, int init,
    PcgScalars* sc, PcgShared* sh) {
  if (mode == 2 && all_done(sh)) return;
  __shared__ double eta_s[kMaxNiLds * NR];
  __shared__ int stop_s;
  const int s = subs[blockIdx.x];
  const int64_t base = sub_ptr[s];
  const int N = (int)(sub_ptr[s + 1] - base);
  const int64_t ro = roff[s];
  const int NP = (int)(roff[s + 1] - ro);
  const FT* lc = Lc + fac_off[s];
  const FT* lr = Lr + fac_off[s];
  const auto* dv = dinv + ro;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t i0 = isub_ptr[s];
  const int ns = mode >= 1 ? (int)(isub_ptr[s + 1] - i0) : 0;
  const double* P = mbf + mbf_off[s];

  if (wave == 0) {
    fwd_sweep<FT, C, NR>(N, NP, lc, dv, rin + base * NR, out + base * NR);
  } else {
    int stop = 0;
    if (mode == 2 && fuse_eta) stop = stop_test<NR>(pb, npb, init, sc, sh) ? 1 : 0;
    if (lane == 0) stop_s = stop;
    if (!stop && ns > 0) {
      if (!fuse_eta) {
        for (int t = lane; t < ns * NR; t += 64)
          eta_s[t] = eta[(size_t)isub_list[i0 + t / NR] * NR + (t % NR)];
      } else {
        // rows I_s[q] of S^{-1} times b, b_m = bpart[2m] + bpart[2m+1]
        for (int q = 0; q < ns; ++q)
          if (lane == 0)
#pragma unroll
            for (int k = 0; k < NR; ++k) eta_s[q * NR + k] = 0.0;
        for (int m0 = 0; m0 < NL; m0 += 64 * kEtaChunk) {
          double bv[kEtaChunk][NR];
#pragma unroll
          for (int u = 0; u < kEtaChunk; ++u) {
            const int m = m0 + lane + 64 * u;
#pragma unroll
            for (int k = 0; k < NR; ++k)
              bv[u][k] = m < NL ? bpart[(size_t)(2 * m) * NR + k] + bpart[(size_t)(2 * m + 1) * NR + k] : 0.0;
          }
          for (int q = 0; q < ns; ++q) {
            const double* row = Sinv + (size_t)isub_list[i0 + q] * ldS;
            double a[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) a[k] = 0.0;
#pragma unroll
            for (int u = 0; u < kEtaChunk; ++u) {
              const int m = m0 + lane + 64 * u;
              const double sv = m < NL ? row[m] : 0.0;
#pragma unroll
              for (int k = 0; k < NR; ++k) a[k] = fma(sv, bv[u][k], a[k]);
            }
#pragma unroll
            for (int k = 0; k < NR; ++k) {
              const double t = wave_sum(a[k]);
              if (lane == 0) eta_s[q * NR + k] += t;
            }
          }
        }
      }
    }
  }
  __syncthreads();
  if (stop_s) return;
  if (wave != 0) return;

  double rz[NR], qz[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) rz[k] = qz[k] = 0.0;
  double* o = out + base * NR;
  const double* rr = rin + base * NR;
  const double* qq = qv + base * NR;
  double ph[kPreQ], rpre[NR], qpre[NR];
#pragma unroll
  for (int q = 0; q < kPreQ; ++q) ph[q] = 0.0;
#pragma unroll
  for (int k = 0; k < NR; ++k) rpre[k] = qpre[k] = 0.0;
  const int npre = min(ns, kPreQ);
  auto pre = [&](int row) {
    if (row >= N) return;
#pragma unroll
    for (int q = 0; q < kPreQ; ++q)
      if (q < npre) ph[q] = P[(size_t)q * N + row];
    if (mode == 2)
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        rpre[k] = rr[(size_t)row * NR + k];
        qpre[k] = qq[(size_t)row * NR + k];
      }
  };
  auto post = [&](int row, double (&x)[NR]) {
    if (row >= N) return;
#pragma unroll
    for (int q = 0; q < kPreQ; ++q)
      if (q < npre)
#pragma unroll
        for (int k = 0; k < NR; ++k) x[k] = fma(ph[q], eta_s[q * NR + k], x[k]);
    for (int q = kPreQ; q < ns; ++q) {
      const double v = P[(size_t)q * N + row];
#pragma unroll
      for (int k = 0; k < NR; ++k) x[k] = fma(v, eta_s[q * NR + k], x[k]);
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) o[(size_t)row * NR + k] = x[k];
    if (mode == 2)
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        rz[k] = fma(rpre[k], x[k], rz[k]);
        qz[k] = fma(qpre[k], x[k], qz[k]);
      }
  };
  bwd_sweep<FT, C, NR>(N, NP, lr, out + base * NR, pre, post);

  if (mode != 2) return;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const double a = wave_sum(rz[k]);
    const double b = wave_sum(qz[k]);
    if (lane == 0) {
      partial[(size_t)(blk_off + blockIdx.x) * 2 * NR + k] = a;
      partial[(size_t)(blk_off + blockIdx.x) * 2 * NR + NR + k] = b;
    }
  }
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
  auto pre = [&](int) {};
  auto post = [&](int row, double (&x)[1]) {
    if (row < N) col[row] = x[0];
  };
  bwd_sweep<FT, C, 1>(N, NP, Lr + fac_off[s], col, pre, post);
}

template <int NR>
__global__ __launch_bounds__(256) void k_bpart(const int64_t* __restrict__ sub_ptr,
                                               const int64_t* __restrict__ isub_ptr,
                                               const int64_t* __restrict__ mbf_off,
                                               const double* __restrict__ mbf,
                                               const int64_t* __restrict__ bdst,
                                               const double* __restrict__ r, double* bpart) {
  __shared__ double lds[4 * 16];  // block sums of up to 16 values
  bpart_sub<NR>(blockIdx.x, sub_ptr, isub_ptr, mbf_off, mbf, bdst, r, bpart, lds);
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
  unsigned off = 0;
  for (int bk = 0; bk < 2; ++bk) {
    const int nb = (int)d.bucket_sub[bk].size();
    if (!nb) continue;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(nb), dim3(128), 0, st, d.d_bucket_sub[bk], d.sub_ptr, d.roff,
                         d.fac_off, (const FT*)d.Lc, (const FT*)d.Lr, (const IT*)d.invd, r, z,
                         mode, d.isub_ptr, d.isub_list, d.mbf_off, d.mbf, eta, d.q, d.red.pd,
                         off, d.fuse_eta, d.Sinv, (int)d.NL, d.ldS, d.bpart, d.red.pb, d.m,
                         init, d.sc, d.shared);
    };
    if (bk == 0)
      go(k_local<FT, 1, NR>);
    else
      go(k_local<FT, 2, NR>);
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
  // mode >= 10: the PCG start pass (mode 2, init = 1)
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
    case 1: hipLaunchKernelGGL(k_bpart<1>, g, b, 0, st, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, d.bdst, r, d.bpart); break;
    case 2: hipLaunchKernelGGL(k_bpart<2>, g, b, 0, st, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, d.bdst, r, d.bpart); break;
    case 4: hipLaunchKernelGGL(k_bpart<4>, g, b, 0, st, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, d.bdst, r, d.bpart); break;
    case 8: hipLaunchKernelGGL(k_bpart<8>, g, b, 0, st, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, d.bdst, r, d.bpart); break;
    case 16: hipLaunchKernelGGL(k_bpart<16>, g, b, 0, st, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, d.bdst, r, d.bpart); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace am
