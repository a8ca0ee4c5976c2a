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
#pragma once
#include <type_traits>

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
    typename AccT<FT>::T* __restrict__ invd, int32_t* __restrict__ fail, int plain) {
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
  // couplings that leave the subdomain on the diagonal (plain: the diagonal
  // block A_ii itself, for block-Jacobi smoothing)
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
    if (!plain) Br[row % WN] -= dout;
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
// Block form of the sweeps, used at solve time.  After the set-up solves,
// every 64 x 64 diagonal block Lt_bb of the unit-diagonal factor is replaced
// in place, in both layouts, by its inverse (k_invert_diag).  With 64-row
// blocks the forward solution is
//   y_b = Lt_bb^{-1} t_b,   t_b = r_b - sum_{c=1..C} L_{b,b-c} y_{b-c},
// so a block costs two passes over its 64 columns, and the steps of a pass
// do not depend on each other:
//   pass B  y = Lt_bb^{-1} t_b: column jj of Lc holds Lt_bb^{-1}[ii][jj] in
//           lanes ii > jj of chunk b % C;
//   pass A  the accumulators of the next C blocks take -L_{b+c,b} y_b: the
//           other lanes (ii <= jj) of that chunk hold L_{b+C,b}[ii][jj], and
//           for C = 2 the other chunk holds the full L_{b+1,b}.
// The backward sweep is the mirror image on the rows of Lr (lanes ii < jj of
// chunk b % C hold Lt_bb^{-1}[jj][ii]; lanes ii >= jj hold L_{b,b-C}[jj][ii];
// the other chunk L_{b,b-1}).  The broadcast operand of a step is read from
// an LDS copy of the block's vector.  Each pass re-reads the columns of the
// other pass of the same block (an L2 hit); the ring prefetches along the
// sequence of both passes, so the first pass of a block is fetched while the
// second pass of the previous block runs.

template <int V> struct IC { static constexpr int v = V; };

// Diagonal-block inversion, one wave per (subdomain, 64-row block): lane k
// computes column k of X = Lt_bb^{-1} by forward substitution,
//   X[ii][k] = delta_ik - sum_{k <= jj < ii} Lt[ii][jj] X[jj][k],
// against the strict lower part of Lt_bb held in LDS (fp64); X replaces
// Lt_bb in the column layout Lc (column 64b+k, rows below the diagonal).
template <typename FT, int C>
__global__ __launch_bounds__(64) void k_invert_diag(const int32_t* __restrict__ subs,
                                                    const int64_t* __restrict__ roff,
                                                    const int64_t* __restrict__ fac_off,
                                                    FT* __restrict__ Lc) {
  constexpr int WP = 64 * C;
  constexpr int PL = 65;  // LDS pitch (doubles)
  __shared__ double Ld[64 * PL];
  __shared__ double X[64 * PL];
  const int s = subs[blockIdx.x];
  const int64_t ro = roff[s];
  const int NP = (int)(roff[s + 1] - ro);
  const int b = blockIdx.y;
  if (64 * b >= NP) return;
  FT* lc = Lc + fac_off[s];
  const int lane = threadIdx.x;
  const int cb = b % C;
  for (int jj = 0; jj < 64; ++jj)
    Ld[lane * PL + jj] =
        lane > jj ? (double)ld_fac(lc + (size_t)(64 * b + jj) * WP + 64 * cb + lane) : 0.0;
  __syncthreads();
  for (int ii = 0; ii < 64; ++ii) {
    double a = ii == lane ? 1.0 : 0.0;
    for (int jj = lane; jj < ii; ++jj) a = fma(-Ld[ii * PL + jj], X[jj * PL + lane], a);
    X[ii * PL + lane] = a;
  }
  __syncthreads();
  // column 64b+jj of Lc: rows ii > jj of the block (coalesced over ii)
  for (int jj = 0; jj < 64; ++jj)
    if (lane > jj) st_fac(lc + (size_t)(64 * b + jj) * WP + 64 * cb + lane, X[lane * PL + jj]);
}

// ---------------------------------------------------------------------------
constexpr int kPreQ = 8;  // MBF columns whose values are fetched a block ahead

// ---------------------------------------------------------------------------
// Tile form of the local solves (solve time).  After set-up only the column
// layout Lc is read, with every 64 x 64 diagonal block of the unit-diagonal
// factor replaced by its inverse (k_invert_diag).  With 64-row blocks,
//   forward   y_b = Lt_bb^{-1} t_b,    t_b = r_b - sum_{c=1..C} L_{b,b-c} y_{b-c}
//   backward  x_b = Lt_bb^{-T} s_b,    s_b = v_b - sum_{c=1..C} L_{b+c,b}^T x_{b+c}
// The 64 columns of block b (C chunks of 64 rows) are contiguous in Lc: the
// tile of block b holds Lt_bb^{-1} below its diagonal (chunk b % C) and the
// couplings L_{b+c,b} to the next C blocks in the remaining entries.  A
// workgroup stages each tile in LDS once per sweep (16-byte coalesced loads
// held in registers one or two tiles ahead, double buffered in LDS); the
// forward sweep reads it by columns
// and the backward sweep by rows (the transpose) from the same tile.  Every
// step of a pass is independent of the others: the W waves of a group take
// 64/W columns each and their partial vectors are summed in LDS in wave
// order; G groups of waves take NT/G right-hand sides each.
// Order a wave's LDS writes before its later LDS reads of other lanes' data
// (one wave, in-order LDS queue: only the compiler must not reorder).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// largest |I_i| the tile kernel holds eta for (checked at set-up)
template <int NT> struct TileMaxNi { static constexpr int v = NT >= 8 ? 64 : 128; };

template <typename FT> struct LdsPitch { static constexpr int v = sizeof(FT) == 2 ? 66 : 65; };

template <typename FT, int C, int NT, int G, int W>
__global__ __launch_bounds__(64 * G * W) void k_localt(
    const int32_t* __restrict__ subs, const int64_t* __restrict__ sub_ptr,
    const int64_t* __restrict__ roff, const int64_t* __restrict__ fac_off,
    const FT* __restrict__ Lc, const typename AccT<FT>::T* __restrict__ dinv, const double* rin,
    double* out, int mode, const int64_t* __restrict__ isub_ptr,
    const int32_t* __restrict__ isub_list, const int64_t* __restrict__ mbf_off,
    const double* __restrict__ mbf, const double* __restrict__ eta, const double* __restrict__ qv,
    double* __restrict__ partial, unsigned blk_off, int fuse_eta, const double* __restrict__ Sinv,
    int NL, int ldS, const double* __restrict__ bpart, const double* __restrict__ pb, int npb,
    int init, PcgScalars* sc, PcgShared* sh, int64_t nrows) {
  using AT = typename AccT<FT>::T;
  constexpr int NR = NT / G;
  constexpr int WP = 64 * C;
  constexpr int PITCH = LdsPitch<FT>::v;
  constexpr int CH = 64 * PITCH;            // LDS elements per chunk
  constexpr int NTHR = 64 * G * W;
  constexpr int VEC = 16 / (int)sizeof(FT);  // factor elements per 16-byte load
  constexpr int NLD = 64 * WP / (VEC * NTHR);
  static_assert((64 * WP) % (VEC * NTHR) == 0, "tile must split into 16-byte loads");
  constexpr int CW = 64 / W;  // columns of a pass per wave
  __shared__ FT tile[2][C * CH];
  __shared__ AT red[2][G][W > 1 ? W : 1][C][W > 1 ? 64 * NR : 1];
  __shared__ double eta_s[TileMaxNi<NT>::v * NT];
  __shared__ double dots[G][W][2 * NR];
  // broadcast copies of block vectors, one per group: each wave writes and
  // reads only the rows of its own columns (no cross-wave dependency)
  __shared__ AT bvec[G][2][64 * NR];
  __shared__ int stop_s;

  const int s = subs ? subs[blockIdx.x] : (int)blockIdx.x;  // null: the identity list
  const int64_t base = sub_ptr[s];
  const int N = (int)(sub_ptr[s + 1] - base);
  const int64_t ro = roff[s];
  const int NP = (int)(roff[s + 1] - ro);
  const int NB = NP / 64;
  const FT* lc = Lc + fac_off[s];
  const AT* dv = dinv + ro;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = wave / W, w = wave % W;
  const int k0 = g * NR;
  const int c0 = w * CW;
  const bool mine = lane >= c0 && lane < c0 + CW;  // rows of this wave's columns
  const int64_t i0 = isub_ptr[s];
  const int ns = mode >= 1 ? (int)(isub_ptr[s + 1] - i0) : 0;
  const double* P = mbf + mbf_off[s];
  // node vectors: value (row, k) of this subdomain at vi(row, k) (see vix)
  auto vi = [&](int row, int k) { return vix<NT>(nrows, base + row, k0 + k); };

  // register prefetch of the next PD tiles of a sweep: the tile of block b
  // travels through pre[b % PD] into LDS buffer b & 1 (slots and buffers
  // follow the block's parity, so every index below is a constant)
  constexpr int PD = (C == 1 || sizeof(FT) < 8) ? 2 : 1;
  uint4 pre[PD][NLD];
  auto tile_load = [&](int b, int slot) {
    const uint4* src = reinterpret_cast<const uint4*>(lc + (size_t)64 * b * WP);
#pragma unroll
    for (int u = 0; u < NLD; ++u) pre[slot][u] = src[u * NTHR + threadIdx.x];
  };
  auto tile_store = [&](int buf, int slot) {
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int e0 = (u * NTHR + (int)threadIdx.x) * VEC;  // column e0 / WP, slots e0 % WP ..
      const int col = e0 / WP, slot_e = e0 % WP;
      FT* dst = tile[buf] + (slot_e / 64) * CH + col * PITCH + (slot_e % 64);
      FT v[VEC];
      __builtin_memcpy(v, &pre[slot][u], 16);
#pragma unroll
      for (int t = 0; t < VEC; ++t) dst[t] = v[t];
    }
  };
  // coefficient (chunk c, row ii, column jj) of the tile in buffer buf
  auto coef = [&](int buf, int c, int ii, int jj) -> AT {
    return (AT)widen_lds(tile[buf][c * CH + jj * PITCH + ii]);
  };

  tile_load(0, 0);
  // Early exit of a solve that has stopped.  With the interface solve fused
  // in, workgroup 0 of this very launch may write all_done while the other
  // workgroups read it, so a per-wave read could split a workgroup; there the
  // decision comes from the stop test below, which every wave evaluates on
  // the same partials, and is shared through stop_s after the barrier.
  // Without it, all_done was written by an earlier launch and is uniform.
  if (mode == 2 && !fuse_eta && all_done(sh)) return;  // (after the first tile is in flight)
  // ---- stop test and eta (every wave takes part) ----
  // Fused interface solve: wave v forms, for every row q of this subdomain,
  // the partial dot of S^{-1}[I_s[q], m] with b_m over its share of the
  // columns m; the partials go to LDS (the second tile buffer, free until the
  // first prefetch is stored) and are summed in wave order after the barrier.
  double* etap = reinterpret_cast<double*>(tile[1]);  // [G*W][ns][NT]
  bool eta_fold = false;
  {
    int stop = 0;
    if (mode == 2 && fuse_eta) stop = stop_test<NT>(pb, npb, init, sc, sh, threadIdx.x == 0) ? 1 : 0;
    if (threadIdx.x == 0) stop_s = stop;
    if (!stop && ns > 0) {
      if (!fuse_eta) {
        for (int t = threadIdx.x; t < ns * NT; t += NTHR)
          eta_s[t] = eta[(size_t)isub_list[i0 + t / NT] * NT + (t % NT)];
      } else {
        eta_fold = true;
        constexpr int EQ = NT >= 8 ? 1 : 8 / NT;  // rows per chunk
        const int per = (NL + G * W - 1) / (G * W);
        const int mb = wave * per, me = min(NL, mb + per);
        for (int q0 = 0; q0 < ns; q0 += EQ) {
          const double* rowp[EQ];
#pragma unroll
          for (int qq = 0; qq < EQ; ++qq)
            rowp[qq] = Sinv + (size_t)isub_list[i0 + min(q0 + qq, ns - 1)] * ldS;
          double a[EQ][NT];
#pragma unroll
          for (int qq = 0; qq < EQ; ++qq)
#pragma unroll
            for (int k = 0; k < NT; ++k) a[qq][k] = 0.0;
#pragma unroll 4
          for (int m = mb + lane; m < me; m += 64) {
            double bm[NT];
#pragma unroll
            for (int k = 0; k < NT; ++k)
              bm[k] = bpart[(size_t)(2 * m) * NT + k] + bpart[(size_t)(2 * m + 1) * NT + k];
#pragma unroll
            for (int qq = 0; qq < EQ; ++qq) {
              const double sv = rowp[qq][m];
#pragma unroll
              for (int k = 0; k < NT; ++k) a[qq][k] = fma(sv, bm[k], a[qq][k]);
            }
          }
#pragma unroll
          for (int qq = 0; qq < EQ; ++qq)
#pragma unroll
            for (int k = 0; k < NT; ++k) {
              const double t = wave_sum(a[qq][k]);
              if (lane == 0 && q0 + qq < ns) etap[((size_t)wave * ns + q0 + qq) * NT + k] = t;
            }
        }
      }
    }
  }
  __syncthreads();
  if (stop_s) return;
  if (eta_fold) {
    for (int t = threadIdx.x; t < ns * NT; t += NTHR) {
      double e = 0.0;
      for (int v = 0; v < G * W; ++v) e += etap[(size_t)v * ns * NT + t];
      eta_s[t] = e;
    }
    __syncthreads();  // etap (tile buffer 1) is read before the prefetch overwrites it
  }
  tile_store(0, 0);
  if (1 < NB) tile_load(1, 1 % PD);
  if (PD == 2 && 2 < NB) tile_load(2, 0);
  __syncthreads();

  // ---- forward sweep ----
  AT T[C][NR];  // accumulators of blocks b .. b+C-1 (identical in the W waves of a group)
  auto ldr = [&](int row, int k) -> AT {
    return (row >= 0 && row < N) ? (AT)rin[vi(row, k)] : (AT)0;
  };
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int k = 0; k < NR; ++k) T[c][k] = ldr(64 * c + lane, k);

  auto fwd_body = [&](const int b, auto parc) {
    constexpr int par = decltype(parc)::v;  // b & 1
    constexpr int cb = C == 2 ? par : 0;
    constexpr int buf = par;
    const int j0 = 64 * b;
    AT rn[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) rn[k] = ldr(j0 + WP + lane, k);
    const AT dvl = dv[j0 + lane];
    // pass B: y = t + sum_{jj < ii} Lt_bb^{-1}[ii][jj] t[jj]
    AT* bv = bvec[g][0];
    wave_lds_sync();
    if (mine)
#pragma unroll
      for (int k = 0; k < NR; ++k) bv[lane * NR + k] = T[0][k];
    wave_lds_sync();
    AT p[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) p[k] = (AT)0;
#pragma unroll 8
    for (int sx = 0; sx < CW; ++sx) {
      const int jj = c0 + sx;
      const AT cf = coef(buf, cb, lane, jj);
      const AT d = lane > jj ? cf : (AT)0;
#pragma unroll
      for (int k = 0; k < NR; ++k) p[k] = fma(d, bv[jj * NR + k], p[k]);
    }
    AT y[NR];
    if constexpr (W > 1) {
#pragma unroll
      for (int k = 0; k < NR; ++k) red[0][g][w][0][lane * NR + k] = p[k];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        AT a = T[0][k];
#pragma unroll
        for (int u = 0; u < W; ++u) a += red[0][g][u][0][lane * NR + k];
        y[k] = a;
      }
    } else {
#pragma unroll
      for (int k = 0; k < NR; ++k) y[k] = T[0][k] + p[k];
    }
    if (w == (b % W) && j0 + lane < N)
#pragma unroll
      for (int k = 0; k < NR; ++k) out[vi(j0 + lane, k)] = (double)(y[k] * dvl);
    // pass A: blocks b+1 .. b+C take -L_{b+c,b} y_b
    AT* by = bvec[g][1];
    wave_lds_sync();
    if (mine)
#pragma unroll
      for (int k = 0; k < NR; ++k) by[lane * NR + k] = y[k];
    wave_lds_sync();
    AT qf[NR], qn[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) qf[k] = qn[k] = (AT)0;
#pragma unroll 8
    for (int sx = 0; sx < CW; ++sx) {
      const int jj = c0 + sx;
      const AT cf = coef(buf, cb, lane, jj);
      const AT e = lane <= jj ? cf : (AT)0;
      AT cn = (AT)0;
      if constexpr (C == 2) cn = coef(buf, 1 - cb, lane, jj);
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const AT yb = by[jj * NR + k];
        qf[k] = fma(e, yb, qf[k]);
        if constexpr (C == 2) qn[k] = fma(cn, yb, qn[k]);
      }
    }
    if (b + 1 < NB) {
      constexpr int nslot = (par + 1) % PD;
      tile_store(1 - par, nslot);
      if (b + 1 + PD < NB) tile_load(b + 1 + PD, nslot);
    }
    if constexpr (W > 1) {
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        red[1][g][w][0][lane * NR + k] = qf[k];
        if constexpr (C == 2) red[1][g][w][1][lane * NR + k] = qn[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      AT sf = qf[k], sn = qn[k];
      if constexpr (W > 1) {
        sf = sn = (AT)0;
#pragma unroll
        for (int u = 0; u < W; ++u) {
          sf += red[1][g][u][0][lane * NR + k];
          if constexpr (C == 2) sn += red[1][g][u][1][lane * NR + k];
        }
      }
      if constexpr (C == 2) {
        T[0][k] = T[1][k] - sn;
        T[1][k] = rn[k] - sf;
      } else {
        T[0][k] = rn[k] - sf;
      }
    }
  };
  for (int b = 0; b < NB; b += 2) {
    fwd_body(b, IC<0>{});
    if (b + 1 < NB) fwd_body(b + 1, IC<1>{});
  }

  // ---- backward sweep (tiles from the last block down) ----
  // The forward sweep leaves the tiles of blocks NB-1 and NB-2 in LDS buffers
  // (NB-1) & 1 and (NB-2) & 1, where the backward steps of those blocks read
  // them (transposed); the ring restarts with block NB-3.
  if (PD == 2 && NB > 2) {
    if ((NB - 3) & 1)
      tile_load(NB - 3, 1 % PD);
    else
      tile_load(NB - 3, 0);
  }
  __syncthreads();  // every wave's forward output rows are written

  double rz[NR], qz[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) rz[k] = qz[k] = 0.0;
  const int npre = min(ns, kPreQ);
  AT X1[NR], X2[NR];  // x of blocks b+1, b+2
#pragma unroll
  for (int k = 0; k < NR; ++k) X1[k] = X2[k] = (AT)0;
  auto ldv = [&](int row, int k) -> AT {
    return (row >= 0 && row < N) ? (AT)out[vi(row, k)] : (AT)0;
  };

  auto bwd_body = [&](const int b, auto parc) {
    constexpr int par = decltype(parc)::v;  // b & 1
    constexpr int cb = C == 2 ? par : 0;
    constexpr int buf = par;
    const int j0 = 64 * b;
    const int row = j0 + lane;
    const bool poster = (w == (b % W)) && row < N;
    double ph[kPreQ], rpre[NR], qpre[NR];
    if (poster) {
#pragma unroll
      for (int q = 0; q < kPreQ; ++q) ph[q] = q < npre ? P[(size_t)q * N + row] : 0.0;
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        rpre[k] = mode == 2 ? rin[vi(row, k)] : 0.0;
        qpre[k] = mode == 2 ? qv[vi(row, k)] : 0.0;
      }
    }
    AT v[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) v[k] = ldv(row, k);
    // pass A: s = v - L_{b+1,b}^T x_{b+1} - L_{b+2,b}^T x_{b+2}
    AT* bx1 = bvec[g][0];
    AT* bx2 = bvec[g][1];
    wave_lds_sync();
    if (mine)
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        bx1[lane * NR + k] = X1[k];
        if constexpr (C == 2) bx2[lane * NR + k] = X2[k];
      }
    wave_lds_sync();
    AT a[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) a[k] = (AT)0;
#pragma unroll 8
    for (int sx = 0; sx < CW; ++sx) {
      const int jj = c0 + sx;
      const AT cf = coef(buf, cb, jj, lane);  // (row jj, column lane) of the tile
      const AT e = lane >= jj ? cf : (AT)0;
      AT cn = (AT)0;
      if constexpr (C == 2) cn = coef(buf, 1 - cb, jj, lane);
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        if constexpr (C == 2) {
          a[k] = fma(cn, bx1[jj * NR + k], a[k]);
          a[k] = fma(e, bx2[jj * NR + k], a[k]);
        } else {
          a[k] = fma(e, bx1[jj * NR + k], a[k]);
        }
      }
    }
    AT t[NR];
    if constexpr (W > 1) {
#pragma unroll
      for (int k = 0; k < NR; ++k) red[0][g][w][0][lane * NR + k] = a[k];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        AT acc = (AT)0;
#pragma unroll
        for (int u = 0; u < W; ++u) acc += red[0][g][u][0][lane * NR + k];
        t[k] = v[k] - acc;
      }
    } else {
#pragma unroll
      for (int k = 0; k < NR; ++k) t[k] = v[k] - a[k];
    }
    // pass B: x = t + sum_{jj > ii} Lt_bb^{-1}[jj][ii] t[jj]
    AT* bt = bvec[g][0];
    wave_lds_sync();
    if (mine)
#pragma unroll
      for (int k = 0; k < NR; ++k) bt[lane * NR + k] = t[k];
    wave_lds_sync();
    AT pb2[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) pb2[k] = (AT)0;
#pragma unroll 8
    for (int sx = 0; sx < CW; ++sx) {
      const int jj = c0 + sx;
      const AT cf = coef(buf, cb, jj, lane);
      const AT d = lane < jj ? cf : (AT)0;
#pragma unroll
      for (int k = 0; k < NR; ++k) pb2[k] = fma(d, bt[jj * NR + k], pb2[k]);
    }
    if (b > 0) {
      constexpr int nslot = (par + 1) % PD;  // (b - 1) % PD
      if (b < NB - 1) tile_store(1 - par, nslot);
      if (b - 1 - PD >= 0) tile_load(b - 1 - PD, nslot);
    }
    if constexpr (W > 1) {
#pragma unroll
      for (int k = 0; k < NR; ++k) red[1][g][w][0][lane * NR + k] = pb2[k];
    }
    __syncthreads();
    AT x[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      AT acc = pb2[k];
      if constexpr (W > 1) {
        acc = (AT)0;
#pragma unroll
        for (int u = 0; u < W; ++u) acc += red[1][g][u][0][lane * NR + k];
      }
      x[k] = t[k] + acc;
      X2[k] = X1[k];
      X1[k] = x[k];
    }
    if (poster) {
      double z[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) z[k] = (double)x[k];
#pragma unroll
      for (int q = 0; q < kPreQ; ++q)
        if (q < npre)
#pragma unroll
          for (int k = 0; k < NR; ++k) z[k] = fma(ph[q], eta_s[q * NT + k0 + k], z[k]);
      for (int q = kPreQ; q < ns; ++q) {
        const double pv = P[(size_t)q * N + row];
#pragma unroll
        for (int k = 0; k < NR; ++k) z[k] = fma(pv, eta_s[q * NT + k0 + k], z[k]);
      }
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        out[vi(row, k)] = z[k];
        rz[k] = fma(rpre[k], z[k], rz[k]);
        qz[k] = fma(qpre[k], z[k], qz[k]);
      }
    }
  };
  {
    int b = NB - 1;
    if (b & 1) bwd_body(b--, IC<1>{});
    for (; b >= 0; b -= 2) {
      bwd_body(b, IC<0>{});
      if (b - 1 >= 0) bwd_body(b - 1, IC<1>{});
    }
  }

  if (mode != 2) return;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const double a = wave_sum(rz[k]);
    const double b2 = wave_sum(qz[k]);
    if (lane == 0) {
      dots[g][w][k] = a;
      dots[g][w][NR + k] = b2;
    }
  }
  __syncthreads();
  if (w == 0 && lane == 0)
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      double a = 0.0, b2 = 0.0;
#pragma unroll
      for (int u = 0; u < W; ++u) {
        a += dots[g][u][k];
        b2 += dots[g][u][NR + k];
      }
      partial[(size_t)(blk_off + blockIdx.x) * 2 * NT + k0 + k] = a;
      partial[(size_t)(blk_off + blockIdx.x) * 2 * NT + NT + k0 + k] = b2;
    }
}

// Tile form for 16 right-hand sides on the matrix cores (window 64, interface
// solve done before the launch).  Each tile pass is a dense 64 x 64 by
// 64 x 16 product, so the four waves of the workgroup each take 16 rows of
// the output block and accumulate all 16 right-hand sides over the 64
// columns: no partial sums cross waves.  FP64 factors use
// v_mfma_f64_16x16x4f64; FP32 and BF16 factors (widened to FP32 when the
// tile is staged) use v_mfma_f32_16x16x4f32 with FP32 block vectors, the
// arithmetic of the vector-unit kernel for those factors.  Both take lane l's
// operands as A[l % 16][l / 16] and B[l / 16][l % 16]; the FP64 result is
// D[l / 16 + 4 v][l % 16], the FP32 one D[4 (l / 16) + v][l % 16] (v < 4).
// With BF16 factors and BFOP, the products are BF16 x BF16 with FP32
// accumulation instead (v_mfma_f32_16x16x16bf16_1k, the block vectors
// rounded to BF16; see mf_pass).  The block vectors (64 rows x 16) live in
// LDS (two buffers, pitch 17); each tile goes through registers (loaded
// while the previous one is in use) into one LDS buffer.
//   forward  y_b = t_b + Nlow_b t_b,   out_b = dinv y_b,
//            t_{b+1} = r_{b+1} - U_b y_b
//   backward s_b = out_b - U_b^T x_{b+1},   x_b = s_b + Nlow_b^T s_b,
//            z_b = x_b + sum_q phat_q eta_q   (mode >= 1), PCG dots (mode 2)
// with Nlow_b the strictly lower part of tile b (the inverted diagonal
// block) and U_b its upper part with the diagonal (the coupling to block
// b + 1).
typedef double am_mf_d4 __attribute__((ext_vector_type(4)));
typedef float am_mf_f4 __attribute__((ext_vector_type(4)));
constexpr int kMfVP = 17;  // LDS pitch of a block-vector row (16 values + 1)
template <typename AT> struct MfAcc;
template <> struct MfAcc<double> {
  using V = am_mf_d4;
  // row of the 16 x 16 result held in element v of a lane with l / 16 = lk
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <> struct MfAcc<float> {
  using V = am_mf_f4;
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};
__device__ __forceinline__ am_mf_d4 mf4(double a, double b, am_mf_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ am_mf_f4 mf4(float a, float b, am_mf_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}


// acc += sum over the 64 columns jj of A[rows][jj] B[jj][.] for a 16-row
// strip, afn(c, m) and bfn(c, m) giving this lane's operands at column
// jj = c + m lk (lk = lane / 16, held by the caller), c and m constants of
// the unrolled loop.  FP64 / FP32 (16x16x4 products): lane holds column 4 kk + lk of
// step kk; the 16 operand pairs are read from LDS first, then four
// independent chains of four products (kk = c mod 4 in chain c) are added in
// chain order.  BF16 (BFOP, FP32 arithmetic type only): four 16x16x16
// products, lane holding columns 16 c + 4 lk .. 16 c + 4 lk + 3 of step c,
// both operands rounded to BF16 (the factor values are BF16 already), two
// chains added in order.
__device__ __forceinline__ short am_bf16_rne(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
typedef short am_mf_s4 __attribute__((ext_vector_type(4)));
template <bool BFOP, typename V, typename AF, typename BF>
__device__ __forceinline__ V mf_pass(V acc, AF&& afn, BF&& bfn) {
  using AT = decltype(afn(0, 0));
  if constexpr (BFOP) {
    static_assert(sizeof(AT) == 4, "BF16 products: FP32 arithmetic type");
    V c[2];
    c[0] = acc;
    c[1] = V{0, 0, 0, 0};
    am_mf_s4 a[4], b[4];
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[st][t] = am_bf16_rne(afn(16 * st + t, 4));
        b[st][t] = am_bf16_rne(bfn(16 * st + t, 4));
      }
#pragma unroll
    for (int st = 0; st < 4; ++st)
      c[st % 2] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[st], b[st], c[st % 2], 0, 0, 0);
    return c[0] + c[1];
  } else {
    V c[4];
    c[0] = acc;
#pragma unroll
    for (int t = 1; t < 4; ++t) c[t] = V{0, 0, 0, 0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // two halves of 8 operand pairs (registers)
      AT a[8], b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a[u] = afn(4 * (8 * h + u), 1);
        b[u] = bfn(4 * (8 * h + u), 1);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) c[u % 4] = mf4(a[u], b[u], c[u % 4]);
    }
    return (c[0] + c[1]) + (c[2] + c[3]);
  }
}

template <typename FT, int NT, bool BFOP = false>
__global__ __launch_bounds__(256) void k_localt_mf(
    const int32_t* __restrict__ subs, const int64_t* __restrict__ sub_ptr,
    const int64_t* __restrict__ roff, const int64_t* __restrict__ fac_off,
    const FT* __restrict__ Lc, const typename AccT<FT>::T* __restrict__ dinv, const double* rin,
    double* out, int mode, const int64_t* __restrict__ isub_ptr,
    const int32_t* __restrict__ isub_list, const int64_t* __restrict__ mbf_off,
    const double* __restrict__ mbf, const double* __restrict__ eta, const double* __restrict__ qv,
    double* __restrict__ partial, unsigned blk_off, PcgShared* sh, int64_t nrows) {
  // 16 right-hand sides fill the 16 columns of a matrix-core tile; one
  // right-hand side takes column 0 (lanes of the other columns carry zeros)
  static_assert(NT == 16 || NT == 1, "one 16-column matrix-core tile");
  using AT = typename AccT<FT>::T;  // arithmetic type: FP64, else FP32
  using V = typename MfAcc<AT>::V;
  constexpr int PITCH = 65;
  constexpr int CH = 64 * PITCH;
  constexpr int NTHR = 256;
  constexpr int VEC = 16 / (int)sizeof(FT);       // factor elements per 16-byte load
  constexpr int NLD = 64 * 64 / (VEC * NTHR);     // 16-byte loads per thread per tile
  constexpr int PD = 1;  // one tile ahead in registers (two workgroups per CU)
  __shared__ AT tile[CH];  // one buffer: two workgroups fit a CU
  __shared__ AT vb[2][64 * kMfVP];
  __shared__ AT eta_s[TileMaxNi<NT>::v * NT];
  __shared__ double dots[4][2 * NT];

  const int s = subs[blockIdx.x];
  const int64_t base = sub_ptr[s];
  const int N = (int)(sub_ptr[s + 1] - base);
  const int64_t ro = roff[s];
  const int NP = (int)(roff[s + 1] - ro);
  const int NB = NP / 64;
  const FT* lc = Lc + fac_off[s];
  const AT* dv = dinv + ro;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane % 16, lk = lane / 16;
  const bool colok = li < NT;  // this lane's column is a right-hand side
  const int64_t i0 = isub_ptr[s];
  const int ns = mode >= 1 ? (int)(isub_ptr[s + 1] - i0) : 0;
  const double* P = mbf + mbf_off[s];
  auto vi = [&](int row, int k) { return vix<NT>(nrows, base + row, k); };

  uint4 pre[PD][NLD];
  auto tile_load = [&](int b, int slot) {
    const uint4* src = reinterpret_cast<const uint4*>(lc + (size_t)64 * b * 64);
#pragma unroll
    for (int u = 0; u < NLD; ++u) pre[slot][u] = src[u * NTHR + threadIdx.x];
  };
  auto tile_store = [&](int slot) {
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int e0 = (u * NTHR + (int)threadIdx.x) * VEC;  // column e0 / 64, rows e0 % 64 ..
      AT* dst = tile + (e0 / 64) * PITCH + (e0 % 64);
      FT v[VEC];
      __builtin_memcpy(v, &pre[slot][u], 16);
#pragma unroll
      for (int t = 0; t < VEC; ++t) dst[t] = (AT)widen_lds(v[t]);
    }
  };
  // rows of this lane's part of the D layout
  auto drow = [&](int v) { return 16 * w + MfAcc<AT>::row(lk, v); };

  tile_load(0, 0);
  if (mode == 2 && all_done(sh)) return;
  for (int t = threadIdx.x; t < ns * NT; t += NTHR)
    eta_s[t] = (AT)eta[(size_t)isub_list[i0 + t / NT] * NT + (t % NT)];
  tile_store(0);
  if (1 < NB) tile_load(1, 0);
  // t_0 = r of block 0 (columns beyond NT: zero)
  for (int e = threadIdx.x; e < 64 * 16; e += NTHR) {
    const int row = e / 16, k = e % 16;
    vb[0][row * kMfVP + k] = (row < N && k < NT) ? (AT)rin[vi(row, k)] : AT(0);
  }
  __syncthreads();

  // ---- forward sweep ----
  auto fwd_body = [&](const int b, auto parc) {
    constexpr int par = decltype(parc)::v;  // b & 1
    const int j0 = 64 * b;
    AT rn[4], dvl[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = j0 + 64 + drow(v);
      rn[v] = (row < N && colok) ? (AT)rin[vi(row, li)] : AT(0);
      dvl[v] = dv[j0 + drow(v)];
    }
    const AT* T = tile;
    // pass B: y = t + Nlow t
    V acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = vb[0][drow(v) * kMfVP + li];
    {
      const int ii = 16 * w + li;
      acc = mf_pass<BFOP>(
          acc, [&](int c, int m) { const int jj = c + m * lk; return ii > jj ? T[jj * PITCH + ii] : AT(0); },
          [&](int c, int m) { const int jj = c + m * lk; return vb[0][jj * kMfVP + li]; });
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      vb[1][drow(v) * kMfVP + li] = acc[v];
      const int row = j0 + drow(v);
      if (row < N && colok) out[vi(row, li)] = (double)(acc[v] * dvl[v]);
    }
    __syncthreads();
    // pass A: t_{b+1} = r_{b+1} - U y
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = rn[v];
    {
      const int ii = 16 * w + li;
      acc = mf_pass<BFOP>(
          acc, [&](int c, int m) { const int jj = c + m * lk; return ii <= jj ? -T[jj * PITCH + ii] : AT(0); },
          [&](int c, int m) { const int jj = c + m * lk; return vb[1][jj * kMfVP + li]; });
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) vb[0][drow(v) * kMfVP + li] = acc[v];
    __syncthreads();  // every wave is done with tile b
    if (b + 1 < NB) {
      tile_store((par + 1) % PD);
      if (b + 1 + PD < NB) tile_load(b + 1 + PD, (par + 1) % PD);
      __syncthreads();
    }
  };
  for (int b = 0; b < NB; b += 2) {
    fwd_body(b, IC<0>{});
    if (b + 1 < NB) fwd_body(b + 1, IC<1>{});
  }

  // ---- backward sweep: tile NB-1 is still in LDS ----
  if (NB > 1) tile_load(NB - 2, 0);
  // x_{NB} = 0
  for (int e = threadIdx.x; e < 64 * 16; e += NTHR) vb[1][(e / 16) * kMfVP + e % 16] = AT(0);
  __syncthreads();
  double rz = 0.0, qz = 0.0;  // column li of this lane's rows
  auto bwd_body = [&](const int b, auto parc) {
    constexpr int par = decltype(parc)::v;  // b & 1
    const int j0 = 64 * b;
    const AT* T = tile;
    AT vv[4];
    double rp[4], qp[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = j0 + drow(v);
      const bool ok = row < N && colok;
      vv[v] = ok ? (AT)out[vi(row, li)] : AT(0);
      rp[v] = (ok && mode == 2) ? rin[vi(row, li)] : 0.0;
      qp[v] = (ok && mode == 2) ? qv[vi(row, li)] : 0.0;
    }
    // basis-function values of this block for the reconstruction, fetched
    // before the passes: A[row 16 w + li][slot q0 + lk] of z += phat eta
    constexpr int NPA = 8;  // slots 0..31 fetched ahead, the rest when used
    const int ra = j0 + 16 * w + li;
    AT pa[NPA];
#pragma unroll
    for (int c = 0; c < NPA; ++c) {
      const int q = 4 * c + lk;
      pa[c] = (q < ns && ra < N) ? (AT)P[(size_t)q * N + ra] : AT(0);
    }
    // pass A: s = out_b - U^T x_{b+1}
    V acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = vv[v];
    {
      const int ii = 16 * w + li;  // output row ii, tile row jj
      acc = mf_pass<BFOP>(
          acc, [&](int c, int m) { const int jj = c + m * lk; return jj <= ii ? -T[ii * PITCH + jj] : AT(0); },
          [&](int c, int m) { const int jj = c + m * lk; return vb[1][jj * kMfVP + li]; });
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) vb[0][drow(v) * kMfVP + li] = acc[v];
    __syncthreads();
    // pass B: x = s + Nlow^T s
    {
      const int ii = 16 * w + li;
      acc = mf_pass<BFOP>(
          acc, [&](int c, int m) { const int jj = c + m * lk; return jj > ii ? T[ii * PITCH + jj] : AT(0); },
          [&](int c, int m) { const int jj = c + m * lk; return vb[0][jj * kMfVP + li]; });
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) vb[1][drow(v) * kMfVP + li] = acc[v];
    // z = x + P_b eta on the matrix cores (slots in chunks of 4)
#pragma unroll
    for (int c = 0; c < NPA; ++c) {
      if (4 * c >= ns) break;  // uniform
      const int q = 4 * c + lk;
      const AT e = (q < ns && colok) ? eta_s[q * NT + li] : AT(0);
      acc = mf4(pa[c], e, acc);
    }
    for (int c = NPA; 4 * c < ns; ++c) {
      const int q = 4 * c + lk;
      const AT av = (q < ns && ra < N) ? (AT)P[(size_t)q * N + ra] : AT(0);
      const AT e = (q < ns && colok) ? eta_s[q * NT + li] : AT(0);
      acc = mf4(av, e, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = j0 + drow(v);
      if (row < N && colok) {
        const double zv = (double)acc[v];
        out[vi(row, li)] = zv;
        rz = fma(rp[v], zv, rz);
        qz = fma(qp[v], zv, qz);
      }
    }
    __syncthreads();  // every wave is done with tile b
    if (b > 0) {
      tile_store((par + 1) % PD);  // tile b - 1
      if (b - 1 - PD >= 0) tile_load(b - 1 - PD, (par + 1) % PD);
      __syncthreads();
    }
  };
  {
    int b = NB - 1;
    if (b & 1) bwd_body(b--, IC<1>{});
    for (; b >= 0; b -= 2) {
      bwd_body(b, IC<0>{});
      if (b - 1 >= 0) bwd_body(b - 1, IC<1>{});
    }
  }

  if (mode != 2) return;
  // lanes l, l ^ 16, l ^ 32, l ^ 48 hold the same column
  rz += __shfl_xor(rz, 16, 64);
  rz += __shfl_xor(rz, 32, 64);
  qz += __shfl_xor(qz, 16, 64);
  qz += __shfl_xor(qz, 32, 64);
  if (lane < NT) {
    dots[w][lane] = rz;
    dots[w][NT + lane] = qz;
  }
  __syncthreads();
  if (threadIdx.x < 2 * NT) {
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) a += dots[u][threadIdx.x];
    partial[(size_t)(blk_off + blockIdx.x) * 2 * NT + threadIdx.x] = a;
  }
}

// The same for window 128 (a bandwidth of 65-128 rows): a column keeps its
// 128 band entries in a ring of two 64-row chunks, so that in tile b the
// chunk b & 1 holds the rows of block b (strictly lower part: the inverted
// diagonal block; upper part with the diagonal: the coupling L_{b+2,b} to
// block b + 2) and the other chunk the full coupling L_{b+1,b}.
//   forward  y_b = t_b + Nlow_b t_b,   out_b = dinv y_b,
//            t_{b+1} = u_{b+1} - L_{b+1,b} y_b,   u_{b+2} = r_{b+2} - L_{b+2,b} y_b
//   backward s_b = out_b - L_{b+1,b}^T x_{b+1} - L_{b+2,b}^T x_{b+2},
//            x_b = s_b + Nlow_b^T s_b,  z_b = x_b + sum_q phat_q eta_q, dots
// Three block vectors live in LDS (forward: t, y, u; backward: x_{b+1},
// x_{b+2}, s, with x_b written over x_{b+2}), with one tile buffer of two
// chunks: about 100 KB, so that a workgroup of the window-64 kernel still
// fits beside it on a CU (the two buckets run side by side).
template <typename FT, int NT, bool BFOP = false>
__global__ __launch_bounds__(256) void k_localt_mf2(
    const int32_t* __restrict__ subs, const int64_t* __restrict__ sub_ptr,
    const int64_t* __restrict__ roff, const int64_t* __restrict__ fac_off,
    const FT* __restrict__ Lc, const typename AccT<FT>::T* __restrict__ dinv, const double* rin,
    double* out, int mode, const int64_t* __restrict__ isub_ptr,
    const int32_t* __restrict__ isub_list, const int64_t* __restrict__ mbf_off,
    const double* __restrict__ mbf, const double* __restrict__ eta, const double* __restrict__ qv,
    double* __restrict__ partial, unsigned blk_off, PcgShared* sh, int64_t nrows) {
  static_assert(NT == 16, "one 16-column matrix-core tile");
  using AT = typename AccT<FT>::T;
  using V = typename MfAcc<AT>::V;
  constexpr int PITCH = 65;
  constexpr int CH = 64 * PITCH;
  constexpr int NTHR = 256;
  constexpr int WP = 128;
  constexpr int VEC = 16 / (int)sizeof(FT);
  constexpr int NLD = 64 * WP / (VEC * NTHR);
  __shared__ AT tile[2 * CH];
  __shared__ AT vb[3][64 * kMfVP];
  __shared__ AT eta_s[64 * NT];
  __shared__ double dots[4][2 * NT];

  const int s = subs[blockIdx.x];
  const int64_t base = sub_ptr[s];
  const int N = (int)(sub_ptr[s + 1] - base);
  const int64_t ro = roff[s];
  const int NP = (int)(roff[s + 1] - ro);
  const int NB = NP / 64;
  const FT* lc = Lc + fac_off[s];
  const AT* dv = dinv + ro;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane % 16, lk = lane / 16;
  const int64_t i0 = isub_ptr[s];
  const int ns = mode >= 1 ? (int)(isub_ptr[s + 1] - i0) : 0;
  const double* P = mbf + mbf_off[s];
  auto vi = [&](int row, int k) { return vix<NT>(nrows, base + row, k); };

  uint4 pre[NLD];
  auto tile_load = [&](int b) {
    const uint4* src = reinterpret_cast<const uint4*>(lc + (size_t)64 * b * WP);
#pragma unroll
    for (int u = 0; u < NLD; ++u) pre[u] = src[u * NTHR + threadIdx.x];
  };
  auto tile_store = [&]() {
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int e0 = (u * NTHR + (int)threadIdx.x) * VEC;  // column e0 / WP, slots e0 % WP ..
      const int col = e0 / WP, slot = e0 % WP;
      AT* dst = tile + (slot / 64) * CH + col * PITCH + (slot % 64);
      FT v[VEC];
      __builtin_memcpy(v, &pre[u], 16);
#pragma unroll
      for (int t = 0; t < VEC; ++t) dst[t] = (AT)widen_lds(v[t]);
    }
  };
  auto drow = [&](int v) { return 16 * w + MfAcc<AT>::row(lk, v); };
  auto ldr = [&](int row) -> AT { return (row >= 0 && row < N) ? (AT)rin[vi(row, li)] : AT(0); };

  tile_load(0);
  if (mode == 2 && all_done(sh)) return;
  for (int t = threadIdx.x; t < ns * NT; t += NTHR)
    eta_s[t] = (AT)eta[(size_t)isub_list[i0 + t / NT] * NT + (t % NT)];
  tile_store();
  if (1 < NB) tile_load(1);
  // t_0 = r of block 0 (vb[0]); u_1 = r of block 1 (vb[2])
  for (int e = threadIdx.x; e < 64 * NT; e += NTHR) {
    const int row = e / NT, k = e % NT;
    vb[0][row * kMfVP + k] = row < N ? (AT)rin[vi(row, k)] : AT(0);
    vb[2][row * kMfVP + k] = row + 64 < N ? (AT)rin[vi(row + 64, k)] : AT(0);
  }
  __syncthreads();

  // ---- forward sweep: vb[0] = t_b, vb[1] = y_b, vb[2] = u_{b+1} ----
  for (int b = 0; b < NB; ++b) {
    const int j0 = 64 * b;
    const AT* Tb = tile + (b & 1) * CH;        // block b's rows
    const AT* Tn = tile + (1 - (b & 1)) * CH;  // block b + 1's rows
    AT rf[4], dvl[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      rf[v] = ldr(j0 + 128 + drow(v));
      dvl[v] = dv[j0 + drow(v)];
    }
    const int ii = 16 * w + li;
    V acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = vb[0][drow(v) * kMfVP + li];
    acc = mf_pass<BFOP>(
        acc, [&](int c, int m) { const int jj = c + m * lk; return ii > jj ? Tb[jj * PITCH + ii] : AT(0); },
        [&](int c, int m) { const int jj = c + m * lk; return vb[0][jj * kMfVP + li]; });
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      vb[1][drow(v) * kMfVP + li] = acc[v];
      const int row = j0 + drow(v);
      if (row < N) out[vi(row, li)] = (double)(acc[v] * dvl[v]);
    }
    __syncthreads();  // y complete; every wave is done reading t_b
    V an, af;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      an[v] = vb[2][drow(v) * kMfVP + li];
      af[v] = rf[v];
    }
    an = mf_pass<BFOP>(
        an, [&](int c, int m) { const int jj = c + m * lk; return -Tn[jj * PITCH + ii]; },
        [&](int c, int m) { const int jj = c + m * lk; return vb[1][jj * kMfVP + li]; });
    af = mf_pass<BFOP>(
        af, [&](int c, int m) { const int jj = c + m * lk; return ii <= jj ? -Tb[jj * PITCH + ii] : AT(0); },
        [&](int c, int m) { const int jj = c + m * lk; return vb[1][jj * kMfVP + li]; });
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      vb[0][drow(v) * kMfVP + li] = an[v];
      vb[2][drow(v) * kMfVP + li] = af[v];
    }
    __syncthreads();  // every wave is done with tile b and with y_b
    if (b + 1 < NB) {
      tile_store();
      if (b + 2 < NB) tile_load(b + 2);
      __syncthreads();
    }
  }

  // ---- backward sweep: tile NB-1 is still in LDS ----
  if (NB > 1) tile_load(NB - 2);
  int i1 = 0, i2 = 1, is = 2;  // buffers of x_{b+1}, x_{b+2}, s
  for (int e = threadIdx.x; e < 64 * NT; e += NTHR) {
    vb[0][(e / NT) * kMfVP + e % NT] = AT(0);
    vb[1][(e / NT) * kMfVP + e % NT] = AT(0);
  }
  __syncthreads();
  double rz = 0.0, qz = 0.0;  // column li of this lane's rows
  for (int b = NB - 1; b >= 0; --b) {
    const int j0 = 64 * b;
    const AT* Tb = tile + (b & 1) * CH;
    const AT* Tn = tile + (1 - (b & 1)) * CH;
    AT vv[4];
    double rp[4], qp[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = j0 + drow(v);
      const bool ok = row < N;
      vv[v] = ok ? (AT)out[vi(row, li)] : AT(0);
      rp[v] = (ok && mode == 2) ? rin[vi(row, li)] : 0.0;
      qp[v] = (ok && mode == 2) ? qv[vi(row, li)] : 0.0;
    }
    constexpr int NPA = 8;  // slots 0..31 fetched ahead, the rest when used
    const int ra = j0 + 16 * w + li;
    AT pa[NPA];
#pragma unroll
    for (int c = 0; c < NPA; ++c) {
      const int q = 4 * c + lk;
      pa[c] = (q < ns && ra < N) ? (AT)P[(size_t)q * N + ra] : AT(0);
    }
    const int ii = 16 * w + li;  // output row ii (a column of the tile)
    const AT* x1 = vb[i1];
    const AT* x2 = vb[i2];
    V acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = vv[v];
    acc = mf_pass<BFOP>(
        acc, [&](int c, int m) { const int jj = c + m * lk; return -Tn[ii * PITCH + jj]; },
        [&](int c, int m) { const int jj = c + m * lk; return x1[jj * kMfVP + li]; });
    acc = mf_pass<BFOP>(
        acc, [&](int c, int m) { const int jj = c + m * lk; return jj <= ii ? -Tb[ii * PITCH + jj] : AT(0); },
        [&](int c, int m) { const int jj = c + m * lk; return x2[jj * kMfVP + li]; });
    AT* sv = vb[is];
#pragma unroll
    for (int v = 0; v < 4; ++v) sv[drow(v) * kMfVP + li] = acc[v];
    __syncthreads();  // s complete; every wave is done reading x_{b+2}
    acc = mf_pass<BFOP>(
        acc, [&](int c, int m) { const int jj = c + m * lk; return jj > ii ? Tb[ii * PITCH + jj] : AT(0); },
        [&](int c, int m) { const int jj = c + m * lk; return sv[jj * kMfVP + li]; });
    AT* xb = vb[i2];  // x_b over x_{b+2}
#pragma unroll
    for (int v = 0; v < 4; ++v) xb[drow(v) * kMfVP + li] = acc[v];
#pragma unroll
    for (int c = 0; c < NPA; ++c) {
      if (4 * c >= ns) break;  // uniform
      const int q = 4 * c + lk;
      const AT e = q < ns ? eta_s[q * NT + li] : AT(0);
      acc = mf4(pa[c], e, acc);
    }
    for (int c = NPA; 4 * c < ns; ++c) {
      const int q = 4 * c + lk;
      const AT av = (q < ns && ra < N) ? (AT)P[(size_t)q * N + ra] : AT(0);
      const AT e = q < ns ? eta_s[q * NT + li] : AT(0);
      acc = mf4(av, e, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = j0 + drow(v);
      if (row < N) {
        const double zv = (double)acc[v];
        out[vi(row, li)] = zv;
        rz = fma(rp[v], zv, rz);
        qz = fma(qp[v], zv, qz);
      }
    }
    {  // x_b becomes x_{b+1} of the next step, x_{b+1} its x_{b+2}
      const int t1 = i1;
      i1 = i2;
      i2 = t1;
    }
    __syncthreads();  // every wave is done with tile b, s and x_b
    if (b > 0) {
      tile_store();
      if (b - 2 >= 0) tile_load(b - 2);
      __syncthreads();
    }
  }

  if (mode != 2) return;
  rz += __shfl_xor(rz, 16, 64);
  rz += __shfl_xor(rz, 32, 64);
  qz += __shfl_xor(qz, 16, 64);
  qz += __shfl_xor(qz, 32, 64);
  if (lane < 16) {
    dots[w][lane] = rz;
    dots[w][NT + lane] = qz;
  }
  __syncthreads();
  if (threadIdx.x < 2 * NT) {
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) a += dots[u][threadIdx.x];
    partial[(size_t)(blk_off + blockIdx.x) * 2 * NT + threadIdx.x] = a;
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
__global__ __launch_bounds__(256) void k_bpart(int64_t n, const int64_t* __restrict__ sub_ptr,
                                               const int64_t* __restrict__ isub_ptr,
                                               const int64_t* __restrict__ mbf_off,
                                               const double* __restrict__ mbf,
                                               const int64_t* __restrict__ bdst,
                                               const double* __restrict__ r, double* bpart) {
  __shared__ double lds[4 * 16];  // block sums of up to 16 values
  bpart_sub<NR>(blockIdx.x, n, sub_ptr, isub_ptr, mbf_off, mbf, bdst, r, bpart, lds);
}

// ---------------------------------------------------------------------------
// launcher templates (instantiated once per factor precision)

template <typename FT>
hipError_t band_factor_t(DeviceState& d, hipStream_t st) {
  using IT = typename AccT<FT>::T;
  for (int bk = 0; bk < 2; ++bk) {
    const int nb = (int)d.bucket_sub[bk].size();
    if (!nb) continue;
    if (bk == 0)
      hipLaunchKernelGGL((k_band_factor<FT, 64>), dim3(nb), dim3(256), 0, st,
                         d.d_bucket_sub[bk], d.sub_ptr, d.roff, d.fac_off, d.prp, d.pci, d.pv,
                         (FT*)d.Lc, (FT*)d.Lr, (IT*)d.invd, d.fail, d.plain);
    else
      hipLaunchKernelGGL((k_band_factor<FT, 128>), dim3(nb), dim3(256), 0, st,
                         d.d_bucket_sub[bk], d.sub_ptr, d.roff, d.fac_off, d.prp, d.pci, d.pv,
                         (FT*)d.Lc, (FT*)d.Lr, (IT*)d.invd, d.fail, d.plain);
  }
  return hipGetLastError();
}

template <typename FT>
hipError_t mbf_t(DeviceState& d, hipStream_t st) {
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

template <typename FT>
hipError_t invert_diag_t(DeviceState& d, hipStream_t st) {
  for (int bk = 0; bk < 2; ++bk) {
    const int nb = (int)d.bucket_sub[bk].size();
    if (!nb) continue;
    const dim3 grid(nb, (unsigned)((d.max_np + 63) / 64));
    if (bk == 0)
      hipLaunchKernelGGL((k_invert_diag<FT, 1>), grid, dim3(64), 0, st, d.d_bucket_sub[bk], d.roff,
                         d.fac_off, (FT*)d.Lc);
    else
      hipLaunchKernelGGL((k_invert_diag<FT, 2>), grid, dim3(64), 0, st, d.d_bucket_sub[bk], d.roff,
                         d.fac_off, (FT*)d.Lc);
  }
  return hipGetLastError();
}

// Wave layout of the tile kernel for NT right-hand sides: G groups of NT/G
// right-hand sides, each pass split over W waves.
// Wave layouts of the tile kernel (G groups of NT/G right-hand sides, each
// pass split over W waves): the candidates the autotuner times for each
// right-hand-side count, the first being the default.
template <int NT> struct TileCands;
template <> struct TileCands<1> {
  static constexpr int n = 3;
  static constexpr int G[4] = {1, 1, 1, 1}, W[4] = {4, 2, 8, 4};
};
template <> struct TileCands<2> {
  static constexpr int n = 2;
  static constexpr int G[4] = {1, 2, 1, 1}, W[4] = {4, 2, 4, 4};
};
template <> struct TileCands<4> {
  static constexpr int n = 3;
  static constexpr int G[4] = {2, 4, 1, 2}, W[4] = {2, 1, 4, 2};
};
template <> struct TileCands<8> {
  static constexpr int n = 3;
  static constexpr int G[4] = {4, 2, 8, 4}, W[4] = {1, 2, 1, 1};
};
template <> struct TileCands<16> {
  static constexpr int n = 3;
  static constexpr int G[4] = {4, 8, 4, 4}, W[4] = {1, 1, 2, 1};
};

// LDS bytes of k_localt for a shape (the static arrays of the kernel)
template <typename FT, int C, int NT, int G, int W>
constexpr size_t tile_lds_bytes() {
  using AT = typename AccT<FT>::T;
  constexpr int NR = NT / G;
  return 2 * (size_t)C * 64 * LdsPitch<FT>::v * sizeof(FT) +
         2 * (size_t)G * (W > 1 ? W : 1) * C * (W > 1 ? 64 * NR : 1) * sizeof(AT) +
         (size_t)TileMaxNi<NT>::v * NT * 8 + (size_t)G * W * 2 * NR * 8 +
         (size_t)G * 2 * 64 * NR * sizeof(AT) + 64;
}
constexpr size_t kLdsBudget = 160 * 1024;

// The shape a candidate stands for at (FT, C): the candidate where its LDS
// fits, otherwise the default.
template <typename FT, int C, int NT, int I> struct TileAt {
  static constexpr int g0 = TileCands<NT>::G[I], w0 = TileCands<NT>::W[I];
  static constexpr bool fits = tile_lds_bytes<FT, C, NT, g0, w0>() <= kLdsBudget;
  static constexpr int G = fits ? g0 : TileCands<NT>::G[0];
  static constexpr int W = fits ? w0 : TileCands<NT>::W[0];
};

template <typename FT, int NT, int I>
hipError_t localt_shape(DeviceState& d, const double* r, double* z, const double* eta, int mode,
                        int init, hipStream_t st) {
  using IT = typename AccT<FT>::T;
  const int nb0 = (int)d.bucket_sub[0].size(), nb1 = (int)d.bucket_sub[1].size();
  // With both window buckets populated, the window-128 bucket (few, long
  // workgroups) runs on a second stream beside the window-64 one: a fork and
  // a join on events, which graph capture records as two parallel branches.
  // In a profiled solve the operation's two events are recorded on st before
  // the fork and after the join, so they time the pair as it runs.
  const bool fork = nb0 > 0 && nb1 > 0 && d.side;
  auto launch_bucket = [&](int bk, hipStream_t s, bool first, bool last) {
    const int nb = bk == 0 ? nb0 : nb1;
    const unsigned off = bk == 0 ? 0u : (unsigned)nb0;  // rows of the partials
    // bucket 0 lists 0 .. m-1 in order when bucket 1 is empty: the kernel
    // then takes its subdomain from blockIdx.x (one dependent load less)
    const int32_t* subs_arg = (bk == 0 && nb1 == 0) ? nullptr : d.d_bucket_sub[bk];
    auto go = [&](auto kern, int threads) {
      am_launch(d, first, last, kern, dim3(nb), dim3(threads), s,
                subs_arg, d.sub_ptr, d.roff, d.fac_off, (const FT*)d.Lc,
                (const IT*)d.invd, r, z, mode, d.isub_ptr, d.isub_list, d.mbf_off, d.mbf, eta,
                d.q, d.red.pd, off, d.fuse_eta, d.Sinv, (int)d.NL, d.ldS, d.bpart, d.red.pb, d.m,
                init, d.sc, d.shared, d.n);
    };
    // the matrix-core kernels of 16 columns (BF16 x BF16 products on request)
    auto go_mf = [&](auto kern) {
      am_launch(d, first, last, kern, dim3(nb), dim3(256), s, d.d_bucket_sub[bk], d.sub_ptr,
                d.roff, d.fac_off, (const FT*)d.Lc, (const IT*)d.invd, r, z, mode, d.isub_ptr,
                d.isub_list, d.mbf_off, d.mbf, eta, d.q, d.red.pd, off, d.shared, d.n);
    };
    constexpr bool kBf = std::is_same<FT, bf16_t>::value;
    if (bk == 0) {
      using S = TileAt<FT, 1, NT, I>;
      bool mf = false;
      if constexpr (NT == 16) {
        if (!d.fuse_eta) {
          mf = true;
          if (kBf && d.bf16_ops)
            go_mf(k_localt_mf<FT, 16, kBf>);
          else
            go_mf(k_localt_mf<FT, 16, false>);
        }
      }
      // one right-hand side with BF16 x BF16 products: column 0 of the
      // matrix-core tiles, where every subdomain is in the window-64 bucket
      if constexpr (NT == 1 && kBf) {
        if (!d.fuse_eta && d.bf16_ops && nb1 == 0) {
          mf = true;
          go_mf(k_localt_mf<FT, 1, true>);
        }
      }
      if (!mf) go(k_localt<FT, 1, NT, S::G, S::W>, 64 * S::G * S::W);
    } else {
      using S = TileAt<FT, 2, NT, I>;
      bool mf = false;
      if constexpr (NT == 16) {
        if (!d.fuse_eta) {
          mf = true;
          if (kBf && d.bf16_ops)
            go_mf(k_localt_mf2<FT, 16, kBf>);
          else
            go_mf(k_localt_mf2<FT, 16, false>);
        }
      }
      if (!mf) go(k_localt<FT, 2, NT, S::G, S::W>, 64 * S::G * S::W);
    }
  };
  if (fork) {
    const hipEvent_t p0 = d.prof_ev[0], p1 = d.prof_ev[1];
    hipError_t e = hipSuccess;
    if (p0) {
      if ((e = hipEventRecord(p0, st)) != hipSuccess) return e;
      d.prof_used[0] = true;
    }
    d.prof_ev[0] = d.prof_ev[1] = nullptr;  // no events on the launches themselves
    e = hipEventRecord(d.ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(d.side, d.ev_fork, 0);
    if (e == hipSuccess) {
      launch_bucket(1, d.side, false, false);
      e = hipEventRecord(d.ev_join, d.side);
    }
    if (e == hipSuccess) {
      launch_bucket(0, st, false, false);
      e = hipStreamWaitEvent(st, d.ev_join, 0);
    }
    d.prof_ev[0] = p0;
    d.prof_ev[1] = p1;
    if (e != hipSuccess) return e;
    if (p1) {
      if ((e = hipEventRecord(p1, st)) != hipSuccess) return e;
      d.prof_used[1] = true;
    }
  } else {
    if (nb0 > 0) launch_bucket(0, st, true, nb1 == 0);
    if (nb1 > 0) launch_bucket(1, st, nb0 == 0, true);
  }
  return hipGetLastError();
}

template <typename FT, int NT>
hipError_t localt_t(DeviceState& d, const double* r, double* z, const double* eta, int mode,
                    int init, hipStream_t st) {
  int c = d.tile_cand[tile_slot(NT)];
  if (c < 0 || c >= TileCands<NT>::n) c = 0;
  switch (c) {
    case 1: return localt_shape<FT, NT, 1>(d, r, z, eta, mode, init, st);
    case 2:
      if constexpr (TileCands<NT>::n > 2) return localt_shape<FT, NT, 2>(d, r, z, eta, mode, init, st);
      break;
    default: break;
  }
  return localt_shape<FT, NT, 0>(d, r, z, eta, mode, init, st);
}

template <typename FT>
hipError_t local_nr(DeviceState& d, const double* r, double* z, const double* eta, int nrhs,
                    int mode, int init, hipStream_t st) {
  switch (nrhs) {
    case 1: return localt_t<FT, 1>(d, r, z, eta, mode, init, st);
    case 2: return localt_t<FT, 2>(d, r, z, eta, mode, init, st);
    case 4: return localt_t<FT, 4>(d, r, z, eta, mode, init, st);
    case 8: return localt_t<FT, 8>(d, r, z, eta, mode, init, st);
    case 16: return localt_t<FT, 16>(d, r, z, eta, mode, init, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace am
