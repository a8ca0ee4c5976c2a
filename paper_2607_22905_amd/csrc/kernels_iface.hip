// Interface kernels for gfx950: assembly of the interface matrix
//   S[n, m] = -delta_nm sum_{e in E_n} a_e + sum_{e in E_n} a_e (phat^(m)_k + phat^(m)_l)/2
// (eq. interface-problem-alg with the sign of Corollary eq. k-schur), its
// symmetrisation, an FP64 tiled Cholesky S = L L^T followed by the explicit
// inverse S^{-1} = L^{-T} L^{-1}, and the per-apply interface solve
// eta = S^{-1} b as a dense GEMV/GEMM (Algorithm 2).
//
// Dense tiles are 64 x 64, row-major with leading dimension ldS (a multiple
// of 64); rows/columns beyond N_Lambda hold the identity.
#include <algorithm>

#include "am_common.h"

namespace am {

// ---------------------------------------------------------------------------
// One wave per interface row n.  Every write to row n comes from lane 0 of
// that wave, in a fixed order.
__global__ __launch_bounds__(256) void k_assemble_S(
    int NL, int ldS, const int64_t* __restrict__ iface_ptr, const int32_t* __restrict__ iface_ij,
    const int32_t* __restrict__ e_kloc, const int32_t* __restrict__ e_lloc,
    const double* __restrict__ e_a, const int64_t* __restrict__ sub_ptr,
    const int64_t* __restrict__ isub_ptr, const int32_t* __restrict__ isub_list,
    const int64_t* __restrict__ mbf_off, const double* __restrict__ mbf, double* S) {
  const int lane = threadIdx.x & 63;
  const int n = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= NL) return;
  const int i = iface_ij[2 * n], j = iface_ij[2 * n + 1];
  const int64_t e0 = iface_ptr[n], e1 = iface_ptr[n + 1];
  double sa = 0.0;
  for (int64_t e = e0 + lane; e < e1; e += 64) sa += e_a[e];
  sa = wave_sum(sa);
  double* Srow = S + (size_t)n * ldS;
  for (int side = 0; side < 2; ++side) {
    const int sd = side == 0 ? i : j;
    const int Ns = (int)(sub_ptr[sd + 1] - sub_ptr[sd]);
    const double* P = mbf + mbf_off[sd];
    const int32_t* loc = side == 0 ? e_kloc : e_lloc;
    const int64_t q0 = isub_ptr[sd];
    const int nq = (int)(isub_ptr[sd + 1] - q0);
    for (int q = 0; q < nq; ++q) {
      const int m = isub_list[q0 + q];
      double v = 0.0;
      for (int64_t e = e0 + lane; e < e1; e += 64) v = fma(e_a[e], P[(size_t)q * Ns + loc[e]], v);
      v = wave_sum(v);
      if (lane == 0) Srow[m] += 0.5 * v;
    }
  }
  if (lane == 0) Srow[n] -= sa;
}

// (S + S^T)/2 on the N_Lambda block; identity on the padding.
__global__ __launch_bounds__(256) void k_symmetrize(int NL, int ldS, double* S) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)ldS * ldS;
  if (t >= tot) return;
  const int r = (int)(t / ldS), c = (int)(t % ldS);
  if (r >= NL || c >= NL) {
    if (r == c) S[t] = 1.0;
    return;
  }
  if (r <= c) return;
  const double v = 0.5 * (S[(size_t)r * ldS + c] + S[(size_t)c * ldS + r]);
  S[(size_t)r * ldS + c] = v;
  S[(size_t)c * ldS + r] = v;
}

// ---------------------------------------------------------------------------
// dense tile helpers (64 x 64, 256 threads, 4 x 4 outputs per thread)
typedef double Tile[64][65];

__device__ __forceinline__ void load_tile(Tile& T, const double* p, int ld, bool trans) {
  for (int t = threadIdx.x; t < 4096; t += blockDim.x) {
    const int r = t >> 6, c = t & 63;
    if (trans)
      T[c][r] = p[(size_t)r * ld + c];
    else
      T[r][c] = p[(size_t)r * ld + c];
  }
}

// A tile through registers, for 256-thread workgroups: tile_fetch issues all
// 16 loads of the thread before any is used (one memory round trip per tile
// instead of one per row of threads), tile_put stores them to LDS.
struct TileRegs {
  double v[16];
};

__device__ __forceinline__ void tile_fetch(TileRegs& R, const double* p, int ld) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int r = (threadIdx.x >> 6) + 4 * u, c = threadIdx.x & 63;
    R.v[u] = p[(size_t)r * ld + c];
  }
}

__device__ __forceinline__ void tile_put(Tile& T, const TileRegs& R, bool trans) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int r = (threadIdx.x >> 6) + 4 * u, c = threadIdx.x & 63;
    if (trans)
      T[c][r] = R.v[u];
    else
      T[r][c] = R.v[u];
  }
}

// acc += A * B for two 64 x 64 tiles on the FP64 matrix cores: wave w owns
// rows 16 w .. 16 w + 15 and keeps four 16 x 16 accumulators (columns 16 t ..);
// v_mfma_f64_16x16x4_f64 lane l holds A[l % 16][l / 16], B[l / 16][l % 16]
// and D[l / 16 + 4 v][l % 16], v < 4.
typedef double am_d4 __attribute__((ext_vector_type(4)));
struct MfAcc {
  am_d4 t[4];
};

__device__ __forceinline__ void mf_zero(MfAcc& acc) {
#pragma unroll
  for (int t = 0; t < 4; ++t) acc.t[t] = am_d4{0.0, 0.0, 0.0, 0.0};
}

// 256 threads = 4 waves
__device__ __forceinline__ void mf_mac(MfAcc& acc, const Tile& A, const Tile& B) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane % 16, lk = lane / 16;
#pragma unroll 4
  for (int ks = 0; ks < 16; ++ks) {
    const double a = A[16 * w + li][4 * ks + lk];
#pragma unroll
    for (int t = 0; t < 4; ++t)
      acc.t[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, B[4 * ks + lk][16 * t + li], acc.t[t], 0, 0, 0);
  }
}

// calls f(row, col, value) for the thread's 16 entries of the tile
template <typename F>
__device__ __forceinline__ void mf_each(const MfAcc& acc, F&& f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane % 16, lk = lane / 16;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) f(16 * w + lk + 4 * v, 16 * t + li, acc.t[t][v]);
}

// Cholesky of the diagonal tile (b, b), in place (lower; upper zeroed), by
// symmetric elimination on unscaled columns: step k takes the pivot
// d_k = a_kk and updates a_ij -= a_ik (a_jk / d_k) for k < j <= i.  Thread
// (column j = tid % 64, rows tid / 64 + 4 u) keeps its 16 entries in
// registers for the whole factorization; the owners of column k + 1 publish
// it (after their step-k update) to one of two LDS column buffers, so each
// step is one barrier.  At the end l_jj = sqrt(d_j) and l_ij = a_ij / l_jj.
// A pivot <= 0 is recorded in fail (and taken as 1).
__global__ __launch_bounds__(256) void k_potrf_diag(double* A, int ld, int b, int32_t* fail) {
  __shared__ double col[2][64];
  __shared__ double sq[64];
  const int tid = threadIdx.x, jj = tid & 63, r0 = tid >> 6;
  double* p = A + (size_t)b * 64 * ld + (size_t)b * 64;
  double v[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) v[u] = p[(size_t)(r0 + 4 * u) * ld + jj];
  if (jj == 0)
#pragma unroll
    for (int u = 0; u < 16; ++u) col[0][r0 + 4 * u] = v[u];
  __syncthreads();
  for (int k = 0; k < 64; ++k) {
    const double* ck = col[k & 1];
    double d = ck[k];
    if (!(d > 0.0)) {
      d = 1.0;
      if (tid == 0 && atomicCAS(fail, -1, b * 64 + k) == -1) fail[1] = b * 64 + k;
    }
    if (tid == 0) sq[k] = sqrt(d);
    const double ajk = ck[jj] * (1.0 / d);  // a_jk / d_k for this thread's column
    if (jj > k)
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = r0 + 4 * u;
        if (i >= jj) v[u] -= ck[i] * ajk;
      }
    if (jj == k + 1)
#pragma unroll
      for (int u = 0; u < 16; ++u) col[(k + 1) & 1][r0 + 4 * u] = v[u];
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int i = r0 + 4 * u;
    p[(size_t)i * ld + jj] = jj < i ? v[u] / sq[jj] : (jj == i ? sq[jj] : 0.0);
  }
}

// Panel: A_ib <- A_ib L_bb^{-T} for i = b+1.. (one tile per workgroup):
// X L^T = A by columns, x_j = (a_j - sum_{c < j} x_c l_jc) (1 / l_jj) with
// the terms in increasing c.  Thread (column j = tid % 64, rows tid / 64 + 4 u)
// keeps its 16 entries in registers; finished column c goes to one of two
// LDS buffers for the others, so each step is one barrier.
__global__ __launch_bounds__(256) void k_trsm_panel(double* A, int ld, int b) {
  __shared__ Tile L;
  __shared__ double col[2][64];
  const int i = b + 1 + blockIdx.x;
  const int tid = threadIdx.x, jj = tid & 63, r0 = tid >> 6;
  const double* pl = A + (size_t)b * 64 * ld + (size_t)b * 64;
  double* pa = A + (size_t)i * 64 * ld + (size_t)b * 64;
  {
    TileRegs rl;
    tile_fetch(rl, pl, ld);
    tile_put(L, rl, false);
  }
  double v[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) v[u] = pa[(size_t)(r0 + 4 * u) * ld + jj];
  __syncthreads();
  const double rjj = 1.0 / L[jj][jj];
  if (jj == 0)
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      v[u] *= rjj;
      col[0][r0 + 4 * u] = v[u];
    }
  __syncthreads();
  for (int c = 0; c < 63; ++c) {
    const double* xc = col[c & 1];
    const double ljc = L[jj][c];
    if (jj > c)
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] -= xc[r0 + 4 * u] * ljc;
    if (jj == c + 1)
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        v[u] *= rjj;
        col[(c + 1) & 1][r0 + 4 * u] = v[u];
      }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) pa[(size_t)(r0 + 4 * u) * ld + jj] = v[u];
}

// Trailing update A_ij -= A_ib A_jb^T for b < j <= i.
__global__ __launch_bounds__(256) void k_syrk_update(double* A, int ld, int b) {
  const int j = b + 1 + blockIdx.x, i = b + 1 + blockIdx.y;
  if (j > i) return;
  __shared__ Tile Ai;
  __shared__ Tile Bj;
  TileRegs ra, rb;
  tile_fetch(ra, A + (size_t)i * 64 * ld + (size_t)b * 64, ld);
  tile_fetch(rb, A + (size_t)j * 64 * ld + (size_t)b * 64, ld);
  tile_put(Ai, ra, false);
  tile_put(Bj, rb, true);
  __syncthreads();
  MfAcc acc;
  mf_zero(acc);
  mf_mac(acc, Ai, Bj);
  double* pc = A + (size_t)i * 64 * ld + (size_t)j * 64;
  mf_each(acc, [&](int r, int c, double v) { pc[(size_t)r * ld + c] -= v; });
}

// Inverse of each diagonal tile of L (lower), one column per thread.
__global__ __launch_bounds__(64) void k_trtri_diag(const double* L, double* Li, int ld) {
  __shared__ Tile T;
  __shared__ Tile X;
  const int b = blockIdx.x;
  load_tile(T, L + (size_t)b * 64 * ld + (size_t)b * 64, ld, false);
  __syncthreads();
  const int c = threadIdx.x;
  for (int r = 0; r < 64; ++r) {
    double v = (r == c) ? 1.0 : 0.0;
    if (r < c) {
      X[r][c] = 0.0;
      continue;
    }
    for (int k = c; k < r; ++k) v -= T[r][k] * X[k][c];
    X[r][c] = v / T[r][r];
  }
  __syncthreads();
  double* p = Li + (size_t)b * 64 * ld + (size_t)b * 64;
  for (int t = threadIdx.x; t < 4096; t += blockDim.x) {
    const int r = t >> 6, cc = t & 63;
    p[(size_t)r * ld + cc] = X[r][cc];
  }
}

// Trailing update with two panels, A_ij -= A_ib A_jb^T + A_i,b+1 A_j,b+1^T
// for b+2 <= j <= i: one read-modify-write of the output tile for two
// panels (the second pair of tiles is fetched while the first is multiplied).
__global__ __launch_bounds__(256) void k_syrk_update2(double* A, int ld, int b) {
  const int j = b + 2 + blockIdx.x, i = b + 2 + blockIdx.y;
  if (j > i) return;
  __shared__ Tile Ai;
  __shared__ Tile Bj;
  TileRegs ra, rb;
  tile_fetch(ra, A + (size_t)i * 64 * ld + (size_t)b * 64, ld);
  tile_fetch(rb, A + (size_t)j * 64 * ld + (size_t)b * 64, ld);
  tile_put(Ai, ra, false);
  tile_put(Bj, rb, true);
  __syncthreads();
  tile_fetch(ra, A + (size_t)i * 64 * ld + (size_t)(b + 1) * 64, ld);
  tile_fetch(rb, A + (size_t)j * 64 * ld + (size_t)(b + 1) * 64, ld);
  MfAcc acc;
  mf_zero(acc);
  mf_mac(acc, Ai, Bj);
  __syncthreads();
  tile_put(Ai, ra, false);
  tile_put(Bj, rb, true);
  __syncthreads();
  mf_mac(acc, Ai, Bj);
  double* pc = A + (size_t)i * 64 * ld + (size_t)j * 64;
  mf_each(acc, [&](int r, int c, double v) { pc[(size_t)r * ld + c] -= v; });
}

// Off-diagonal tiles of L^{-1} at distance d: Li_ij = -Li_ii sum_{k=j}^{i-1} L_ik Li_kj.
__global__ __launch_bounds__(256) void k_trtri_off(const double* L, double* Li, int ld, int d) {
  const int i = d + blockIdx.x, j = blockIdx.x;
  __shared__ Tile As;
  __shared__ Tile Bs;
  MfAcc acc;
  mf_zero(acc);
  // the tiles of step k + 1 are in flight while step k runs on the matrix cores
  TileRegs ra, rb;
  tile_fetch(ra, L + (size_t)i * 64 * ld + (size_t)j * 64, ld);
  tile_fetch(rb, Li + (size_t)j * 64 * ld + (size_t)j * 64, ld);
  for (int k = j; k < i; ++k) {
    tile_put(As, ra, false);
    tile_put(Bs, rb, false);
    __syncthreads();
    if (k + 1 < i) {
      tile_fetch(ra, L + (size_t)i * 64 * ld + (size_t)(k + 1) * 64, ld);
      tile_fetch(rb, Li + (size_t)(k + 1) * 64 * ld + (size_t)j * 64, ld);
    } else {
      tile_fetch(ra, Li + (size_t)i * 64 * ld + (size_t)i * 64, ld);
    }
    mf_mac(acc, As, Bs);
    __syncthreads();
  }
  mf_each(acc, [&](int r, int c, double v) { Bs[r][c] = v; });
  tile_put(As, ra, false);
  __syncthreads();
  mf_zero(acc);
  mf_mac(acc, As, Bs);
  double* p = Li + (size_t)i * 64 * ld + (size_t)j * 64;
  mf_each(acc, [&](int r, int c, double v) { p[(size_t)r * ld + c] = -v; });
}

// The sum of k_trtri_off split over nchunk workgroups per tile, for the
// launches with few tiles: workgroup (j, c) forms the share
//   part[j nchunk + c] = sum_{k = k0}^{k1 - 1} L_ik Li_kj,
// k0 = j + c d / nchunk, k1 = j + (c + 1) d / nchunk, as a row-major 64 x 64
// block (nchunk <= d, so no share is empty).
__global__ __launch_bounds__(256) void k_trtri_part(const double* L, const double* Li, int ld,
                                                    int d, int nchunk, double* part) {
  const int j = blockIdx.x / nchunk, c = blockIdx.x % nchunk, i = j + d;
  const int k0 = j + (int)((int64_t)c * d / nchunk);
  const int k1 = j + (int)((int64_t)(c + 1) * d / nchunk);
  __shared__ Tile As;
  __shared__ Tile Bs;
  MfAcc acc;
  mf_zero(acc);
  TileRegs ra, rb;
  tile_fetch(ra, L + (size_t)i * 64 * ld + (size_t)k0 * 64, ld);
  tile_fetch(rb, Li + (size_t)k0 * 64 * ld + (size_t)j * 64, ld);
  for (int k = k0; k < k1; ++k) {
    tile_put(As, ra, false);
    tile_put(Bs, rb, false);
    __syncthreads();
    if (k + 1 < k1) {
      tile_fetch(ra, L + (size_t)i * 64 * ld + (size_t)(k + 1) * 64, ld);
      tile_fetch(rb, Li + (size_t)(k + 1) * 64 * ld + (size_t)j * 64, ld);
    }
    mf_mac(acc, As, Bs);
    __syncthreads();
  }
  double* p = part + (size_t)blockIdx.x * 4096;
  mf_each(acc, [&](int r, int cc, double v) { p[r * 64 + cc] = v; });
}

// Li_ij = -Li_ii sum_c part[j nchunk + c], the shares added in order c = 0, 1, ..
__global__ __launch_bounds__(256) void k_trtri_fin(double* Li, int ld, int d, int nchunk,
                                                   const double* part) {
  const int j = blockIdx.x, i = j + d;
  __shared__ Tile As;
  __shared__ Tile Bs;
  TileRegs sum, t;
  tile_fetch(sum, part + (size_t)j * nchunk * 4096, 64);
  for (int c = 1; c < nchunk; ++c) {
    tile_fetch(t, part + ((size_t)j * nchunk + c) * 4096, 64);
#pragma unroll
    for (int u = 0; u < 16; ++u) sum.v[u] += t.v[u];
  }
  tile_put(Bs, sum, false);
  tile_fetch(t, Li + (size_t)i * 64 * ld + (size_t)i * 64, ld);
  tile_put(As, t, false);
  __syncthreads();
  MfAcc acc;
  mf_zero(acc);
  mf_mac(acc, As, Bs);
  double* p = Li + (size_t)i * 64 * ld + (size_t)j * 64;
  mf_each(acc, [&](int r, int c, double v) { p[(size_t)r * ld + c] = -v; });
}

// S^{-1}_ij = sum_{k >= max(i,j)} Li_ki^T Li_kj for i >= j, mirrored.
__global__ __launch_bounds__(256) void k_lauum(const double* Li, double* Sinv, int ld, int T) {
  const int j = blockIdx.x, i = blockIdx.y;
  if (j > i) return;
  __shared__ Tile As;
  __shared__ Tile Bs;
  MfAcc acc;
  mf_zero(acc);
  // the tiles of step k + 1 are in flight while step k runs on the matrix cores
  TileRegs ra, rb;
  tile_fetch(ra, Li + (size_t)i * 64 * ld + (size_t)i * 64, ld);
  tile_fetch(rb, Li + (size_t)i * 64 * ld + (size_t)j * 64, ld);
  for (int k = i; k < T; ++k) {
    tile_put(As, ra, true);
    tile_put(Bs, rb, false);
    __syncthreads();
    if (k + 1 < T) {
      tile_fetch(ra, Li + (size_t)(k + 1) * 64 * ld + (size_t)i * 64, ld);
      tile_fetch(rb, Li + (size_t)(k + 1) * 64 * ld + (size_t)j * 64, ld);
    }
    mf_mac(acc, As, Bs);
    __syncthreads();
  }
  mf_each(acc, [&](int r, int c, double v) {
    const size_t gr = (size_t)i * 64 + r, gc = (size_t)j * 64 + c;
    if (gr < gc) return;  // diagonal tile: the lower half defines both halves
    Sinv[gr * ld + gc] = v;
    Sinv[gc * ld + gr] = v;
  });
}

// ---------------------------------------------------------------------------
// eta = S^{-1} b, b_m = bpart[2m] + bpart[2m+1], as a sum of outer products
// over the rows of the symmetric S^{-1}: eta[r] = sum_m S^{-1}[m][r] b_m.
// Wave (rb, p) takes the 64 entries r = 64 rb + lane and the rows m of part
// p: each row is one coalesced 64-value load and NR FMAs with b_m, a uniform
// (scalar) load, so S^{-1} is read exactly once per product.  The loads are
// non-temporal: S^{-1} is streamed once per product and would otherwise evict
// the vectors and the SpMV arrays from L2 and the Infinity Cache.  The part
// sums go to ypart[p][r][k]; k_iface_reduce adds them in part order.
template <int NR>
__global__ __launch_bounds__(256) void k_iface_op(int NL, int ldS, const double* __restrict__ Sinv,
                                                  const double* __restrict__ bpart,
                                                  double* __restrict__ ypart, int P, int pcg,
                                                  int init, const PcgShared* sh) {
  if (pcg && !init && all_done(sh)) return;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  const int nrb = (NL + 63) / 64;
  if (wv >= nrb * P) return;
  const int rb = wv % nrb, p = wv / nrb;
  const int per = (NL + P - 1) / P;
  const int mb = p * per, me = min(NL, mb + per);
  const int r = rb * 64 + lane;  // < ldS (padded to 64)
  const double* col = Sinv + r;
  double acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = 0.0;
#pragma unroll 8
  for (int m = mb; m < me; ++m) {
    const double sv = __builtin_nontemporal_load(col + (size_t)m * ldS);
#pragma unroll
    for (int k = 0; k < NR; ++k)
      acc[k] = fma(sv, bpart[(size_t)(2 * m) * NR + k] + bpart[(size_t)(2 * m + 1) * NR + k], acc[k]);
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) ypart[((size_t)p * ldS + r) * NR + k] = acc[k];
}

// The same product for 4 to 16 right-hand sides on the FP64 matrix cores:
// wave (rb, p) accumulates the 64 x NR block ypart[p][64 rb ..][.] as four
// 16 x 16 tiles, D += A B with A = S^{-1}[m0 .. m0+3][16 rows] (symmetric,
// so the rows m of S^{-1} stand for its columns) and B = b[m0 .. m0+3][NR
// columns, zero-padded to 16].  v_mfma_f64_16x16x4_f64 lane l holds
// A[l % 16][l / 16], B[l / 16][l % 16] and D[l / 16 + 4 v][l % 16], v < 4.
// S^{-1} is read once (four coalesced 128-byte rows per load, non-temporal
// as in k_iface_op); the FMAs run on the matrix cores, so 16 right-hand sides
// cost no more issue slots than 4.
template <int NR>
__global__ __launch_bounds__(256) void k_iface_op_mfma(int NL, int ldS, const double* __restrict__ Sinv,
                                                       const double* __restrict__ bpart,
                                                       double* __restrict__ ypart, int P, int pcg,
                                                       int init, const PcgShared* sh) {
  static_assert(NR >= 1 && NR <= 16, "one 16-column tile");
  if (pcg && !init && all_done(sh)) return;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  const int nrb = (NL + 63) / 64;
  if (wv >= nrb * P) return;
  const int rb = wv % nrb, p = wv / nrb;
  const int per = (NL + P - 1) / P;
  const int mb = p * per, me = min(NL, mb + per);
  const int li = lane % 16, lk = lane / 16;
  const double* col = Sinv + 64 * rb + li;  // column 64 rb + 16 sub + li of row m
  am_d4 acc[4];
#pragma unroll
  for (int sub = 0; sub < 4; ++sub) acc[sub] = am_d4{0.0, 0.0, 0.0, 0.0};
  // U chunks of 4 rows per step, every load of the step issued before its
  // products.  U = 2 leaves room for five waves per SIMD: the loads wait on
  // memory far longer than the products take, and more waves hide more of
  // it than more loads per wave (at 16 RHS on 14,616 rows: 396 us against
  // 435 with U = 4 and 419 with U = 1)
  constexpr int U = 2;
  for (int m0 = mb; m0 < me; m0 += 4 * U) {
    double av[U][4], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = m0 + 4 * u + lk;
      const bool ok = m < me;
      bv[u] = (ok && li < NR)
                  ? bpart[(size_t)(2 * m) * NR + li] + bpart[(size_t)(2 * m + 1) * NR + li]
                  : 0.0;
#pragma unroll
      for (int sub = 0; sub < 4; ++sub) av[u][sub] = ok ? __builtin_nontemporal_load(col + (size_t)m * ldS + 16 * sub) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int sub = 0; sub < 4; ++sub)
        acc[sub] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][sub], bv[u], acc[sub], 0, 0, 0);
  }
  if (li < NR)
#pragma unroll
    for (int sub = 0; sub < 4; ++sub)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 64 * rb + 16 * sub + lk + 4 * v;
        ypart[((size_t)p * ldS + r) * NR + li] = acc[sub][v];
      }
}

// eta[r][k] = sum_p ypart[p][r][k] in part order.  In PCG mode workgroup 0
// first folds the ||r||^2 partials of the update launch and applies the stop
// test ||r|| <= tol ||b|| (the next launches read its outcome).
template <int NR>
__global__ __launch_bounds__(256) void k_iface_reduce(int NL, int ldS, const double* __restrict__ ypart,
                                                      int P, double* __restrict__ eta, int pcg,
                                                      int init, const double* __restrict__ pb,
                                                      int npb, PcgScalars* sc, PcgShared* sh) {
  __shared__ double lds[4 * NR];
  if (pcg && !init && all_done(sh)) return;
  if (pcg && blockIdx.x == 0) {
    const int nrhs = sh->nrhs, maxit = sh->maxit;
    double rr[NR];
    reduce_partials<NR>(rr, pb, (unsigned)npb, lds);
    int alld = 1;
    for (int k = 0; k < nrhs; ++k) {
      const PcgScalars S = sc[k];
      int done = S.done, conv = S.conv, status = S.status;
      double bb = S.bb;
      if (!done) {
        if (init) {
          bb = rr[k];
          if (bb == 0.0) done = conv = 1;
        } else if (rr[k] <= S.tol2 * S.bb) {
          done = conv = 1;
        } else if (S.it >= maxit) {
          done = 1;
          status = AM_ERR_NO_CONVERGENCE;
        }
      }
      alld &= done;
      if (threadIdx.x == 0) {
        sc[k].rr = rr[k];
        sc[k].bb = bb;
        sc[k].done = done;
        sc[k].conv = conv;
        sc[k].status = status;
      }
    }
    if (threadIdx.x == 0) sh->all_done = alld;
  }
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)NL * NR) return;
  const int64_t r = t / NR;
  const int k = (int)(t % NR);
  double e = 0.0;
  for (int p = 0; p < P; ++p) e += ypart[((size_t)p * ldS + r) * NR + k];
  eta[r * NR + k] = e;
}

// ---------------------------------------------------------------------------
hipError_t launch_assemble_S(DeviceState& d, hipStream_t st) {
  if (d.NL == 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(d.S, 0, sizeof(double) * (size_t)d.ldS * d.ldS, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_assemble_S, dim3((unsigned)((d.NL + 3) / 4)), dim3(256), 0, st, (int)d.NL,
                     d.ldS, d.iface_ptr, d.iface_ij, d.e_kloc, d.e_lloc, d.e_a, d.sub_ptr,
                     d.isub_ptr, d.isub_list, d.mbf_off, d.mbf, d.S);
  const int64_t tot = (int64_t)d.ldS * d.ldS;
  hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     (int)d.NL, d.ldS, d.S);
  return hipGetLastError();
}

// Shares per tile of the distance-d launch of the triangular inverse: enough
// workgroups for two per CU, at most 16 shares, none empty.
int trtri_chunks(int T, int d) {
  const int nb = T - d;
  return std::max(1, std::min(std::min(16, d), 512 / nb));
}

// Scratch tiles the split launches need (0 if none is split).
int64_t trtri_part_tiles(int T) {
  int64_t mx = 0;
  for (int dd = 1; dd < T; ++dd) {
    const int c = trtri_chunks(T, dd);
    if (c > 1) mx = std::max<int64_t>(mx, (int64_t)(T - dd) * c);
  }
  return mx;
}

hipError_t dense_cholesky_inverse(DeviceState& d, double* L, double* Li, double* part,
                                  hipStream_t st) {
  const int ld = d.ldS, T = ld / 64;
  if (T == 0) return hipSuccess;
  hipError_t e = hipMemcpyAsync(L, d.S, sizeof(double) * (size_t)ld * ld, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(Li, 0, sizeof(double) * (size_t)ld * ld, st);
  if (e != hipSuccess) return e;
  // right-looking tiled Cholesky with a look-ahead of one panel: after panel
  // b, only column b+1 is updated; panel b+1 is factored; then panels b and
  // b+1 update the rest of the trailing matrix together
  for (int b = 0; b < T;) {
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, st, L, ld, b, d.fail + 2);
    if (b + 1 == T) break;
    hipLaunchKernelGGL(k_trsm_panel, dim3(T - b - 1), dim3(256), 0, st, L, ld, b);
    if (b + 2 == T) {  // one tile left
      hipLaunchKernelGGL(k_syrk_update, dim3(1, 1), dim3(256), 0, st, L, ld, b);
      b += 1;
      continue;
    }
    hipLaunchKernelGGL(k_syrk_update, dim3(1, T - b - 1), dim3(256), 0, st, L, ld, b);
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, st, L, ld, b + 1, d.fail + 2);
    hipLaunchKernelGGL(k_trsm_panel, dim3(T - b - 2), dim3(256), 0, st, L, ld, b + 1);
    hipLaunchKernelGGL(k_syrk_update2, dim3(T - b - 2, T - b - 2), dim3(256), 0, st, L, ld, b);
    b += 2;
  }
  hipLaunchKernelGGL(k_trtri_diag, dim3(T), dim3(64), 0, st, L, Li, ld);
  for (int dd = 1; dd < T; ++dd) {
    const int c = trtri_chunks(T, dd);
    if (c == 1) {
      hipLaunchKernelGGL(k_trtri_off, dim3(T - dd), dim3(256), 0, st, L, Li, ld, dd);
    } else {
      hipLaunchKernelGGL(k_trtri_part, dim3((T - dd) * c), dim3(256), 0, st, L, Li, ld, dd, c, part);
      hipLaunchKernelGGL(k_trtri_fin, dim3(T - dd), dim3(256), 0, st, Li, ld, dd, c, part);
    }
  }
  hipLaunchKernelGGL(k_lauum, dim3(T, T), dim3(256), 0, st, Li, d.Sinv, ld, T);
  return hipGetLastError();
}

hipError_t launch_lauum(const double* Li, double* out, int ld, int T, hipStream_t st) {
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lauum, dim3(T, T), dim3(256), 0, st, Li, out, ld, T);
  return hipGetLastError();
}

template <int NR>
static void gemv_t(DeviceState& d, hipStream_t st, int pcg, int init) {
  const int nrb = (int)((d.NL + 63) / 64);
  const unsigned nw = (unsigned)std::max(1, nrb * d.op_parts);
  if constexpr (NR >= 4)
    am_launch(d, true, false, k_iface_op_mfma<NR>, dim3((nw + 3) / 4), dim3(256), st, (int)d.NL,
              d.ldS, d.Sinv, d.bpart, d.ypart, d.op_parts, pcg, init, d.shared);
  else
    am_launch(d, true, false, k_iface_op<NR>, dim3((nw + 3) / 4), dim3(256), st, (int)d.NL, d.ldS,
              d.Sinv, d.bpart, d.ypart, d.op_parts, pcg, init, d.shared);
  const unsigned nb = (unsigned)std::max<int64_t>(1, (d.NL * NR + 255) / 256);
  am_launch(d, false, true, k_iface_reduce<NR>, dim3(nb), dim3(256), st, (int)d.NL, d.ldS, d.ypart,
            d.op_parts, d.eta, pcg, init, d.red.pb, d.m, d.sc, d.shared);
}

hipError_t launch_iface_gemv(DeviceState& d, int nr, int pcg, int init, hipStream_t st) {
  if (d.NL == 0 && !pcg) return hipSuccess;
  if (d.nd.on) return launch_nd_solve(d, nr, pcg, init, st);
  if (d.ix.on) return launch_ix_solve(d, nr, pcg, init, st);
  // the part sums exist only on handles whose interface solve is not fused
  // into the local kernel (with no interface, the launches only take the
  // stop decision and touch no part sums)
  if (d.NL > 0 && (d.ypart == nullptr || d.op_parts < 1 || nr > d.max_nrhs))
    return hipErrorInvalidValue;
  switch (nr) {
    case 1: gemv_t<1>(d, st, pcg, init); break;
    case 2: gemv_t<2>(d, st, pcg, init); break;
    case 4: gemv_t<4>(d, st, pcg, init); break;
    case 8: gemv_t<8>(d, st, pcg, init); break;
    case 16: gemv_t<16>(d, st, pcg, init); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace am
