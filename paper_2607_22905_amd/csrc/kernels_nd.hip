// Nested-dissection interface solve eta = S^{-1} b for gfx950 (the interface
// solve of Algorithm 2; S is SPD, Corollary cor-schur-eta).
//
// The host layout (iface_nd.cpp) orders the basis functions so that the
// first rows form mutually uncoupled diagonal blocks B of S and the last ones
// are the separators T above them.  Block elimination then gives
//   y_B   = S_BB^{-1} b_B                          k_nd_blocks, pass 0
//   eta_T = C^{-1} (b_T - S_TB y_B)                 k_nd_top (row parts), k_nd_fold
//   eta_B = S_BB^{-1} (b_B - S_BT eta_T)            k_nd_blocks, pass 1
// where C = S_TT - S_TB S_BB^{-1} S_BT.  Every S_bb^{-1} and C^{-1} is held
// explicitly (dense, exactly symmetric), so each step is a set of matrix
// products with no dependent chain inside a launch.  In this order C^{-1} is
// the T block of S^{-1}, and S_bb^{-1} = L_bb^{-T} L_bb^{-1} with L the
// Cholesky factor of the reordered S (the blocks of L over B are those of
// the uncoupled blocks).  Set-up therefore runs the tiled dense Cholesky and
// triangular inverse of kernels_iface.hip once on the reordered S, padded
// so that every block starts on a 64-row tile, and forms the block products
// L_bb^{-T} L_bb^{-1} with the same tile kernel.
//
// Right-hand sides b_n = bpart[2n] + bpart[2n+1] (interface slots, see
// bpart_sub); eta is written in the original basis-function order, [n][NR].
#include <algorithm>

#include "am_common.h"
#include "iface_products.h"

namespace am {

// rows of a block (and of a part of the top rows) whose right-hand side a
// workgroup keeps in LDS: at most 64 KB
template <int NR> struct NdCap {
  static constexpr int rows = (7936 / NR) < 4096 ? 7936 / NR : 4096;
};

int64_t nd_max_rows(int nr_max) {
  switch (nr_max) {
    case 1: return NdCap<1>::rows;
    case 2: return NdCap<2>::rows;
    case 4: return NdCap<4>::rows;
    case 8: return NdCap<8>::rows;
    default: return NdCap<16>::rows;
  }
}

// Workgroup (block b, rows row0 .. row0 + 63 of it): the block's right-hand
// side goes to LDS, then out = Sbb^{-1} rhs for those 64 rows, the eight
// waves taking an eighth of the block's columns each (nd_wave_product); their
// partial sums are added in wave order.  Pass 0 writes y_B (ND order), pass 1
// subtracts S_BT eta_T from the right-hand side first (or, with from_y1,
// takes that right-hand side from y1, where k_nd_rb formed it) and writes
// eta_B in the original order.  Dynamic LDS: max(rows of the largest block,
// 512) NR doubles.
template <int NR> struct NdWaves { static constexpr int v = 8; };

// x - sum_{q in [qb, qe)} val[q] vec[pos[q] NR + k], the terms subtracted in
// q order; the positions, values and gathers of four couplings are issued
// before their products, so a row's chain waits once per four couplings.
template <int NR>
__device__ __forceinline__ double nd_sub_couplings(double x, int64_t qb, int64_t qe,
                                                   const int32_t* __restrict__ pos,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ vec, int k) {
  int64_t q = qb;
  for (; q + 4 <= qe; q += 4) {
    int32_t c[4];
    double a[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      c[u] = pos[q + u];
      a[u] = val[q + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) y[u] = vec[(size_t)c[u] * NR + k];
#pragma unroll
    for (int u = 0; u < 4; ++u) x = fma(-a[u], y[u], x);
  }
  for (; q < qe; ++q) x = fma(-val[q], vec[(size_t)pos[q] * NR + k], x);
  return x;
}

template <int NR>
__global__ __launch_bounds__(64 * NdWaves<NR>::v) void k_nd_blocks(
    int pass, int from_y1, int nwg, const int32_t* __restrict__ wg_blk,
    const int32_t* __restrict__ wg_row0, const int64_t* __restrict__ blk_off,
    const int64_t* __restrict__ inv_off, const double* __restrict__ binv,
    const int32_t* __restrict__ ord, const double* __restrict__ bpart,
    const int64_t* __restrict__ b_ptr, const int32_t* __restrict__ b_top,
    const double* __restrict__ b_val, const double* __restrict__ eta2, double* __restrict__ y1,
    double* __restrict__ eta, int pcg, int init, const double* __restrict__ opb, int npb,
    PcgScalars* sc, PcgShared* sh) {
  constexpr int NW = NdWaves<NR>::v;
  extern __shared__ double rhs[];
  __shared__ int skip;
  __shared__ double red[NW * NR];
  if (threadIdx.x == 0) skip = (pcg && !init && all_done(sh)) ? 1 : 0;
  __syncthreads();
  if (skip) return;  // uniform: one read for the whole workgroup
  if ((int)blockIdx.x == nwg) {
    // the extra workgroup of the first launch of the solve: the PCG stop
    // decision, beside the products (the later launches read its outcome;
    // the other workgroups of this launch may see it or not, which changes
    // nothing but work that the stop makes unneeded)
    stop_test_wg<NR>(opb, npb, init, sc, sh, red);
    return;
  }
  const int b = wg_blk[blockIdx.x];
  const int row0 = wg_row0[blockIdx.x];
  const int64_t o = blk_off[b];
  const int s = (int)(blk_off[b + 1] - o);
  if (from_y1) {  // pass 1: b_B - S_BT eta_T, formed by k_nd_rb
    for (int t = threadIdx.x; t < s * NR; t += blockDim.x) rhs[t] = y1[(size_t)o * NR + t];
  } else {
    for (int t = threadIdx.x; t < s * NR; t += blockDim.x) {
      const int j = t / NR, k = t % NR;
      const int64_t n = ord[o + j];
      double v = bpart[(size_t)(2 * n) * NR + k] + bpart[(size_t)(2 * n + 1) * NR + k];
      if (pass)
        v = nd_sub_couplings<NR>(v, b_ptr[o + j], b_ptr[o + j + 1], b_top, b_val, eta2, k);
      rhs[t] = v;
    }
  }
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int per = (s + NW - 1) / NW;
  const int jb = min(s, w * per), je = min(s, jb + per);
  nd_d4 acc[4];
  nd_wave_product<NR, false>(binv + inv_off[b], s, row0, s, jb, je, rhs, 0, acc);
  __syncthreads();  // every wave is done with rhs
  double* part = rhs;  // [NW][64][NR]
  nd_wave_each<NR>(acc, [&](int l, int k, double v) { part[(w * 64 + l) * NR + k] = v; });
  __syncthreads();
  for (int t = threadIdx.x; t < 64 * NR; t += blockDim.x) {
    const int l = t / NR, k = t % NR;
    const int r = row0 + l;
    if (r >= s) continue;
    double v = part[l * NR + k];
#pragma unroll
    for (int u = 1; u < NW; ++u) v += part[(64 * u + l) * NR + k];
    if (pass == 0)
      y1[(size_t)(o + r) * NR + k] = v;
    else
      eta[(size_t)ord[o + r] * NR + k] = v;
  }
}

// Row parts of eta_T = C^{-1} r_T, r_T = b_T - S_TB y_B.  Workgroup
// (part p, group g): the part's rows j of r_T are formed in LDS (each from its
// couplings to block rows), then wave w of the group takes the 64 outputs
// 64 (4 g + w) .. and sums over the part's j (nd_wave_product; C^{-1} is
// streamed once, non-temporal).  The part sums go to ypart[p][row][k].
// Dynamic LDS: rows per part times NR doubles.
template <int NR, bool PRE>
__global__ __launch_bounds__(256) void k_nd_top(
    int R, int ldC, const double* __restrict__ cinv, int P, int per, int nrb,
    const int32_t* __restrict__ ord_top, const double* __restrict__ bpart,
    const int64_t* __restrict__ t_ptr, const int32_t* __restrict__ t_pos,
    const double* __restrict__ t_val, const double* __restrict__ y1,
    const double* __restrict__ eta2, double* __restrict__ ypart, int pcg, int init,
    const PcgShared* sh) {
  extern __shared__ double r2[];
  __shared__ int skip;
  if (threadIdx.x == 0) skip = (pcg && !init && all_done(sh)) ? 1 : 0;
  __syncthreads();
  if (skip) return;
  const int p = blockIdx.x % P, g = blockIdx.x / P;
  const int jb = min(R, p * per), je = min(R, jb + per);
  const double* v = r2;  // the part's rows of r_T
  int vbase = jb;
  if (PRE) {  // formed by k_nd_rt (held in eta2 until k_nd_fold)
    v = eta2;
    vbase = 0;
  } else {
    for (int t = threadIdx.x; t < (je - jb) * NR; t += blockDim.x) {
      const int j = jb + t / NR, k = t % NR;
      const int64_t n = ord_top[j];
      double x = bpart[(size_t)(2 * n) * NR + k] + bpart[(size_t)(2 * n + 1) * NR + k];
      r2[t] = nd_sub_couplings<NR>(x, t_ptr[j], t_ptr[j + 1], t_pos, t_val, y1, k);
    }
    __syncthreads();
  }
  const int w = threadIdx.x >> 6;
  const int rb = 4 * g + w;
  if (rb >= nrb) return;
  nd_d4 acc[4];
  nd_wave_product<NR, true>(cinv, ldC, 64 * rb, ldC, jb, je, v, vbase, acc);
  double* out = ypart + (size_t)p * ldC * NR;
  nd_wave_each<NR>(acc, [&](int l, int k, double v) { out[(size_t)(64 * rb + l) * NR + k] = v; });
}

// eta_T = sum of the part sums, to eta2 (ND order, for pass 1) and to eta
// (original order).  Eight neighbouring lanes share an output: lane u sums
// the parts u, u + 8, ... in order (their loads all in flight), then the
// eight lane sums are added pairwise by shuffles (every lane ends with the
// same bits, as a + b = b + a exactly).  The order is fixed, so the result
// is the same on every run.
constexpr int kNdFoldLanes = 8;
template <int NR>
__global__ __launch_bounds__(256) void k_nd_fold(int R, int ldC, int P,
                                                 const double* __restrict__ ypart,
                                                 const int32_t* __restrict__ ord_top,
                                                 double* __restrict__ eta2, double* __restrict__ eta,
                                                 int pcg, int init, const PcgShared* sh) {
  if (pcg && !init && all_done(sh)) return;
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kNdFoldLanes;
  const int u = threadIdx.x % kNdFoldLanes;
  const bool ok = t < (int64_t)R * NR;  // the lanes of an output agree
  const int64_t tc = ok ? t : 0;
  const int64_t r = tc / NR;
  const int k = (int)(tc % NR);
  double v = 0.0;
#pragma unroll 8
  for (int p = u; p < P; p += kNdFoldLanes) v += ypart[((size_t)p * ldC + r) * NR + k];
#pragma unroll
  for (int off = 1; off < kNdFoldLanes; off <<= 1) v += __shfl_xor(v, off, 64);
  if (ok && u == 0) {
    eta2[r * NR + k] = v;
    eta[(size_t)ord_top[r] * NR + k] = v;
  }
}

// r_T = b_T - S_TB y_B, one thread per (top row, column), into eta2 (which
// holds eta_T only from k_nd_fold on)
template <int NR>
__global__ __launch_bounds__(256) void k_nd_rt(int R, const int32_t* __restrict__ ord_top,
                                               const double* __restrict__ bpart,
                                               const int64_t* __restrict__ t_ptr,
                                               const int32_t* __restrict__ t_pos,
                                               const double* __restrict__ t_val,
                                               const double* __restrict__ y1,
                                               double* __restrict__ rt, int pcg, int init,
                                               const PcgShared* sh) {
  if (pcg && !init && all_done(sh)) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)R * NR) return;
  const int64_t j = t / NR;
  const int k = (int)(t % NR);
  const int64_t n = ord_top[j];
  double x = bpart[(size_t)(2 * n) * NR + k] + bpart[(size_t)(2 * n + 1) * NR + k];
  rt[t] = nd_sub_couplings<NR>(x, t_ptr[j], t_ptr[j + 1], t_pos, t_val, y1, k);
}

// b_B - S_BT eta_T, one thread per (block row, column), into y1 (y_B is no
// longer needed once r_T is formed)
template <int NR>
__global__ __launch_bounds__(256) void k_nd_rb(int64_t nrows, const int32_t* __restrict__ ord,
                                               const double* __restrict__ bpart,
                                               const int64_t* __restrict__ b_ptr,
                                               const int32_t* __restrict__ b_top,
                                               const double* __restrict__ b_val,
                                               const double* __restrict__ eta2,
                                               double* __restrict__ rb, int pcg, int init,
                                               const PcgShared* sh) {
  if (pcg && !init && all_done(sh)) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * NR) return;
  const int64_t j = t / NR;
  const int k = (int)(t % NR);
  const int64_t n = ord[j];
  double x = bpart[(size_t)(2 * n) * NR + k] + bpart[(size_t)(2 * n + 1) * NR + k];
  rb[t] = nd_sub_couplings<NR>(x, b_ptr[j], b_ptr[j + 1], b_top, b_val, eta2, k);
}

// Launch sequence.  1-2 columns: four launches, the coupling terms formed in
// the prologues of the top product and of the second block pass (few
// couplings per row there, and no launch boundary to pay).  4-16 columns:
// r_T and b_B - S_BT eta_T get launches of their own, so that the products
// read them instead of each workgroup forming its share again.
template <int NR>
static void nd_solve_t(DeviceState& d, hipStream_t st, int pcg, int init) {
  constexpr bool PRE = NR >= 4;
  constexpr int NW = NdWaves<NR>::v;
  const NdDevice& nd = d.nd;
  const size_t shb = (size_t)std::max<int64_t>(nd.smax, 64 * NW) * NR * sizeof(double);
  // the PCG stop test rides in one extra workgroup of the first launch
  const unsigned extra = pcg ? 1u : 0u;
  if (nd.R > 0) {
    am_launch_shm(d, true, false, k_nd_blocks<NR>, dim3(nd.nwg + extra), dim3(64 * NW), shb, st,
                  0, 0, nd.nwg, nd.wg_blk, nd.wg_row0, nd.blk_off, nd.inv_off, nd.binv, nd.ord,
                  d.bpart, nd.b_ptr, nd.b_top, nd.b_val, nd.eta2, nd.y1, d.eta, pcg, init,
                  d.red.pb, d.m, d.sc, d.shared);
    if (PRE)
      am_launch(d, false, false, k_nd_rt<NR>, dim3((unsigned)((nd.R * NR + 255) / 256)),
                dim3(256), st, nd.R, nd.ord + nd.nrows, d.bpart, nd.t_ptr, nd.t_pos, nd.t_val,
                nd.y1, nd.eta2, pcg, init, d.shared);
    const int nrb = (nd.ldC + 63) / 64;
    am_launch_shm(d, false, false, k_nd_top<NR, PRE>, dim3(nd.P * ((nrb + 3) / 4)), dim3(256),
                  PRE ? 0 : (size_t)nd.per * NR * sizeof(double), st, nd.R, nd.ldC, nd.cinv, nd.P,
                  nd.per, nrb, nd.ord + nd.nrows, d.bpart, nd.t_ptr, nd.t_pos, nd.t_val, nd.y1,
                  nd.eta2, nd.ypart, pcg, init, d.shared);
  }
  const unsigned nb =
      (unsigned)std::max<int64_t>(1, ((int64_t)nd.R * NR * kNdFoldLanes + 255) / 256);
  if (nd.R > 0)
    am_launch(d, false, false, k_nd_fold<NR>, dim3(nb), dim3(256), st, nd.R, nd.ldC, nd.P,
              nd.ypart, nd.ord + nd.nrows, nd.eta2, d.eta, pcg, init, d.shared);
  if (PRE && nd.R > 0)
    am_launch(d, false, false, k_nd_rb<NR>, dim3((unsigned)((nd.nrows * NR + 255) / 256)),
              dim3(256), st, nd.nrows, nd.ord, d.bpart, nd.b_ptr, nd.b_top, nd.b_val, nd.eta2,
              nd.y1, pcg, init, d.shared);
  // with no top rows this is the only launch (it then carries the stop test)
  const unsigned extra1 = nd.R > 0 ? 0u : extra;
  am_launch_shm(d, nd.R == 0, true, k_nd_blocks<NR>, dim3(nd.nwg + extra1), dim3(64 * NW), shb,
                st, 1, (PRE && nd.R > 0) ? 1 : 0, nd.nwg, nd.wg_blk, nd.wg_row0, nd.blk_off,
                nd.inv_off, nd.binv, nd.ord, d.bpart, nd.b_ptr, nd.b_top, nd.b_val, nd.eta2, nd.y1,
                d.eta, pcg, init, d.red.pb, d.m, d.sc, d.shared);
}

hipError_t launch_nd_solve(DeviceState& d, int nr, int pcg, int init, hipStream_t st) {
  if (nr > d.max_nrhs) return hipErrorInvalidValue;
  switch (nr) {
    case 1: nd_solve_t<1>(d, st, pcg, init); break;
    case 2: nd_solve_t<2>(d, st, pcg, init); break;
    case 4: nd_solve_t<4>(d, st, pcg, init); break;
    case 8: nd_solve_t<8>(d, st, pcg, init); break;
    case 16: nd_solve_t<16>(d, st, pcg, init); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---- set-up ----------------------------------------------------------------

// Sp[a][c] = S[src[a]][src[c]] over the padded ND order (src = -1: padding,
// which holds the identity)
__global__ __launch_bounds__(256) void k_nd_gather(const double* __restrict__ S, int ldS,
                                                   const int32_t* __restrict__ src, int ldp,
                                                   double* __restrict__ Sp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)ldp * ldp) return;
  const int a = (int)(t / ldp), c = (int)(t % ldp);
  const int32_t sa = src[a], sc = src[c];
  Sp[t] = (sa < 0 || sc < 0) ? (a == c ? 1.0 : 0.0) : S[(size_t)sa * ldS + sc];
}

// C^{-1}[j][c] = X[top0 + j][top0 + c] for c < R, 0 for R <= c < ldC
__global__ __launch_bounds__(256) void k_nd_extract_top(const double* __restrict__ X, int ldp,
                                                        int64_t top0, int R, int ldC,
                                                        double* __restrict__ cinv) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)R * ldC) return;
  const int64_t j = t / ldC, c = t % ldC;
  cinv[t] = c < R ? X[(size_t)(top0 + j) * ldp + top0 + c] : 0.0;
}

// block b's inverse as a full square (leading dimension s_b) from the
// diagonal block of X that starts at pad_off[b]
__global__ __launch_bounds__(256) void k_nd_extract_blocks(const double* __restrict__ X, int ldp,
                                                           const int64_t* __restrict__ pad_off,
                                                           const int64_t* __restrict__ blk_off,
                                                           const int64_t* __restrict__ inv_off,
                                                           double* __restrict__ binv) {
  const int b = blockIdx.y;
  const int64_t s = blk_off[b + 1] - blk_off[b], po = pad_off[b];
  double* out = binv + inv_off[b];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < s * s;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = t / s, c = t % s;
    out[t] = X[(size_t)(po + a) * ldp + po + c];
  }
}

// out[q] = S[ri[q]][ci[q]]
__global__ __launch_bounds__(256) void k_nd_pairs(const double* __restrict__ S, int ldS,
                                                  const int32_t* __restrict__ ri,
                                                  const int32_t* __restrict__ ci, int64_t cnt,
                                                  double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) out[t] = S[(size_t)ri[t] * ldS + ci[t]];
}

// The numeric part of the set-up, on the S of the handle (original order):
// reorder, factor and invert (tiled, kernels_iface.hip), form the block
// inverses and C^{-1}, gather the coupling values.  L, Li: ldp x ldp scratch,
// Sp: ldp x ldp scratch, part: trtri_part_tiles(ldp / 64) tiles.  d.Sinv
// receives the reordered S^{-1} (ld ldp).
hipError_t nd_numeric(DeviceState& d, double* Sp, double* L, double* Li, double* part,
                      hipStream_t st) {
  NdDevice& nd = d.nd;
  const int ldp = nd.ldp;
  const int64_t tot = (int64_t)ldp * ldp;
  hipLaunchKernelGGL(k_nd_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, d.S,
                     d.ldS, nd.src, ldp, Sp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the tiled factorization reads d.S with leading dimension d.ldS
  double* S0 = d.S;
  const int32_t ld0 = d.ldS;
  d.S = Sp;
  d.ldS = ldp;
  e = dense_cholesky_inverse(d, L, Li, part, st);
  d.S = S0;
  d.ldS = ld0;
  if (e != hipSuccess) return e;
  // block products L_bb^{-T} L_bb^{-1} into the (now free) factor buffer
  for (int b = 0; b < nd.nblk; ++b) {
    const int64_t po = nd.h_pad_off[b];
    const int T = (int)((nd.h_blk_off[b + 1] - nd.h_blk_off[b] + 63) / 64);
    e = launch_lauum(Li + po * ldp + po, L + po * ldp + po, ldp, T, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_nd_extract_blocks, dim3(64, nd.nblk), dim3(256), 0, st, L, ldp, nd.pad_off,
                     nd.blk_off, nd.inv_off, nd.binv);
  if (nd.R > 0) {
    const int64_t nc = (int64_t)nd.R * nd.ldC;
    hipLaunchKernelGGL(k_nd_extract_top, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st,
                       d.Sinv, ldp, nd.h_pad_off[nd.nblk], nd.R, nd.ldC, nd.cinv);
  }
  if (nd.nt_pairs > 0)
    hipLaunchKernelGGL(k_nd_pairs, dim3((unsigned)((nd.nt_pairs + 255) / 256)), dim3(256), 0, st,
                       d.S, d.ldS, nd.t_ri, nd.t_ci, nd.nt_pairs, nd.t_val);
  if (nd.nb_pairs > 0)
    hipLaunchKernelGGL(k_nd_pairs, dim3((unsigned)((nd.nb_pairs + 255) / 256)), dim3(256), 0, st,
                       d.S, d.ldS, nd.b_ri, nd.b_ci, nd.nb_pairs, nd.b_val);
  return hipGetLastError();
}

}  // namespace am
