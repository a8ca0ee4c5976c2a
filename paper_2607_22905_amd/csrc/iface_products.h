// Wave-level products with symmetric dense interface operators (the blocks
// of the nested-dissection solve and of the block-Jacobi preconditioner of
// the inexact interface solve).  Internal header.
#pragma once

#include "am_common.h"

namespace am {

typedef double nd_d4 __attribute__((ext_vector_type(4)));

// One wave's share of out[r][k] = sum_{m in [mb, me)} X[m][r] v[m][k] for the
// 64 outputs r = r0 .. r0 + 63 of a symmetric matrix X (leading dimension
// ld; its row m stands for column m), v[m][.] in LDS at v + (m - vbase) NR.
// NR <= 2: lane = r, NR FMAs per coalesced load of 64 values.  NR >= 4: four
// 16 x 16 tiles on the FP64 matrix cores (v_mfma_f64_16x16x4f64: lane l holds
// A[l % 16][l / 16] = X[m0 + l / 16][r0 + 16 t + l % 16], B[l / 16][l % 16] =
// v[m0 + l / 16][l % 16] (zero beyond NR) and D[l / 16 + 4 q][l % 16]), two
// steps of four rows of X loaded before their products.  Rows r >= rmax and
// columns m >= me read as zero.  acc: [4][4] (matrix cores: tile t, entry
// q) or [NR] (lane = row) in acc[0..NR-1][0].
template <int NR, bool NT>
__device__ __forceinline__ void nd_wave_product(const double* __restrict__ X, int64_t ld, int r0,
                                                int rmax, int mb, int me, const double* v,
                                                int vbase, nd_d4 (&acc)[4]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = nd_d4{0.0, 0.0, 0.0, 0.0};
  if constexpr (NR <= 2) {
    const int r = r0 + lane;
    if (r >= rmax) return;
    const double* col = X + r;
    double a0[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) a0[k] = 0.0;
#pragma unroll 4
    for (int m = mb; m < me; ++m) {
      const double a = NT ? __builtin_nontemporal_load(col + (size_t)m * ld) : col[(size_t)m * ld];
#pragma unroll
      for (int k = 0; k < NR; ++k) a0[k] = fma(a, v[(m - vbase) * NR + k], a0[k]);
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k][0] = a0[k];
  } else {
    const int li = lane % 16, lk = lane / 16;
    constexpr int U = 2;
    for (int m0 = mb; m0 < me; m0 += 4 * U) {
      double av[U][4], bv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int m = m0 + 4 * u + lk;
        const bool ok = m < me;
        bv[u] = (ok && li < NR) ? v[(m - vbase) * NR + li] : 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int r = r0 + 16 * t + li;
          const double* pa = X + (size_t)m * ld + r;
          av[u][t] = (ok && r < rmax) ? (NT ? __builtin_nontemporal_load(pa) : *pa) : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][t], bv[u], acc[t], 0, 0, 0);
    }
  }
}

// calls f(row offset in 0 .. 63, column k, value) for the wave's results
template <int NR, typename F>
__device__ __forceinline__ void nd_wave_each(const nd_d4 (&acc)[4], F&& f) {
  const int lane = threadIdx.x & 63;
  if constexpr (NR <= 2) {
#pragma unroll
    for (int k = 0; k < NR; ++k) f(lane, k, acc[k][0]);
  } else {
    const int li = lane % 16, lk = lane / 16;
    if (li < NR)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) f(16 * t + lk + 4 * q, li, acc[t][q]);
  }
}

}  // namespace am
