// Small device helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "am_device.h"
#include <hip/hip_ext.h>

namespace am {

// Kernel launch that, in a profiled solve, attaches d.prof_ev[0] to the
// first launch of an operation and d.prof_ev[1] to its last (the events
// then hold the start and end of those dispatches, without the latency of a
// separate event record).  Arguments are converted to the kernel's parameter
// types, as the extended launch packs them as given.
template <typename... KArgs, typename... Args>
inline void am_launch_shm(DeviceState& d, bool first, bool last, void (*kern)(KArgs...), dim3 grid,
                          dim3 block, size_t shmem, hipStream_t st, Args&&... args) {
  static_assert(sizeof...(KArgs) == sizeof...(Args), "argument count");
  hipEvent_t e0 = first ? d.prof_ev[0] : nullptr, e1 = last ? d.prof_ev[1] : nullptr;
  if (e0 || e1) {
    hipExtLaunchKernelGGL(kern, grid, block, shmem, st, e0, e1, 0, static_cast<KArgs>(args)...);
    if (e0) d.prof_used[0] = true;
    if (e1) d.prof_used[1] = true;
  } else {
    hipLaunchKernelGGL(kern, grid, block, shmem, st, static_cast<KArgs>(args)...);
  }
}
// the same with no dynamic LDS
template <typename... KArgs, typename... Args>
inline void am_launch(DeviceState& d, bool first, bool last, void (*kern)(KArgs...), dim3 grid,
                      dim3 block, hipStream_t st, Args&&... args) {
  am_launch_shm(d, first, last, kern, grid, block, 0, st, static_cast<Args&&>(args)...);
}

typedef uint16_t bf16_t;

__device__ __forceinline__ double readlane_d(double v, int lane) {
  int2 b = __builtin_bit_cast(int2, v);
  b.x = __builtin_amdgcn_readlane(b.x, lane);
  b.y = __builtin_amdgcn_readlane(b.y, lane);
  return __builtin_bit_cast(double, b);
}
__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ double readlane(double v, int lane) { return readlane_d(v, lane); }
__device__ __forceinline__ float readlane(float v, int lane) { return readlane_f(v, lane); }
// The LLVM intrinsic behind v_writelane_b32 (no clang builtin exposes it).
__device__ int am_writelane_i32(int v, int lane, int old) __asm("llvm.amdgcn.writelane.i32");
// old with lane `lane` replaced by the uniform value v
__device__ __forceinline__ double writelane(double v, int lane, double old) {
  int2 a = __builtin_bit_cast(int2, v), o = __builtin_bit_cast(int2, old);
  o.x = am_writelane_i32(a.x, lane, o.x);
  o.y = am_writelane_i32(a.y, lane, o.y);
  return __builtin_bit_cast(double, o);
}
__device__ __forceinline__ float writelane(float v, int lane, float old) {
  return __builtin_bit_cast(float, am_writelane_i32(__builtin_bit_cast(int, v), lane,
                                                    __builtin_bit_cast(int, old)));
}

// factor element loads (bf16 is stored as raw bits, widened to fp32)
__device__ __forceinline__ double ld_fac(const double* p) { return *p; }
__device__ __forceinline__ float ld_fac(const float* p) { return *p; }
__device__ __forceinline__ float ld_fac(const bf16_t* p) {
  return __builtin_bit_cast(float, ((uint32_t)*p) << 16);
}
// raw element loads kept in a prefetch ring, widened only when consumed
__device__ __forceinline__ double ld_raw(const double* p) { return *p; }
__device__ __forceinline__ float ld_raw(const float* p) { return *p; }
__device__ __forceinline__ uint32_t ld_raw(const bf16_t* p) { return (uint32_t)*p; }
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ float widen(uint32_t v) { return __builtin_bit_cast(float, v << 16); }
// LDS copies of factor tiles keep the storage type; widened when read
__device__ __forceinline__ double widen_lds(double v) { return v; }
__device__ __forceinline__ float widen_lds(float v) { return v; }
__device__ __forceinline__ float widen_lds(bf16_t v) {
  return __builtin_bit_cast(float, (uint32_t)v << 16);
}
template <typename FT> struct RawT { using T = FT; };
template <> struct RawT<bf16_t> { using T = uint32_t; };
// round-to-nearest-even conversions from fp64
__device__ __forceinline__ void st_fac(double* p, double v) { *p = v; }
__device__ __forceinline__ void st_fac(float* p, double v) { *p = (float)v; }
__device__ __forceinline__ void st_fac(bf16_t* p, double v) {
  float f = (float)v;
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  *p = (bf16_t)(u >> 16);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of v[k] over the block (fixed tree); result valid in every thread.
// lds must hold (blockDim.x/64) * NR doubles.
template <int NR>
__device__ __forceinline__ void block_sum(double (&v)[NR], double* lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NR; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NR; ++k) lds[w * NR + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += lds[i * NR + k];
    v[k] = s;
  }
  __syncthreads();
}

// Publish this block's sums and tell whether it is the last block of the
// launch to do so.  The last block then reads every block's partial sums (in
// block order, so the total is deterministic) and resets the counter.
template <int NR>
__device__ __forceinline__ bool publish_partial(const double (&v)[NR], double* partial,
                                                unsigned* counter, unsigned nblocks) {
  __shared__ int last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NR; ++k) partial[(size_t)blockIdx.x * NR + k] = v[k];
    __threadfence();
    unsigned prev = atomicAdd(counter, 1u);
    last = (prev == nblocks - 1) ? 1 : 0;
  }
  __syncthreads();
  if (last) __threadfence();
  return last != 0;
}

// tot[k] += part[b * NR + k] over the rows b = first, first + step, ... < nb,
// in that order.  U rows at a time have their loads issued together: the
// row index is clamped into range and a row past the end adds exact zeros,
// so no branch separates the loads (a loop with one guarded load per row
// waits for each load before the next).
template <int NR>
__device__ __forceinline__ void fold_rows(const double* __restrict__ part, int nb, int first,
                                          int step, double (&tot)[NR]) {
  constexpr int U = NR >= 8 ? 2 : 16 / NR;
  for (int b0 = first; b0 < nb; b0 += U * step) {
    double v[U][NR];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = min(b0 + u * step, nb - 1);
#pragma unroll
      for (int k = 0; k < NR; ++k) v[u][k] = part[(size_t)b * NR + k];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = b0 + u * step < nb;
#pragma unroll
      for (int k = 0; k < NR; ++k) tot[k] += ok ? v[u][k] : 0.0;
    }
  }
}

template <int NR>
__device__ __forceinline__ void reduce_partials(double (&tot)[NR], const double* partial,
                                                unsigned nblocks, double* lds) {
#pragma unroll
  for (int k = 0; k < NR; ++k) tot[k] = 0.0;
  fold_rows<NR>(partial, (int)nblocks, threadIdx.x, blockDim.x, tot);
  block_sum<NR>(tot, lds);
}

// Node vectors with NT right-hand sides: value (row, k) at row * NT + k, the
// NT columns of a row contiguous (a 128-byte line for 16 columns), so that a
// gathered neighbour brings all its columns in one line.  Kernels give each
// thread a group of KG = min(NT, 4) columns of a row; with more columns the
// NT / KG threads of a row are neighbouring lanes.
template <int NT> struct KGroup { static constexpr int v = NT <= 4 ? NT : 4; };
template <int NT>
__device__ __forceinline__ size_t vix(int64_t /*n*/, int64_t row, int k) {
  return (size_t)row * NT + k;
}

__device__ __forceinline__ bool all_done(const PcgShared* sh) {
  return *(volatile const int32_t*)&sh->all_done != 0;
}

// The PCG stop test of one iteration, in one wave: folds the ||r||^2
// partials of the update launch (same order in every workgroup), and
// workgroup 0 (lane 0, when `writer`) stores the column states and all_done.
template <int NR>
__device__ __forceinline__ bool stop_test(const double* __restrict__ pb, int npb, int init,
                                          PcgScalars* sc, PcgShared* sh, bool writer = true) {
  // one wave: fold the ||r||^2 partials in block order (same order in every
  // workgroup); the scalars are loaded first, independently of the partials
  const int lane = threadIdx.x & 63;
  const int nrhs = sh->nrhs, maxit = sh->maxit;
  PcgScalars S[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) S[k] = sc[k];
  double rr[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) rr[k] = 0.0;
  fold_rows<NR>(pb, npb, lane, 64, rr);
#pragma unroll
  for (int k = 0; k < NR; ++k) rr[k] = wave_sum(rr[k]);
  int alld = 1;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (k >= nrhs) continue;
    int done = S[k].done, conv = S[k].conv, status = S[k].status;
    double bb = S[k].bb;
    if (!done) {
      if (init) {
        bb = rr[k];
        if (bb == 0.0) done = conv = 1;
      } else if (rr[k] <= S[k].tol2 * S[k].bb) {
        done = conv = 1;
      } else if (S[k].it >= maxit) {
        done = 1;
        status = AM_ERR_NO_CONVERGENCE;
      }
    }
    alld &= done;
    if (blockIdx.x == 0 && lane == 0 && writer) {
      sc[k].rr = rr[k];
      sc[k].bb = bb;
      sc[k].done = done;
      sc[k].conv = conv;
      sc[k].status = status;
    }
  }
  if (blockIdx.x == 0 && lane == 0 && writer) sh->all_done = alld;
  return alld != 0;
}

// The same stop test taken by a whole workgroup (every thread of it calls
// this): the partials are folded by all its threads (reduce_partials, a
// fixed order), thread 0 stores the column states and all_done.  lds holds
// (blockDim.x / 64) NR doubles.
template <int NR>
__device__ __forceinline__ void stop_test_wg(const double* __restrict__ pb, int npb, int init,
                                             PcgScalars* sc, PcgShared* sh, double* lds) {
  const int nrhs = sh->nrhs, maxit = sh->maxit;
  double rr[NR];
  reduce_partials<NR>(rr, pb, (unsigned)npb, lds);
  int alld = 1;
  for (int k = 0; k < nrhs && k < NR; ++k) {
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

// ---------------------------------------------------------------------------
// Interface partial right-hand sides from r (not from pbar): for subdomain s
// and slot q (basis function n = I_s[q]),
//   bpart[s,q] = 1/4 * phat^(n)_s . r_s,
// stored at slot 2n + side (side 0 for the lower subdomain i, 1 for j), so that
// b_n = bpart[2n] + bpart[2n+1] = -sum_{e in E_n} a_e (pbar_k + pbar_l)/2.
// (A_s is symmetric and phat^(n)_s = A_s^{-1}(-B_s psi_n) = 4 A_s^{-1} w with
// w_k = -sum a_e / 2 the weights of the edge average.)
template <int NR>
__device__ __forceinline__ void bpart_sub(int s, int64_t n, const int64_t* __restrict__ sub_ptr,
                                          const int64_t* __restrict__ isub_ptr,
                                          const int64_t* __restrict__ mbf_off,
                                          const double* __restrict__ mbf,
                                          const int64_t* __restrict__ bdst, const double* r,
                                          double* bpart, double* lds) {
  constexpr int QB = NR <= 2 ? 8 : (NR <= 4 ? 4 : (NR <= 8 ? 2 : 1));  // slots per round
  const int64_t base = sub_ptr[s];
  const int N = (int)(sub_ptr[s + 1] - base);
  const int64_t i0 = isub_ptr[s];
  const int ns = (int)(isub_ptr[s + 1] - i0);
  const double* P = mbf + mbf_off[s];
  for (int q0 = 0; q0 < ns; q0 += QB) {
    double v[QB * NR];
#pragma unroll
    for (int t = 0; t < QB * NR; ++t) v[t] = 0.0;
#pragma unroll 2
    for (int row = threadIdx.x; row < N; row += blockDim.x) {
      double rv[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) rv[k] = r[vix<NR>(n, base + row, k)];
#pragma unroll
      for (int qq = 0; qq < QB; ++qq) {
        const double ph = (q0 + qq < ns) ? P[(size_t)(q0 + qq) * N + row] : 0.0;
#pragma unroll
        for (int k = 0; k < NR; ++k) v[qq * NR + k] = fma(ph, rv[k], v[qq * NR + k]);
      }
    }
    block_sum<QB * NR>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
      for (int qq = 0; qq < QB; ++qq)
        if (q0 + qq < ns)
#pragma unroll
          for (int k = 0; k < NR; ++k)
            bpart[(size_t)bdst[i0 + q0 + qq] * NR + k] = 0.25 * v[qq * NR + k];
  }
}

}  // namespace am
