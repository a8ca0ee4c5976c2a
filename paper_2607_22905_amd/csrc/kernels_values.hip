// New values for an existing handle (same pattern and partition): the checks
// of the set-up's validation on the device, and the gathers that place the
// values where the numeric set-up (Algorithm 1) reads them.  Every gather
// copies or sums in the set-up's order, so a refreshed handle holds the same
// bits as one set up from scratch on the new values.
#include "am_common.h"

namespace am {

// Entry p of the caller's CSR: code[p] = -2 on the diagonal (must be > 0),
// -1 for a coupling without a stored transpose (must be zero), else the
// position of the transpose (bitwise equal, not positive).  cross[p] = 1 for
// a coupling between subdomains that was nonzero at set-up (an interface
// edge: must stay nonzero), 2 for one that was zero (must stay zero), 0
// inside a subdomain.  The lowest failing position goes to *bad.
__global__ __launch_bounds__(256) void k_check_values(int64_t nnz, const double* __restrict__ v,
                                                      const int64_t* __restrict__ code,
                                                      const int8_t* __restrict__ cross,
                                                      unsigned long long* bad) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const double a = v[p];
  const int64_t t = code[p];
  bool ok = isfinite(a);
  if (ok) {
    if (t == -2) {
      ok = a > 0.0;
    } else {
      const double b = t >= 0 ? v[t] : 0.0;
      const bool same = __double_as_longlong(a) == __double_as_longlong(b) || (a == 0.0 && b == 0.0);
      ok = same && !(a > 0.0);
      if (ok && cross[p] == 1) ok = a != 0.0;
      if (ok && cross[p] == 2) ok = a == 0.0;
    }
  }
  if (!ok) atomicMin(bad, (unsigned long long)p);
}

// out[q] = v[pos[q]]
__global__ __launch_bounds__(256) void k_gather_values(int64_t m, const int64_t* __restrict__ pos,
                                                       const double* __restrict__ v,
                                                       double* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) out[q] = v[pos[q]];
}

// ELL values (column-major, padding 0) from the device-order CSR values
__global__ __launch_bounds__(256) void k_ell_values(int64_t n, int w, const int64_t* __restrict__ prp,
                                                    const double* __restrict__ pv,
                                                    double* __restrict__ ell_val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = prp[i], e = prp[i + 1];
  for (int c = 0; c < w; ++c) ell_val[(int64_t)c * n + i] = b + c < e ? pv[b + c] : 0.0;
}

// Boundary weights -B_s psi_n: entry t is the sum of -2 a_e over its edges,
// added in the set-up's order (-2 a is exact, so no rounding but the sums')
__global__ __launch_bounds__(256) void k_boundary_weights(int64_t nbw, const int64_t* __restrict__ ptr,
                                                          const int32_t* __restrict__ src,
                                                          const double* __restrict__ e_a,
                                                          double* __restrict__ bw_val) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbw) return;
  const int64_t j0 = ptr[t], j1 = ptr[t + 1];
  double acc = -2.0 * e_a[src[j0]];
  for (int64_t j = j0 + 1; j < j1; ++j) acc += -2.0 * e_a[src[j]];
  bw_val[t] = acc;
}

static inline unsigned nblk(int64_t m) { return (unsigned)std::max<int64_t>(1, (m + 255) / 256); }

hipError_t launch_check_values(const ValueMaps& vm, const double* v, hipStream_t st) {
  hipError_t e = hipMemsetAsync(vm.bad, 0xFF, sizeof(unsigned long long), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_check_values, dim3(nblk(vm.nnz)), dim3(256), 0, st, vm.nnz, v, vm.code,
                     vm.cross, vm.bad);
  return hipGetLastError();
}

hipError_t launch_place_values(DeviceState& d, const ValueMaps& vm, const double* v, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_values, dim3(nblk(vm.nnz)), dim3(256), 0, st, vm.nnz, vm.vpos, v, d.pv);
  hipLaunchKernelGGL(k_ell_values, dim3(nblk(d.n)), dim3(256), 0, st, d.n, d.ell_w, d.prp, d.pv,
                     d.ell_val);
  if (d.NE > 0) {
    hipLaunchKernelGGL(k_gather_values, dim3(nblk(d.NE)), dim3(256), 0, st, (int64_t)d.NE, vm.epos,
                       v, d.e_a);
    hipLaunchKernelGGL(k_boundary_weights, dim3(nblk(vm.nbw)), dim3(256), 0, st, vm.nbw, vm.bw_ptr,
                       vm.bw_src, d.e_a, d.bw_val);
  }
  return hipGetLastError();
}

}  // namespace am
