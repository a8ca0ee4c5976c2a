// Subdomain kernels: launch entry points.  The kernels and the launcher
// templates live in local_kernels.h; each factor precision is instantiated
// in its own translation unit (kernels_local_f64/f32/bf16.hip) so that the
// three compile in parallel.
#include "local_kernels.h"

namespace am {

#define AM_LOCAL_EXTERN(FT)                                                                  \
  extern template hipError_t band_factor_t<FT>(DeviceState&, hipStream_t);                  \
  extern template hipError_t mbf_t<FT>(DeviceState&, hipStream_t);                          \
  extern template hipError_t invert_diag_t<FT>(DeviceState&, hipStream_t);                  \
  extern template hipError_t local_nr<FT>(DeviceState&, const double*, double*, const double*, \
                                          int, int, int, hipStream_t);
AM_LOCAL_EXTERN(double)
AM_LOCAL_EXTERN(float)
AM_LOCAL_EXTERN(bf16_t)
#undef AM_LOCAL_EXTERN

hipError_t launch_band_factor(DeviceState& d, hipStream_t st) {
  switch (d.prec) {
    case AM_FP64: return band_factor_t<double>(d, st);
    case AM_FP32: return band_factor_t<float>(d, st);
    default: return band_factor_t<bf16_t>(d, st);
  }
}

hipError_t launch_mbf(DeviceState& d, hipStream_t st) {
  switch (d.prec) {
    case AM_FP64: return mbf_t<double>(d, st);
    case AM_FP32: return mbf_t<float>(d, st);
    default: return mbf_t<bf16_t>(d, st);
  }
}

hipError_t launch_invert_diag(DeviceState& d, hipStream_t st) {
  switch (d.prec) {
    case AM_FP64: return invert_diag_t<double>(d, st);
    case AM_FP32: return invert_diag_t<float>(d, st);
    default: return invert_diag_t<bf16_t>(d, st);
  }
}

int tile_candidates(int nrhs) {
  switch (tile_slot(nrhs)) {
    case 0: return TileCands<1>::n;
    case 1: return TileCands<2>::n;
    case 2: return TileCands<4>::n;
    case 3: return TileCands<8>::n;
    default: return TileCands<16>::n;
  }
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
    case 1: hipLaunchKernelGGL(k_bpart<1>, g, b, 0, st, d.n, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, d.bdst, r, d.bpart); break;
    case 2: hipLaunchKernelGGL(k_bpart<2>, g, b, 0, st, d.n, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, d.bdst, r, d.bpart); break;
    case 4: hipLaunchKernelGGL(k_bpart<4>, g, b, 0, st, d.n, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, d.bdst, r, d.bpart); break;
    case 8: hipLaunchKernelGGL(k_bpart<8>, g, b, 0, st, d.n, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, d.bdst, r, d.bpart); break;
    case 16: hipLaunchKernelGGL(k_bpart<16>, g, b, 0, st, d.n, d.sub_ptr, d.isub_ptr, d.mbf_off, d.mbf, d.bdst, r, d.bpart); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The stop test of a PCG iteration as a launch of its own (one wave): used
// where the preconditioner is not the local kernel itself.
template <int NR>
__global__ __launch_bounds__(64) void k_stop(const double* __restrict__ pb, int npb, int init,
                                             PcgScalars* sc, PcgShared* sh) {
  stop_test<NR>(pb, npb, init, sc, sh);
}

hipError_t launch_stop_test(DeviceState& d, int nr, int init, hipStream_t st) {
  switch (nr) {
    case 1: hipLaunchKernelGGL(k_stop<1>, dim3(1), dim3(64), 0, st, d.red.pb, d.m, init, d.sc, d.shared); break;
    case 2: hipLaunchKernelGGL(k_stop<2>, dim3(1), dim3(64), 0, st, d.red.pb, d.m, init, d.sc, d.shared); break;
    case 4: hipLaunchKernelGGL(k_stop<4>, dim3(1), dim3(64), 0, st, d.red.pb, d.m, init, d.sc, d.shared); break;
    case 8: hipLaunchKernelGGL(k_stop<8>, dim3(1), dim3(64), 0, st, d.red.pb, d.m, init, d.sc, d.shared); break;
    case 16: hipLaunchKernelGGL(k_stop<16>, dim3(1), dim3(64), 0, st, d.red.pb, d.m, init, d.sc, d.shared); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace am
