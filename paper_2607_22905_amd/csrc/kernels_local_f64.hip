// Subdomain kernels instantiated for f64 factors.
#include "local_kernels.h"

namespace am {
template hipError_t band_factor_t<double>(DeviceState&, hipStream_t);
template hipError_t mbf_t<double>(DeviceState&, hipStream_t);
template hipError_t invert_diag_t<double>(DeviceState&, hipStream_t);
template hipError_t local_nr<double>(DeviceState&, const double*, double*, const double*, int, int,
                                  int, hipStream_t);
}  // namespace am
