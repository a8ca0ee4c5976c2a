// Subdomain kernels instantiated for f32 factors.
#include "local_kernels.h"

namespace am {
template hipError_t band_factor_t<float>(DeviceState&, hipStream_t);
template hipError_t mbf_t<float>(DeviceState&, hipStream_t);
template hipError_t invert_diag_t<float>(DeviceState&, hipStream_t);
template hipError_t local_nr<float>(DeviceState&, const double*, double*, const double*, int, int,
                                  int, hipStream_t);
}  // namespace am
