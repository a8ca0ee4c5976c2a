// Subdomain kernels instantiated for bf16 factors.
#include "local_kernels.h"

namespace am {
template hipError_t band_factor_t<bf16_t>(DeviceState&, hipStream_t);
template hipError_t mbf_t<bf16_t>(DeviceState&, hipStream_t);
template hipError_t invert_diag_t<bf16_t>(DeviceState&, hipStream_t);
template hipError_t local_nr<bf16_t>(DeviceState&, const double*, double*, const double*, int, int,
                                  int, hipStream_t);
}  // namespace am
