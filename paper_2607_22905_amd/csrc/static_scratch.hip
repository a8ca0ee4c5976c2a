// Scratch of algmortar_apply_static: a file-scope device array, so that the
// entry point allocates nothing.  Every GPU the library runs on holds its own
// copy of the array (at its own address) until the process ends.  In host
// code the array's name stands for a host-side shadow, never for device
// memory: host code reaches the array only through the address that
// hipGetSymbolAddress returns on each device, kept here per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "am_device.h"

namespace am {

static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (p == nullptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

double* static_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return static_cast<double*>(g_scratch_ptr[device]);
}

}  // namespace am
