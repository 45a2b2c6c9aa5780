// Library-owned device workspace for handles made by lbm_create_static: a
// file-scope device array (one copy on every GPU the library runs on, held
// until the process ends) whose address is resolved once per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lbm_internal.h"

namespace pplbm {

static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the current device's copy of `scratch`.  In host code
// the array's name is only a stand-in for the symbol; kernels and copies must
// use the address hipGetSymbolAddress returns for the device.
hipError_t static_workspace(void** ptr) {
  *ptr = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace pplbm
