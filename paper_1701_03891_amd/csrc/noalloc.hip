// noalloc.hip -- the fixed device workspace of dsi_recover_noalloc.
//
// A file-scope __device__ array: every device that loads the library's code
// object holds its own copy, at its own address, until the process ends.  In
// host code the name `scratch` is only a host-side stand-in, never a device
// address; the device address comes from hipGetSymbolAddress, taken once per
// device with that device current and kept in g_ptr.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/dsi.h"
#include "internal.h"

static __device__ __align__(256) unsigned char scratch[DSI_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
}  // namespace

namespace dsi {

hipError_t noalloc_scratch(int device, void **ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

}  // namespace dsi
