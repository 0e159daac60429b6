// Fixed device scratch for callers that cannot allocate (code under graph
// capture, tight serving loops, harnesses that forbid hipMalloc): a file-scope
// device array, one copy per GPU, whose address is looked up once per device.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "hierarchy_internal.hpp"

namespace vk {

namespace {

// Every GPU the library runs on holds this array until the process ends.  In
// host code its name is only a host-side stand-in: device code reaches it
// through the address hipGetSymbolAddress returns for the current device.
__device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

void* noalloc_scratch(int device) {
  require(device >= 0 && device < kMaxDevices, VK_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    HIPCHECK(hipGetDevice(&cur));
    if (cur != device) HIPCHECK(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || p == nullptr)
      throw Error(VK_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[device] = p;
  }
  return g_ptr[device];
}

}  // namespace vk
