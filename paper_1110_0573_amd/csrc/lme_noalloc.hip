// lme_noalloc.hip -- the device scratch array of lme_evolve_noalloc.
//
// Callers that cannot allocate device memory during a call (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc) use
// lme_evolve_noalloc, whose step tables, pack tables and adaptive stage
// derivatives live in this one file-scope array instead of handle-owned
// allocations.  Each GPU the library runs on holds its own copy of the array
// (at its own address) until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per GPU
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on the current device (resolved once per
// device with hipGetSymbolAddress, that device being current) and its size.
// Host code must use this address, never the array's name, wherever it
// needs the array's memory.
extern "C" hipError_t lme_internal_noalloc_scratch(void **ptr, size_t *bytes) {
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = kScratchBytes;
  return hipSuccess;
}
