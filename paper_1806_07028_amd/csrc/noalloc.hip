// Path orientation (Alg. 3, Steps 5-7: every path of a cover walked from its
// smaller end) for callers that cannot allocate device memory: the pointer-
// jumping workspace lives in a fixed device array of this library instead of
// coming from the allocator.  Each GPU holds its own copy of the array from
// the first call on it until the process ends; calls that overlap on one GPU
// share it and race.
#include <mutex>

#include "solver.hpp"

namespace pcamg {
namespace {

constexpr int32_t NOALLOC_MAX_N = PCAMG_ORIENT_NOALLOC_MAX_N;
constexpr size_t SCRATCH_INTS = 12 * (size_t)NOALLOC_MAX_N + 1;  // = orient_ws_ints(NOALLOC_MAX_N)

// The workspace.  In host code this name is not a device address: kernels
// receive the address looked up for the current device below.
__device__ __align__(256) int32_t scratch[SCRATCH_INTS];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
int32_t* g_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per device.
int32_t* scratch_ptr() {
  int dev = 0;
  PCAMG_HIP(hipGetDevice(&dev));
  require(dev >= 0 && dev < MAX_DEVICES, PCAMG_EUNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    PCAMG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    require(p != nullptr, PCAMG_EHIP, "no device address for the orientation workspace");
    g_ptr[dev] = static_cast<int32_t*>(p);
  }
  return g_ptr[dev];
}

}  // namespace

int32_t* orient_noalloc_scratch() { return scratch_ptr(); }

}  // namespace pcamg
