// Face-slot workspace of the allocation-free operator apply
// (sdg_apply_velocity_operator_noalloc): a file-scope device array, one copy
// per GPU, held until the process ends.  Host code never passes the array's
// name to a kernel (in host code it is only a stand-in); it resolves the
// array's device address once per device with hipGetSymbolAddress, with that
// device current, and passes that address.
#include <mutex>
#include <vector>

#include "context.hpp"

namespace sdg {

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // 256 MiB per GPU

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // device address per device (null: not resolved yet)

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Device address of this device's copy of the scratch array; resolved on
// the first call for a device (which must be the current device).
void* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    SDG_HIP(hipGetDevice(&cur));
    require(cur == device, SDG_EDEVICE, "the scratch array is resolved with its device current");
    void* ptr = nullptr;
    SDG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    require(ptr != nullptr, SDG_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

}  // namespace sdg
