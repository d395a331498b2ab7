// Fixed device scratch of the allocation-free entry point
// (dm_mesh_transform_noalloc).  The array lives in the library's code object:
// every GPU the library runs on holds its own copy, at its own address, until
// the process ends.  Host code never uses the array's name as a device
// address: dm_create resolves the address once per device (with that device
// current) and the entry point passes that pointer to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/deltamic.h"
#include "dm_internal.h"

namespace dm {

namespace {

__device__ __align__(256) char scratch[DM_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // per device, nullptr until resolved

}  // namespace

hipError_t scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((size_t)device >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)device + 1, nullptr);
  if (g_scratch_ptr[(size_t)device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;   // the caller makes the device current
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[(size_t)device] = p;
  return hipSuccess;
}

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || (size_t)device >= g_scratch_ptr.size()) return nullptr;
  return g_scratch_ptr[(size_t)device];
}

}  // namespace dm
