// Fixed device scratch of lddmm_shoot_grad_noalloc: the workspace of one
// loss+gradient evaluation (trajectory, FP64 state and adjoint, partial sums)
// lives in a file-scope device array instead of a buffer the context
// allocates.  Each GPU the library runs on holds its own copy of the array
// from module load until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device (hipGetSymbolAddress, with that
// device current) and only that address is handed to kernels.
#include "shoot_internal.h"

#include <mutex>
#include <vector>

namespace lddmm {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void** out) {
  static std::mutex mu;
  static std::vector<void*> addr;   // per device ordinal; null until looked up
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((size_t)device < addr.size() && addr[device]) {
    *out = addr[device];
    return hipSuccess;
  }
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return e;
  if ((size_t)device >= addr.size()) addr.resize((size_t)device + 1, nullptr);
  addr[device] = p;
  *out = p;
  return hipSuccess;
}

}  // namespace lddmm
