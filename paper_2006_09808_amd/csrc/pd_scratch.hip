// pd_scratch.hip - the library's fixed device scratch for the entry point
// that allocates nothing (pd_apply_kernel_noalloc in pd.h).
//
// A file-scope device array: every GPU the library runs on holds its own copy
// from the moment the code object is loaded until the process ends.  Host
// code never passes the array's name to a kernel or a copy (on the host it
// is only a stand-in symbol); the device address of each GPU's copy comes
// from hipGetSymbolAddress, taken once per device by pd_create with that
// device current, and is what the kernels receive.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pd.h"

namespace pdk {

static __device__ __align__(256) unsigned char scratch[PD_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
std::mutex g_use[kMaxDevices];
}  // namespace

// Device address of `device`'s copy of the scratch array; the device must be
// current.  Looked up once per device, then cached.
hipError_t static_scratch(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

// Calls that use one device's scratch hold this lock for their whole
// duration, so two contexts of one process never overlap in it.
std::mutex& static_scratch_lock(int device) { return g_use[device < 0 || device >= kMaxDevices ? 0 : device]; }

}  // namespace pdk
