// The allocation-free CCMM entry point: hfe_ccmm's lift, contraction and rescale with the call's
// device buffers (query planes, contraction output or small-modulus residues) carved from one
// static device array instead of the allocator, for callers that cannot allocate device memory
// (code under stream capture, tight serving loops, harnesses that forbid it).
//
// The array is a file-scope __device__ variable: every GPU the library runs on holds its own copy
// at its own address from the load of this code object until the process ends.  Host code never
// passes the array's name to the device; it resolves the address once per device with
// hipGetSymbolAddress (with that device current) and passes that pointer.
#include <mutex>

#include "hfe_internal.h"

namespace hfe {
namespace {

__device__ __align__(256) uint8_t scratch[HFE_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's copy of `scratch`, resolved on first use (device `dev` current).
hfe_status scratch_for(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(HFE_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> l(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(HFE_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HFE_OK;
}

}  // namespace
}  // namespace hfe

using namespace hfe;

hfe_status hfe_noalloc_init(void) {
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(HFE_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  }
  void* ptr = nullptr;
  return scratch_for(dev, &ptr);
}

hfe_status hfe_ccmm_noalloc(const hfe_db* db, const hfe_qct* q, int64_t row0, int64_t rows, int32_t form,
                            uint64_t* out, void* stream) {
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(HFE_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  }
  void* ptr = nullptr;
  HFE_TRY(scratch_for(dev, &ptr));
  return ccmm_region(db, q, row0, rows, form, (hipStream_t)stream, out, ptr, (size_t)HFE_NOALLOC_SCRATCH_BYTES);
}
