// Element Hessians for callers that cannot allocate device memory during a
// call: the device staging of ppn_eval_element_hessians (the element ids in,
// the 12x12 matrices out before their copy to the caller's host buffer) lives
// in one file-scope device array instead of two allocations per call.
//
// Every GPU the library runs on holds its own copy of `scratch` until the
// process ends.  Its name is not a device address in host code: the address of
// a device's copy is taken once, with that device current, through
// hipGetSymbolAddress and kept per device; only that address is handed to
// copies and kernels.  Calls on one GPU share the array, so they are
// serialised per device here (the call is synchronous: it returns after the
// copy back to the host); nothing in it has to start at zero, because every
// call writes the part it reads.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "scene.h"

namespace ppn {

constexpr size_t kScratchIdsBytes = size_t(kNoAllocMaxElements) * sizeof(int32_t);
constexpr size_t kScratchBytes = kScratchIdsBytes + size_t(kNoAllocMaxElements) * 144 * sizeof(double);
static_assert(kScratchIdsBytes % 256 == 0, "the matrices start 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct DeviceScratch {
  std::mutex use;       // held for the whole of a call on this device
  void* ptr = nullptr;  // this device's copy of scratch
};

std::mutex g_table_mu;
std::map<int, DeviceScratch> g_table;

// The entry for `device`, with its address resolved (that device current).
DeviceScratch& scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_table_mu);
  DeviceScratch& d = g_table[device];
  if (!d.ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw HipError{std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e),
                     PPN_ERR_DEVICE};
    d.ptr = p;
  }
  return d;
}

// Makes `device` current for the call and restores the previous one.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int device) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != device) {
      const hipError_t e = hipSetDevice(device);
      if (e != hipSuccess)
        throw HipError{std::string("hipSetDevice: ") + hipGetErrorString(e), PPN_ERR_DEVICE};
    }
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

void Scene::eval_element_hessians_noalloc(const double* x, const uint8_t* mask, int32_t n,
                                          const int32_t* ids, double* out) {
  if (!out) throw HipError{"H_out must not be NULL", PPN_ERR_ARG};
  n = element_hessians_count(n, ids);
  if (n > kNoAllocMaxElements)
    throw HipError{"n = " + std::to_string(n) + " element Hessians exceed the no-allocation limit of " +
                       std::to_string(kNoAllocMaxElements) + " per call",
                   PPN_ERR_ARG};
  DeviceGuard dg(device_);
  DeviceScratch& d = scratch_of(device_);
  std::lock_guard<std::mutex> lk(d.use);
  unsigned char* base = static_cast<unsigned char*>(d.ptr);
  eval_element_hessians_staged(x, mask, n, ids, reinterpret_cast<int32_t*>(base),
                               reinterpret_cast<double*>(base + kScratchIdsBytes), out);
}

}  // namespace ppn
