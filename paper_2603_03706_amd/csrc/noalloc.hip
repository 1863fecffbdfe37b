// Fixed device scratch of the no-allocation run (mm_run_noalloc).
//
// The array below is a static device variable: every GPU the library runs
// on holds its own copy for the life of the process.  Host code must not
// pass the array's name to a kernel (on the host it names a stand-in, not
// device memory); it asks for the device address once per device, with that
// device current, and uses only that address.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "mmcav.h"
#include "launch.h"

namespace {

static __device__ __align__(256) unsigned char scratch[MM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_lookup_mu;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_run_mu[kMaxDevices];

__global__ void k_fill_zero(uint4* __restrict__ p, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

}  // namespace

// Device address of this device's scratch array (looked up on the first call
// for the device, which must be current) and its size in bytes.
hipError_t mmk_noalloc_scratch(int dev, void** ptr, size_t* bytes) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_lookup_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  *bytes = MM_NOALLOC_SCRATCH_BYTES;
  return hipSuccess;
}

// Lock that serialises the no-allocation runs of one process on one device.
std::mutex& mmk_noalloc_lock(int dev) { return g_run_mu[dev < 0 || dev >= kMaxDevices ? 0 : dev]; }

// Zero `bytes` (a multiple of 16) at the 16-byte aligned device address p
// with a fill kernel on stream s.
hipError_t mmk_launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  const size_t blocks = (n16 + 255) / 256;
  MM_LAUNCH(k_fill_zero, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, (uint4*)p, n16);
  return hipGetLastError();
}
