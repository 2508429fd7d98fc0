// The fixed device area behind polar_scl_decode_batch_noalloc, the decode
// entry point for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops).  The area is a file-scope device
// array: every GPU the library runs on holds its own copy, at its own
// address, until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in for the symbol); it looks
// the device address up once per device and passes that.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/polar_scl.h"
#include "batch.h"

namespace {

static __device__ __align__(256) unsigned char scratch[polar::kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_base[kMaxDevices] = {};

constexpr uint32_t kPtrPack = 256;  // pointers per launch (2 KB of kernel arguments)
struct PtrPack {
  const void* p[kPtrPack];
};

__global__ void __launch_bounds__(kPtrPack) k_store_ptrs(const void** dst, PtrPack pk, uint32_t n) {
  const uint32_t i = threadIdx.x;
  if (i < n) dst[i] = pk.p[i];
}

}  // namespace

namespace polar {

int noalloc_area(char** base) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return POLAR_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return POLAR_EUNSUP;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_base[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return POLAR_EHIP;
    g_base[dev] = static_cast<char*>(p);
  }
  *base = g_base[dev];
  return POLAR_OK;
}

int launch_store_ptrs(const void** dst, const void* const* src, uint32_t n, hipStream_t s) {
  for (uint32_t i = 0; i < n; i += kPtrPack) {
    PtrPack pk{};
    const uint32_t m = n - i < kPtrPack ? n - i : kPtrPack;
    for (uint32_t j = 0; j < m; ++j) pk.p[j] = src[i + j];
    hipLaunchKernelGGL(k_store_ptrs, dim3(1), dim3(kPtrPack), 0, s, dst + i, pk, m);
    if (hipGetLastError() != hipSuccess) return POLAR_EHIP;
  }
  return POLAR_OK;
}

}  // namespace polar
