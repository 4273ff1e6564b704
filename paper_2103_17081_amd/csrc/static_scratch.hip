// Device scratch for callers that cannot allocate (HIP graph capture, tight serving
// loops): a file-scope array each GPU holds from the moment the library's code object is
// loaded on it until the process ends.
//
// Host code never passes `scratch` itself to a kernel or a copy: in host code the name is
// a host-side stand-in, not the device address.  The address is taken once per device
// with hipGetSymbolAddress (with that device current) and cached; kernels receive that
// pointer as an ordinary argument.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "kernels.hpp"

namespace ddh {

namespace {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;   // 64 MiB per device

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

__global__ void __launch_bounds__(256) zero_words_kernel(unsigned long long* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) p[i] = 0ull;
}

}  // namespace

hipError_t static_scratch(void** ptr, size_t* bytes) {
  static std::mutex mu;
  static std::vector<void*> addr;   // device address of `scratch`, per device
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize((size_t)dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = kStaticScratchBytes;
  return hipSuccess;
}

hipError_t launch_zero_words(void* p, size_t words, hipStream_t st) {
  if (words == 0) return hipSuccess;
  const long long n = (long long)words;
  const unsigned blocks = (unsigned)std::min<long long>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(zero_words_kernel, dim3(blocks), dim3(256), 0, st, (unsigned long long*)p, n);
  return hipGetLastError();
}

}  // namespace ddh
