// Plain device-to-device streaming copy: the practical HBM ceiling that the
// sweeps' achieved bandwidth is compared with (no stencil, no arithmetic,
// every byte read once and written once).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace oreg {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// One 16-byte word per thread; stores bypass the caches on the way out, as
// the sweeps' stores do.
__global__ __launch_bounds__(256) void copy_kernel(const u32x4* __restrict__ src,
                                                   u32x4* __restrict__ dst, int64_t words) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < words) __builtin_nontemporal_store(src[i], &dst[i]);
}

}  // namespace

hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t s) {
  const int64_t words = bytes / 16;
  if (words <= 0) return hipSuccess;
  const int64_t blocks = (words + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  copy_kernel<<<(unsigned int)blocks, 256, 0, s>>>(static_cast<const u32x4*>(src),
                                                   static_cast<u32x4*>(dst), words);
  return hipGetLastError();
}

}  // namespace oreg
