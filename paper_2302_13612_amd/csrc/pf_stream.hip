// Streaming copy: the attainable HBM rate of a kernel that does nothing but
// move bytes, the reference beside which the passes' rates are read (the
// 8 TB/s datasheet figure stays the roofline's peak). Each lane moves 16
// bytes per access with the nontemporal hint on both sides, grid-stride over
// a grid of many blocks (65536 x 512 threads measured best on this part:
// 6.5 TB/s read + write for 1 GiB).
#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/pf.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kStreamThreads = 512;
constexpr unsigned kStreamBlocks = 65536;

__global__ __launch_bounds__(kStreamThreads) void k_stream_copy(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                                                size_t n) {
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

extern "C" int pf_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src || bytes % 16 || (reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16)
    return PF_EINVAL;
  const size_t n = bytes / 16;
  if (n == 0) return PF_OK;
  const unsigned blocks = (unsigned)((n + kStreamThreads - 1) / kStreamThreads < kStreamBlocks
                                         ? (n + kStreamThreads - 1) / kStreamThreads
                                         : kStreamBlocks);
  k_stream_copy<<<blocks, kStreamThreads, 0, reinterpret_cast<hipStream_t>(hip_stream)>>>(
      reinterpret_cast<const v4f*>(src), reinterpret_cast<v4f*>(dst), n);
  return hipGetLastError() == hipSuccess ? PF_OK : PF_EDEVICE;
}
