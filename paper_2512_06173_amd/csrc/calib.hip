// Bandwidth calibration: a plain streaming copy of known size, the yardstick for
// what the HBM of this part sustains under a simple read-once / write-once stream
// (the fused sweep's access pattern at its simplest).  Each thread moves UNROLL
// 16-byte words per pass, all loads issued before the first store so that many
// bytes are in flight; variants differ in the cache policy of the loads and
// stores.
#include "mlk.h"
#include <hip/hip_runtime.h>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kThreads = 256;
constexpr int kUnroll = 8;

template <bool NT_LOAD, bool NT_STORE>
__global__ __launch_bounds__(kThreads) void k_copy(const f4* __restrict__ src,
                                                   f4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * kThreads * kUnroll;
  for (size_t base = (size_t)blockIdx.x * kThreads * kUnroll + threadIdx.x; base < n;
       base += stride) {
    f4 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const size_t q = base + (size_t)u * kThreads;
      if (q < n) v[u] = NT_LOAD ? __builtin_nontemporal_load(&src[q]) : src[q];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const size_t q = base + (size_t)u * kThreads;
      if (q < n) {
        if (NT_STORE) __builtin_nontemporal_store(v[u], &dst[q]);
        else dst[q] = v[u];
      }
    }
  }
}

}  // namespace

extern "C" mlk_status mlk_stream_copy(const void* src, void* dst, size_t bytes, int32_t variant,
                                      int32_t blocks, void* stream) {
  if (!src || !dst || bytes % 16 != 0 || variant < 0 || variant > 3 || blocks <= 0)
    return MLK_EINVAL;
  const size_t n = bytes / 16;
  const hipStream_t st = (hipStream_t)stream;
  const f4* s = (const f4*)src;
  f4* d = (f4*)dst;
  switch (variant) {
    case 0: hipLaunchKernelGGL((k_copy<false, false>), dim3(blocks), dim3(kThreads), 0, st, s, d, n); break;
    case 1: hipLaunchKernelGGL((k_copy<false, true>), dim3(blocks), dim3(kThreads), 0, st, s, d, n); break;
    case 2: hipLaunchKernelGGL((k_copy<true, false>), dim3(blocks), dim3(kThreads), 0, st, s, d, n); break;
    default: hipLaunchKernelGGL((k_copy<true, true>), dim3(blocks), dim3(kThreads), 0, st, s, d, n); break;
  }
  return hipGetLastError() == hipSuccess ? MLK_OK : MLK_EDEVICE;
}
