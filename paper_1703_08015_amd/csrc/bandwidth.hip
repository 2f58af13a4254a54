// Achievable-bandwidth reference of the step: a device copy written for
// gfx950.  Each thread moves 16 bytes per access with non-temporal loads and
// stores (the data is touched once), four independent accesses in flight per
// thread, and the grid is a fixed number of workgroups per compute unit that
// strides over the buffers, so the copy runs at the rate the memory system
// sustains for one read and one write stream rather than at a rate set by
// workgroup launch.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

using lbm::set_error;

namespace {

typedef unsigned v4u __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kUnroll = 4;
constexpr int kBlocksPerCU = 8;

__global__ void __launch_bounds__(kThreads) k_copy16(v4u *__restrict__ dst, const v4u *__restrict__ src, int64_t n) {
  const int64_t G = (int64_t)gridDim.x * kThreads;
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  for (; i + (kUnroll - 1) * G < n; i += kUnroll * G) {
    v4u v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(src + i + u * G);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) __builtin_nontemporal_store(v[u], dst + i + u * G);
  }
  for (; i < n; i += G) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

extern "C" int lbm_device_copy(void *dst, const void *src, size_t bytes, void *stream) {
  if (!dst || !src) return set_error(LBM_ERR_ARG, "lbm_device_copy: NULL buffer");
  if (((uintptr_t)dst | (uintptr_t)src | bytes) % 16)
    return set_error(LBM_ERR_ARG, "lbm_device_copy: buffers and size must be multiples of 16 bytes");
  const uintptr_t d = (uintptr_t)dst, s = (uintptr_t)src;
  if (d < s + bytes && s < d + bytes) return set_error(LBM_ERR_ARG, "lbm_device_copy: buffers overlap");
  if (bytes == 0) return LBM_OK;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return set_error(LBM_ERR_HIP, "lbm_device_copy: %s", hipGetErrorString(e));
  const int64_t n = (int64_t)(bytes / 16);
  int64_t blocks = (int64_t)cus * kBlocksPerCU;
  const int64_t need = (n + kThreads - 1) / kThreads;
  if (blocks > need) blocks = need;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(kThreads), 0, static_cast<hipStream_t>(stream),
                     static_cast<v4u *>(dst), static_cast<const v4u *>(src), n);
  e = hipGetLastError();
  if (e != hipSuccess) return set_error(LBM_ERR_HIP, "lbm_device_copy: %s", hipGetErrorString(e));
  return LBM_OK;
}
