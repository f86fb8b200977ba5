// HBM streaming-copy probe: the bandwidth a plain copy reaches on this part, measured beside
// the solver's sweeps so their roofline fractions can be read against it.  Each lane keeps
// `U` 16-byte loads in flight, then writes them with non-temporal stores (the destination is
// not read again); consecutive lanes touch consecutive 16-byte words (coalesced), and the
// grid strides over the buffer.
#include <hip/hip_runtime.h>

#include <string>

#include "chf_internal.h"

namespace {

template <int U>
__global__ void __launch_bounds__(256) k_stream_copy(uint4 *__restrict__ dst, const uint4 *__restrict__ src,
                                                     long long n16) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const long long span = (long long)gridDim.x * blockDim.x * U;
  for (long long base = (long long)blockIdx.x * blockDim.x * U + threadIdx.x; base < n16; base += span) {
    u4 v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const long long i = base + (long long)u * blockDim.x;
      if (i < n16) {
        const uint4 x = src[i];
        v[u] = u4{x.x, x.y, x.z, x.w};
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const long long i = base + (long long)u * blockDim.x;
      if (i < n16) __builtin_nontemporal_store(v[u], reinterpret_cast<u4 *>(dst + i));
    }
  }
}

}  // namespace

extern "C" chf_status chf_stream_copy(void *dst_dev, const void *src_dev, uint64_t bytes, int32_t loads_in_flight,
                                      int32_t blocks, void *stream) {
  if (!dst_dev || !src_dev || bytes % 16 || (uintptr_t)dst_dev % 16 || (uintptr_t)src_dev % 16 || blocks < 1) {
    chf::set_error("chf_stream_copy: NULL or misaligned buffer, size not a multiple of 16, or blocks < 1");
    return CHF_EINVAL;
  }
  const long long n16 = (long long)(bytes / 16);
  hipStream_t s = (hipStream_t)stream;
  uint4 *d = (uint4 *)dst_dev;
  const uint4 *a = (const uint4 *)src_dev;
  switch (loads_in_flight) {
    case 1: hipLaunchKernelGGL(k_stream_copy<1>, dim3(blocks), dim3(256), 0, s, d, a, n16); break;
    case 2: hipLaunchKernelGGL(k_stream_copy<2>, dim3(blocks), dim3(256), 0, s, d, a, n16); break;
    case 4: hipLaunchKernelGGL(k_stream_copy<4>, dim3(blocks), dim3(256), 0, s, d, a, n16); break;
    case 8: hipLaunchKernelGGL(k_stream_copy<8>, dim3(blocks), dim3(256), 0, s, d, a, n16); break;
    default:
      chf::set_error("chf_stream_copy: loads_in_flight must be 1, 2, 4 or 8");
      return CHF_EINVAL;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    chf::set_error(std::string("chf_stream_copy: ") + hipGetErrorString(e));
    return CHF_EHIP;
  }
  return CHF_OK;
}
