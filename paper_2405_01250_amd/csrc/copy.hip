// copy.hip -- device-to-device copy by a streaming kernel: the circuit
// drivers' state copies (scratch -> state, psi0 -> psi) and, exported as
// diaq_copy, the plain-copy reference of the bandwidth measurements; and a
// zero fill (a kernel rather than a memset, so that recorded circuit graphs
// hold no memset node).
#include "internal.hpp"

namespace diaq {

namespace {

constexpr int kBlock = 256;

// One 16-byte vector per lane, full grid, non-temporal loads and stores
// (the fastest shape measured: 6.44 TB/s at 4 GiB, 6.16 without the hints).
__global__ __launch_bounds__(kBlock) void copy16_kernel(int64_t n16, const double2* __restrict__ src,
                                                       double2* __restrict__ dst) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n16) {
    typedef double N2 __attribute__((ext_vector_type(2)));
    const N2 t = __builtin_nontemporal_load(reinterpret_cast<const N2*>(src + i));
    __builtin_nontemporal_store(t, reinterpret_cast<N2*>(dst + i));
  }
}

__global__ __launch_bounds__(kBlock) void zero16_kernel(int64_t n16, double2* __restrict__ dst) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n16) dst[i] = double2{0.0, 0.0};
}

}  // namespace

diaq_status_t launch_zero(hipStream_t stream, void* dst, size_t bytes) {
  if (bytes == 0) return DIAQ_OK;
  if ((reinterpret_cast<uintptr_t>(dst) | bytes) & 15)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "fill needs a 16-byte aligned pointer and a multiple of 16 bytes");
  const int64_t n16 = int64_t(bytes / 16);
  const int64_t blocks = (n16 + kBlock - 1) / kBlock;
  if (blocks > 0x7fffffffLL) return fail(DIAQ_ERR_UNSUPPORTED, "fill of %zu bytes", bytes);
  hipLaunchKernelGGL(zero16_kernel, dim3(unsigned(blocks)), dim3(kBlock), 0, stream, n16, static_cast<double2*>(dst));
  DIAQ_HIP(hipGetLastError());
  return DIAQ_OK;
}

diaq_status_t launch_copy(hipStream_t stream, const void* src, void* dst, size_t bytes) {
  if (bytes == 0) return DIAQ_OK;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst) | bytes) & 15)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "copy needs 16-byte aligned pointers and a multiple of 16 bytes");
  const char* s = static_cast<const char*>(src);
  char* d = static_cast<char*>(dst);
  if (s < d + bytes && d < s + bytes) return fail(DIAQ_ERR_INVALID_ARGUMENT, "copy source and destination overlap");
  const int64_t n16 = int64_t(bytes / 16);
  const int64_t blocks = (n16 + kBlock - 1) / kBlock;
  if (blocks > 0x7fffffffLL) return fail(DIAQ_ERR_UNSUPPORTED, "copy of %zu bytes", bytes);
  hipLaunchKernelGGL(copy16_kernel, dim3(unsigned(blocks)), dim3(kBlock), 0, stream, n16,
                     static_cast<const double2*>(src), static_cast<double2*>(dst));
  DIAQ_HIP(hipGetLastError());
  return DIAQ_OK;
}

}  // namespace diaq
