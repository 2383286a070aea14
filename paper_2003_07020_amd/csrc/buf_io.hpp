// Raw buffer access for the FFT kernels (gfx9 descriptor with a 4-byte data format, so the
// hardware range check applies): an access whose byte range is not inside [0, nbytes) reads
// zero or is dropped.
#pragma once
#include <hip/hip_runtime.h>

namespace rfde {

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, nbytes, 0x00020000);
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, int idx) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, idx * 8, 0, 0));
}
// complex element idx of a double2 or float2 buffer
template <typename C> __device__ __forceinline__ C buf_load_c(__amdgpu_buffer_rsrc_t r, int idx) {
  if constexpr (sizeof(C) == 16)
    return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128(r, idx * 16, 0, 0));
  else
    return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b64(r, idx * 8, 0, 0));
}
// real part of complex element idx of a double2 or float2 buffer
template <typename C>
__device__ __forceinline__ auto buf_load_re(__amdgpu_buffer_rsrc_t r, int idx) {
  if constexpr (sizeof(C) == 16)
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, idx * 16, 0, 0));
  else
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, idx * 8, 0, 0));
}
template <typename C>
__device__ __forceinline__ void buf_store_c(__amdgpu_buffer_rsrc_t r, int idx, C x) {
  if constexpr (sizeof(C) == 16) {
    using V4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4, x), r, idx * 16, 0, 0);
  } else {
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, x), r, idx * 8, 0, 0);
  }
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, int idx, double x) {
  using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, x), r, idx * 8, 0, 0);
}

}  // namespace rfde
