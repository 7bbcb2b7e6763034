// Buffer loads and stores: a 32-bit byte offset from a base held in scalar
// registers (the buffer resource), instead of a 64-bit address per lane.
#pragma once

#include <hip/hip_runtime.h>

namespace ldq {

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ inline float buf_ld(float *, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
__device__ inline double buf_ld(double *, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
__device__ inline void buf_st(float v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, vo, so, 0);
}
__device__ inline void buf_st(double v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, vo, so, 0);
}

}  // namespace ldq
