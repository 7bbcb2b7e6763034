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

// Two consecutive elements per lane (8-byte / 16-byte accesses).
template <typename T>
struct Pair {
  T a, b;
};
// (the 8-byte forms go through a 64-bit integer: indexing the two-element
// vector the b64 builtin returns reads the low dword twice)
__device__ inline Pair<float> buf_ld2(float *, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  const unsigned long long v = __builtin_bit_cast(unsigned long long, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
  return Pair<float>{__builtin_bit_cast(float, (unsigned)(v & 0xffffffffull)), __builtin_bit_cast(float, (unsigned)(v >> 32))};
}
__device__ inline Pair<double> buf_ld2(double *, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0);
  const unsigned long long a = ((unsigned long long)(unsigned)v[1] << 32) | (unsigned)v[0];
  const unsigned long long b = ((unsigned long long)(unsigned)v[3] << 32) | (unsigned)v[2];
  return Pair<double>{__builtin_bit_cast(double, a), __builtin_bit_cast(double, b)};
}
__device__ inline void buf_st2(Pair<float> v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
  const unsigned long long w = ((unsigned long long)__builtin_bit_cast(unsigned, v.b) << 32) |
                               (unsigned long long)__builtin_bit_cast(unsigned, v.a);
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, w), r, vo, so, 0);
}
__device__ inline void buf_st2(Pair<double> v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
  const unsigned long long a = __builtin_bit_cast(unsigned long long, v.a);
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v.b);
  V w;
  w[0] = (int)(unsigned)(a & 0xffffffffull);
  w[1] = (int)(unsigned)(a >> 32);
  w[2] = (int)(unsigned)(b & 0xffffffffull);
  w[3] = (int)(unsigned)(b >> 32);
  __builtin_amdgcn_raw_buffer_store_b128(w, r, vo, so, 0);
}

}  // namespace ldq
