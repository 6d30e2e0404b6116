// Plane-relative global-memory access for kernels whose blocks work on one
// plane k (or march over planes) of a padded array: every access goes
// through a buffer resource of that plane and variable (a wave-uniform
// descriptor formed with scalar instructions) with a 32-bit per-thread byte
// offset within the plane.  One offset register then serves every variable
// and plane, no 64-bit vector address is formed per access, and the
// resource spans exactly one plane, so the hardware range check keeps every
// access inside it (an offset beyond the plane reads 0 and writes nothing).
//
// The compiler does not order accesses through different resources by
// itself when they may alias: callers issue a group's loads before its
// stores in program order.
#pragma once

#include "common.hpp"

namespace lesjet {

// dword 3 of a buffer descriptor on this architecture: 32-bit data format,
// no swizzle, no index
constexpr int RSRC_DW3 = 0x00020000;

// variable c of plane k (padded index k + NG) of a padded array of T
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const T* A, const Grid& g, int c, int k) {
  return __builtin_amdgcn_make_buffer_rsrc(
      (void*)(A + ((long long)c * g.vs + (long long)(k + NG) * g.plane)), (short)0,
      g.plane * (int)sizeof(T), RSRC_DW3);
}

template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// load / store variable c of plane k at byte offset `off` within the plane
template <typename T>
__device__ __forceinline__ T gld(const T* A, const Grid& g, int c, int k, unsigned off) {
  return buf_ld<T>(plane_rsrc(A, g, c, k), off);
}
template <typename T>
__device__ __forceinline__ void gst(T* A, const Grid& g, int c, int k, unsigned off, T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit elements");
  const __amdgpu_buffer_rsrc_t r = plane_rsrc(A, g, c, k);
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r, (int)off, 0, 0);
}

// byte offset of column (i, j) within a plane of a padded array of T
template <typename T>
__device__ __forceinline__ unsigned col_off(const Grid& g, int i, int j) {
  return (unsigned)((j + NG) * g.pitch + (i + NG)) * (unsigned)sizeof(T);
}

}  // namespace lesjet
