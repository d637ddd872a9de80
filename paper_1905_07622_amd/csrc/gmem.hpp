// Explicit global-memory accesses for the gfx950 kernels.
//
// Pointers that a kernel reads from memory (the per-simulation records of a
// batch, the relay state) are generic pointers to the compiler, which then
// emits FLAT instructions for them.  A flat access counts against the LDS
// counter as well as the vector-memory counter, so every wait for an LDS
// read also waits for every flat load still in flight: a gather that issues
// the next planes' loads and then reads the current plane from LDS would
// wait for those loads at once, and its prefetch would hide nothing.
//
// gld/gst address global memory explicitly, as a uniform base plus a 32-bit
// byte offset (the scalar-base form of the global instructions: no 64-bit
// address arithmetic per lane).  The caller keeps element offsets below
// 2^32 / sizeof(T) (the library bounds node and element counts).  gld_at /
// gst_at take a per-lane address (e.g. a select between a vector and a sink).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace femheat {

#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
using gcptr = const __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ T gld(const T* base, uint32_t i) {
  gcptr<char> b = (gcptr<char>)base;
  return *(gcptr<T>)(b + (uint32_t)(i * (uint32_t)sizeof(T)));
}

template <typename T>
__device__ __forceinline__ void gst(T* base, uint32_t i, T v) {
  gptr<char> b = (gptr<char>)base;
  *(gptr<T>)(b + (uint32_t)(i * (uint32_t)sizeof(T))) = v;
}

// Records larger than 16 bytes (the relay state) move as 8-byte words: an
// aggregate copy would become a memory copy that loses the address space.
template <typename T>
__device__ __forceinline__ T gld_at(const T* p) {
  if constexpr (sizeof(T) > 16 && sizeof(T) % 8 == 0) {
    uint64_t w[sizeof(T) / 8];
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 8); ++k) w[k] = ((gcptr<uint64_t>)p)[k];
    T v;
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
  } else {
    return *(gcptr<T>)p;
  }
}

template <typename T>
__device__ __forceinline__ void gst_at(T* p, T v) {
  if constexpr (sizeof(T) > 16 && sizeof(T) % 8 == 0) {
    uint64_t w[sizeof(T) / 8];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 8); ++k) ((gptr<uint64_t>)p)[k] = w[k];
  } else {
    *(gptr<T>)p = v;
  }
}

#else
// The host pass only checks the kernels' source; it never runs them.
template <typename T>
__device__ T gld(const T* base, uint32_t i) {
  return base[i];
}
template <typename T>
__device__ void gst(T* base, uint32_t i, T v) {
  base[i] = v;
}
template <typename T>
__device__ T gld_at(const T* p) {
  return *p;
}
template <typename T>
__device__ void gst_at(T* p, T v) {
  *p = v;
}
#endif

}  // namespace femheat
