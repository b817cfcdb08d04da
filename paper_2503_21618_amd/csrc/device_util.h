// Device helpers shared by the kernel translation units.
#pragma once
#include "kernels.h"

namespace slrf {

constexpr int WAVE = 64;
constexpr int WG = 256;

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Read-only data (batch tables, CSR arrays) seen through the constant address
// space: a load whose address is the same on every lane then becomes a scalar
// load, and values read this way are known to be wave-uniform.  Only for memory
// that no kernel writes while it runs.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) { return (cptr<T>)p; }

// Loads a trivially copyable struct from constant memory word by word.
template <typename T>
__device__ __forceinline__ T ldc(cptr<T> p) {
  static_assert(sizeof(T) % 8 == 0 && alignof(T) >= 8, "ldc needs 8-byte words");
  union U {
    T t;
    uint64_t w[sizeof(T) / 8];
  } u;
  const cptr<uint64_t> q = (cptr<uint64_t>)p;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 8); ++k) u.w[k] = q[k];
  return u.t;
}
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> cdiv(cx<R> a, cx<R> b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    R q = b.im / b.re, den = b.re + b.im * q;
    return {(a.re + a.im * q) / den, (a.im - a.re * q) / den};
  }
  R q = b.re / b.im, den = b.re * q + b.im;
  return {(a.re * q + a.im) / den, (a.im * q - a.re) / den};
}

}  // namespace slrf
