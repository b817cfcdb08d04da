// Device helpers shared by the kernel translation units.
#pragma once
#include "kernels.h"

namespace slrf {

constexpr int WAVE = 64;
constexpr int WG = 256;

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
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
