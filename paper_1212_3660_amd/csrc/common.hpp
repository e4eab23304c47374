// Shared device/host helpers for the shifted-Krylov library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace shk {

// ---------------------------------------------------------------- complex ---
template <typename R> struct cx { R re, im; };
using c64 = cx<float>;
using c128 = cx<double>;

template <typename R> __host__ __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __host__ __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
template <typename R> __host__ __device__ __forceinline__ R abs2(cx<R> a) { return a.re * a.re + a.im * a.im; }
// conj(a) * b
template <typename R> __host__ __device__ __forceinline__ cx<R> cdot(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R> __host__ __device__ __forceinline__ cx<R> cdiv(cx<R> a, cx<R> b) {
  // Smith's algorithm: avoids overflow in |b|^2 for widely scaled operands
  if (fabs(b.re) >= fabs(b.im)) {
    R r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  R r = b.re / b.im, d = b.im + b.re * r;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
template <typename To, typename From> __host__ __device__ __forceinline__ cx<To> cvt(cx<From> a) {
  return {static_cast<To>(a.re), static_cast<To>(a.im)};
}

// Streaming store of a complex value (non-temporal hint: written through
// rather than kept dirty in L2 until the end of the kernel).
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_nt(cx<double>* p, cx<double> v) {
  d2v t = {v.re, v.im};
  __builtin_nontemporal_store(t, reinterpret_cast<d2v*>(p));
}
__device__ __forceinline__ void st_nt(cx<float>* p, cx<float> v) {
  f2v t = {v.re, v.im};
  __builtin_nontemporal_store(t, reinterpret_cast<f2v*>(p));
}
template <bool NT, typename R> __device__ __forceinline__ void st(cx<R>* p, cx<R> v) {
  if constexpr (NT) st_nt(p, v);
  else *p = v;
}

// ----------------------------------------------------------- wave / block ---
constexpr int WAVE = 64;

template <typename T> __device__ __forceinline__ T shfl_xor(T v, int m) { return __shfl_xor(v, m, WAVE); }

// Sum a complex value over the lanes of a wave that share the same value of
// (lane % lanes_per_group): offsets >= group are folded.  group is a power of
// two <= 64.  Fixed tree order: deterministic.
template <typename R> __device__ __forceinline__ cx<R> wave_sum_strided(cx<R> v, int group) {
  for (int off = WAVE / 2; off >= group; off >>= 1) {
    v.re += shfl_xor(v.re, off);
    v.im += shfl_xor(v.im, off);
  }
  return v;
}
template <typename R> __device__ __forceinline__ R wave_sum_strided(R v, int group) {
  for (int off = WAVE / 2; off >= group; off >>= 1) v += shfl_xor(v, off);
  return v;
}

__host__ __device__ __forceinline__ int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

}  // namespace shk
