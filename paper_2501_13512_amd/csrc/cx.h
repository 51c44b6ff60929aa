// Complex arithmetic for device code (float and double), plain structs that
// match the interleaved (re, im) memory layout of C99 _Complex and of
// torch.complex64 / complex128.
#pragma once
#include <hip/hip_runtime.h>

template <typename R>
struct __attribute__((aligned(2 * sizeof(R)))) cx {
  R x, y;
};

using c64 = cx<float>;
using c128 = cx<double>;

template <typename R>
__host__ __device__ __forceinline__ cx<R> mk(R a, R b) {
  cx<R> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) {
  return mk<R>(a.x + b.x, a.y + b.y);
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) {
  return mk<R>(a.x - b.x, a.y - b.y);
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) {
  return mk<R>(s * a.x, s * a.y);
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> conj(cx<R> a) {
  return mk<R>(a.x, -a.y);
}
// a * (+i) and a * (-i)
template <typename R>
__host__ __device__ __forceinline__ cx<R> mul_i(cx<R> a) {
  return mk<R>(-a.y, a.x);
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> mul_mi(cx<R> a) {
  return mk<R>(a.y, -a.x);
}
// conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ cx<R> cdot1(cx<R> a, cx<R> b) {
  return mk<R>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename R>
__host__ __device__ __forceinline__ R abs2(cx<R> a) {
  return a.x * a.x + a.y * a.y;
}
template <typename D, typename S>
__host__ __device__ __forceinline__ cx<D> cvt(cx<S> a) {
  return mk<D>(static_cast<D>(a.x), static_cast<D>(a.y));
}
