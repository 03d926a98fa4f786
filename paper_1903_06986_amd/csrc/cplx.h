// Minimal complex arithmetic for device code (double and float), with
// 8/16-byte vector loads and stores of interleaved (re, im) pairs.
#pragma once

#include <hip/hip_runtime.h>

namespace lqcd {

template <class R>
struct vec2;
template <>
struct vec2<double> {
  using type = double2;
};
template <>
struct vec2<float> {
  using type = float2;
};

template <class R>
struct cx {
  R re, im;
};

template <class R>
__host__ __device__ inline cx<R> mk(R a, R b) {
  return cx<R>{a, b};
}
template <class R>
__host__ __device__ inline cx<R> operator+(cx<R> a, cx<R> b) {
  return {a.re + b.re, a.im + b.im};
}
template <class R>
__host__ __device__ inline cx<R> operator-(cx<R> a, cx<R> b) {
  return {a.re - b.re, a.im - b.im};
}
template <class R>
__host__ __device__ inline cx<R> operator-(cx<R> a) {
  return {-a.re, -a.im};
}
template <class R>
__host__ __device__ inline cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R>
__host__ __device__ inline cx<R> operator*(R s, cx<R> a) {
  return {s * a.re, s * a.im};
}
// conj(a) * b
template <class R>
__host__ __device__ inline cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a
template <class R>
__host__ __device__ inline cx<R> iz(cx<R> a) {
  return {-a.im, a.re};
}
// -i * a
template <class R>
__host__ __device__ inline cx<R> miz(cx<R> a) {
  return {a.im, -a.re};
}

template <class R>
__device__ inline cx<R> ldc(const cx<R> *p) {
  auto v = *reinterpret_cast<const typename vec2<R>::type *>(p);
  return {v.x, v.y};
}
template <class R>
__device__ inline void stc(cx<R> *p, cx<R> a) {
  typename vec2<R>::type v;
  v.x = a.re;
  v.y = a.im;
  *reinterpret_cast<typename vec2<R>::type *>(p) = v;
}

}  // namespace lqcd
