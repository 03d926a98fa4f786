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

// Non-temporal forms (streamed data that is not read again soon).
template <class R>
__device__ inline cx<R> ldc_nt(const cx<R> *p) {
  typedef R v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
  return {v.x, v.y};
}
template <class R>
__device__ inline void stc_nt(cx<R> *p, cx<R> a) {
  typedef R v2 __attribute__((ext_vector_type(2)));
  v2 v;
  v.x = a.re;
  v.y = a.im;
  __builtin_nontemporal_store(v, reinterpret_cast<v2 *>(p));
}

}  // namespace lqcd
