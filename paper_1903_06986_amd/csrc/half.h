// 16-bit storage of FP32 spinor fields with one scale per site.
//
// A stored half field (one parity, Vh sites, 12 complex components c =
// spin * 3 + colour) is a uint32 array:
//   words [0, 12 Vh):      16-byte granules [3][Vh][4]: component c of site
//                          i at word hword(c, i, Vh) = 4 ((c / 4) Vh + i) +
//                          c % 4, the real part in the low 16 bits, the
//                          imaginary part in the high 16 bits, each value
//                          divided by the site's scale (a stencil lane
//                          gathers a site with three 16-byte loads);
//   words [12 Vh, 13 Vh):  the FP32 scale of site i (bit pattern): the
//                          largest |re| or |im| over its 24 reals.
// Stored values therefore lie in [-1, 1], where FP16 keeps 11 significant
// bits without underflow for the large components of every site, and BF16
// keeps 8.  Arithmetic stays FP32.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cplx.h"

namespace lqcd {

enum class HKind { F16 = 0, BF16 = 1 };

template <HKind K>
struct Codec;

template <>
struct Codec<HKind::F16> {
  __device__ static inline uint32_t pack(float re, float im) {
    const _Float16 a = static_cast<_Float16>(re), b = static_cast<_Float16>(im);  // round to nearest even
    uint16_t ua, ub;
    __builtin_memcpy(&ua, &a, 2);
    __builtin_memcpy(&ub, &b, 2);
    return uint32_t(ua) | (uint32_t(ub) << 16);
  }
  __device__ static inline cx<float> unpack(uint32_t v) {
    const uint16_t ua = uint16_t(v & 0xffffu), ub = uint16_t(v >> 16);
    _Float16 a, b;
    __builtin_memcpy(&a, &ua, 2);
    __builtin_memcpy(&b, &ub, 2);
    return mk(static_cast<float>(a), static_cast<float>(b));
  }
};

template <>
struct Codec<HKind::BF16> {
  // round to nearest even on the upper 16 bits of the FP32 pattern (finite
  // inputs; the stored values are bounded by 1)
  __device__ static inline uint32_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
  }
  __device__ static inline uint32_t pack(float re, float im) {
    return to_bf16(re) | (to_bf16(im) << 16);
  }
  __device__ static inline cx<float> unpack(uint32_t v) {
    return mk(__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u));
  }
};

__host__ __device__ inline size_t hword(int c, size_t i, size_t Vh) {
  return 4 * ((size_t(c) >> 2) * Vh + i) + (size_t(c) & 3);
}

// Words of one stored half field of Vh sites, rounded up to 256 bytes so
// that consecutive vectors of a basis stay aligned.
inline size_t hvec_words(size_t Vh) {
  const size_t w = 13 * Vh;
  return (w + 63) / 64 * 64;
}

}  // namespace lqcd
