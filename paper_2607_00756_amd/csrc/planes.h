// Storage of complex contraction operands as separate real planes.
//
//   FP32        : re, im                      (4-byte elements)
//   SPLIT_BF16  : re_hi, re_lo, im_hi, im_lo   (2-byte elements; lo = bf16 of
//                 the residual x - hi, so hi + lo carries ~16 mantissa bits)
//   BF16        : re, im                      (2-byte elements)
//   FP16        : re, im                      (2-byte IEEE half elements)
//
// Element idx of plane k sits at idx + k * plane (in elements).
#pragma once

#include "bip_internal.h"

namespace bip {

__device__ inline uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ inline uint16_t f2h(float f) { return __builtin_bit_cast(uint16_t, (_Float16)f); }
__device__ inline float h2f(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

template <int PREC>
__device__ inline void store_planes(void* out, int64_t idx, int64_t plane, float re, float im) {
  if constexpr (PREC == BIP_PREC_FP32) {
    float* o = (float*)out;
    o[idx] = re;
    o[idx + plane] = im;
  } else if constexpr (PREC == BIP_PREC_SPLIT_BF16) {
    uint16_t* o = (uint16_t*)out;
    const uint16_t rh = f2bf(re), ih = f2bf(im);
    o[idx] = rh;
    o[idx + plane] = f2bf(re - bf2f(rh));
    o[idx + 2 * plane] = ih;
    o[idx + 3 * plane] = f2bf(im - bf2f(ih));
  } else if constexpr (PREC == BIP_PREC_FP16) {
    uint16_t* o = (uint16_t*)out;
    o[idx] = f2h(re);
    o[idx + plane] = f2h(im);
  } else {
    uint16_t* o = (uint16_t*)out;
    o[idx] = f2bf(re);
    o[idx + plane] = f2bf(im);
  }
}

template <int PREC>
__device__ inline float2 load_planes(const void* in, int64_t idx, int64_t plane) {
  if constexpr (PREC == BIP_PREC_FP32) {
    const float* o = (const float*)in;
    return make_float2(o[idx], o[idx + plane]);
  } else if constexpr (PREC == BIP_PREC_SPLIT_BF16) {
    const uint16_t* o = (const uint16_t*)in;
    return make_float2(bf2f(o[idx]) + bf2f(o[idx + plane]),
                       bf2f(o[idx + 2 * plane]) + bf2f(o[idx + 3 * plane]));
  } else if constexpr (PREC == BIP_PREC_FP16) {
    const uint16_t* o = (const uint16_t*)in;
    return make_float2(h2f(o[idx]), h2f(o[idx + plane]));
  } else {
    const uint16_t* o = (const uint16_t*)in;
    return make_float2(bf2f(o[idx]), bf2f(o[idx + plane]));
  }
}

}  // namespace bip
