// Device helpers shared by the FCC kernels: complex arithmetic and the
// storage formats of the whitened spectra.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fcc {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmul_conj(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// ---- storage formats: one complex value per element -----------------------

struct SpecF32 { using T = float2; static constexpr int bytes = 8; };
struct SpecBF16 { using T = uint32_t; static constexpr int bytes = 4; };
struct SpecF16 { using T = uint32_t; static constexpr int bytes = 4; };
struct SpecE4M3 { using T = uint16_t; static constexpr int bytes = 2; };

__device__ __forceinline__ uint32_t f32_bits(float f) { return __float_as_uint(f); }

// round to nearest even; NaN stays NaN
__device__ __forceinline__ uint32_t bf16_rne(float f) {
  uint32_t u = f32_bits(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ uint32_t f16_rne(float f) {
  _Float16 h = (_Float16)f;
  return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_f32(uint32_t h) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

// OCP FP8 e4m3: bias 7, 3 mantissa bits, largest finite 448, saturating,
// round to nearest even.
__device__ __forceinline__ uint32_t e4m3_rne(float v) {
  const uint32_t sign = (f32_bits(v) >> 24) & 0x80u;
  const float x = fabsf(v);
  if (!(x == x)) return 0x7fu;
  uint32_t code;
  if (x < 0.015625f) {                        // below 2^-6: subnormal steps of 2^-9
    code = (uint32_t)rintf(x * 512.0f);       // 0 .. 8 (8 = smallest normal)
  } else {
    int e = __builtin_amdgcn_frexp_expf(x) - 1;   // x = 1.f * 2^e
    const float q = rintf(ldexpf(x, 3 - e));      // 8 .. 16
    code = (uint32_t)((e + 7) << 3) + (uint32_t)q - 8u;
  }
  if (code > 0x7eu) code = 0x7eu;
  return sign | code;
}
__device__ __forceinline__ float e4m3_to_f32(uint32_t b) {
  const uint32_t e = (b >> 3) & 15u, mnt = b & 7u;
  const float mag = e == 0 ? ldexpf((float)mnt, -9) : ldexpf((float)(8u + mnt), (int)e - 10);
  return (b & 0x80u) ? -mag : mag;
}

template <class S> __device__ __forceinline__ typename S::T spec_encode(float2 v);
template <> __device__ __forceinline__ float2 spec_encode<SpecF32>(float2 v) { return v; }
template <> __device__ __forceinline__ uint32_t spec_encode<SpecBF16>(float2 v) {
  return bf16_rne(v.x) | (bf16_rne(v.y) << 16);
}
template <> __device__ __forceinline__ uint32_t spec_encode<SpecF16>(float2 v) {
  return f16_rne(v.x) | (f16_rne(v.y) << 16);
}
template <> __device__ __forceinline__ uint16_t spec_encode<SpecE4M3>(float2 v) {
  return (uint16_t)(e4m3_rne(v.x) | (e4m3_rne(v.y) << 8));
}

template <class S> __device__ __forceinline__ float2 spec_decode(typename S::T v);
template <> __device__ __forceinline__ float2 spec_decode<SpecF32>(float2 v) { return v; }
template <> __device__ __forceinline__ float2 spec_decode<SpecBF16>(uint32_t v) {
  return make_float2(bf16_to_f32(v & 0xffffu), bf16_to_f32(v >> 16));
}
template <> __device__ __forceinline__ float2 spec_decode<SpecF16>(uint32_t v) {
  return make_float2(f16_to_f32(v & 0xffffu), f16_to_f32(v >> 16));
}
template <> __device__ __forceinline__ float2 spec_decode<SpecE4M3>(uint16_t v) {
  return make_float2(e4m3_to_f32(v & 0xffu), e4m3_to_f32(v >> 8));
}

}  // namespace fcc
