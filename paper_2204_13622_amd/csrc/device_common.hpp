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

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ float f16_to_f32(uint32_t h) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}
// OCP FP8 e4m3: bias 7, 3 mantissa bits, largest finite 448
__device__ __forceinline__ float e4m3_to_f32(uint32_t b) {
  const uint32_t e = (b >> 3) & 15u, mnt = b & 7u;
  const float mag = e == 0 ? ldexpf((float)mnt, -9) : ldexpf((float)(8u + mnt), (int)e - 10);
  return (b & 0x80u) ? -mag : mag;
}

// Encoders: the hardware pack conversions, round to nearest even (the
// whitened values lie in [-1, 1], far inside every format's range).
typedef float enc_f2 __attribute__((ext_vector_type(2)));
typedef _Float16 enc_h2 __attribute__((ext_vector_type(2)));
typedef __bf16 enc_b2 __attribute__((ext_vector_type(2)));

template <class S> __device__ __forceinline__ typename S::T spec_encode(float2 v);
template <> __device__ __forceinline__ float2 spec_encode<SpecF32>(float2 v) { return v; }
template <> __device__ __forceinline__ uint32_t spec_encode<SpecBF16>(float2 v) {
  const enc_b2 b = {(__bf16)v.x, (__bf16)v.y};                 // v_cvt_pk_bf16_f32
  return __builtin_bit_cast(uint32_t, b);
}
template <> __device__ __forceinline__ uint32_t spec_encode<SpecF16>(float2 v) {
  const enc_f2 f = {v.x, v.y};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, enc_h2));   // v_cvt_pk_f16_f32
}
template <> __device__ __forceinline__ uint16_t spec_encode<SpecE4M3>(float2 v) {
  return (uint16_t)__builtin_amdgcn_cvt_pk_fp8_f32(v.x, v.y, 0, false);   // v_cvt_pk_fp8_f32
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
