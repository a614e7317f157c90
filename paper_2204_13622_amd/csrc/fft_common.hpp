// Building blocks of the in-register / LDS Stockham FFTs of the front end
// and of the GCC-PHAT comparator: compile-time radix-16 butterflies, the
// split of a transform size into at most three radix passes, the padded LDS
// index and one LDS exchange pass.
#pragma once
#include "device_common.hpp"

namespace fcc {
namespace fft {

// exp(-j 2 pi m / 16), m = 0 .. 15 (cos and sin of multiples of pi/8)
__device__ __forceinline__ float2 w16(int m) {
  constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508978f, c2 = 0.70710678118654752f;
  switch (m & 15) {
    case 0: return make_float2(1.f, 0.f);
    case 1: return make_float2(c1, -s1);
    case 2: return make_float2(c2, -c2);
    case 3: return make_float2(s1, -c1);
    case 4: return make_float2(0.f, -1.f);
    case 5: return make_float2(-s1, -c1);
    case 6: return make_float2(-c2, -c2);
    case 7: return make_float2(-c1, -s1);
    case 8: return make_float2(-1.f, 0.f);
    case 9: return make_float2(-c1, s1);
    case 10: return make_float2(-c2, c2);
    case 11: return make_float2(-s1, c1);
    case 12: return make_float2(0.f, 1.f);
    case 13: return make_float2(s1, c1);
    case 14: return make_float2(c2, c2);
    default: return make_float2(c1, s1);
  }
}

// v * exp(-j 2 pi M / 16) with the trivial rotations done exactly
template <int M>
__device__ __forceinline__ float2 rot16(float2 v) {
  constexpr int m = M & 15;
  if constexpr (m == 0) return v;
  else if constexpr (m == 4) return make_float2(v.y, -v.x);
  else if constexpr (m == 8) return make_float2(-v.x, -v.y);
  else if constexpr (m == 12) return make_float2(-v.y, v.x);
  else return cmul(v, w16(m));
}

// In-register DFT of R points (natural order in and out), radix-2
// decimation in time with compile-time twiddles; R divides 16.  The R inputs
// sit at u[0], u[S], u[2S], ... (stride S in registers).
template <int R>
struct Dft {
  template <int S = 1>
  __device__ __forceinline__ static void run(float2* u) {
    Dft<R / 2>::template run<2 * S>(u);        // even-indexed inputs
    Dft<R / 2>::template run<2 * S>(u + S);    // odd-indexed inputs
    float2 out[R];
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const float2 e = u[2 * S * k], o = u[2 * S * k + S];
      const float2 t = twiddle(o, k);
      out[k] = cadd(e, t);
      out[k + R / 2] = csub(e, t);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) u[S * k] = out[k];
  }
  // o * exp(-j 2 pi k / R) = o * exp(-j 2 pi (16 k / R) / 16)
  __device__ __forceinline__ static float2 twiddle(float2 o, int k) {
    switch ((16 / R) * k) {
      case 0: return rot16<0>(o);
      case 1: return rot16<1>(o);
      case 2: return rot16<2>(o);
      case 3: return rot16<3>(o);
      case 4: return rot16<4>(o);
      case 5: return rot16<5>(o);
      case 6: return rot16<6>(o);
      default: return rot16<7>(o);
    }
  }
};
template <>
struct Dft<1> {
  template <int S = 1>
  __device__ __forceinline__ static void run(float2*) {}
};

template <int NH>
struct Radices {
  static constexpr int R0 = NH >= 16 ? 16 : NH;        // first pass
  static constexpr int rem0 = NH / R0;
  static constexpr int R1 = rem0 >= 16 ? 16 : rem0;    // second pass (1 = none)
  static constexpr int rem1 = rem0 / R1;
  static constexpr int R2 = rem1;                      // third pass (1 = none)
  static constexpr int LF = NH >= 16 ? NH / 16 : 1;    // lanes per transform
};

// Position of point n in a transform's LDS buffer: one pad slot after every
// 16 points, so the stride-16 accesses of the passes spread over the banks.
__device__ __forceinline__ int pidx(int n) { return n + (n >> 4); }

// Ordering of one exchange through LDS: a workgroup barrier, or (WAVE) when
// every transform's lanes lie in one wavefront, a fence at wavefront scope,
// so wavefronts run their transforms independently of each other.
template <bool WAVE>
__device__ __forceinline__ void exchange_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One LDS pass of radix R after P points have been combined; twp[r * P + k]
// holds exp(-j 2 pi r k / (P R)).
template <int R, int P, int NH, int LF, bool WAVE = false>
__device__ __forceinline__ void lds_pass(float2* buf, const float2* twp, int lf, bool active) {
  static_assert(!WAVE || (LF <= 64 && 64 % LF == 0), "a transform's lanes must share a wavefront");
  constexpr int NB = NH / R;          // butterflies
  constexpr int BPL = NB / LF;        // per lane
  float2 u[BPL][R];
  if (active) {
#pragma unroll
    for (int b = 0; b < BPL; ++b) {
      const int i = lf + b * LF;
#pragma unroll
      for (int r = 0; r < R; ++r) u[b][r] = buf[pidx(i + r * NB)];
    }
  }
  exchange_sync<WAVE>();
  if (active) {
#pragma unroll
    for (int b = 0; b < BPL; ++b) {
      const int i = lf + b * LF;
      const int k = i % P;
#pragma unroll
      for (int r = 1; r < R; ++r) u[b][r] = cmul(u[b][r], twp[r * P + k]);
      Dft<R>::run(u[b]);
      const int j = (i - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pidx(j + r * P)] = u[b][r];
    }
  }
  exchange_sync<WAVE>();
}

}  // namespace fft
}  // namespace fcc
