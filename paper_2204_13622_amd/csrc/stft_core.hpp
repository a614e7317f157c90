// Device code of the front end (framing, periodic Hann window, real DFT,
// per-microphone PHAT), shared by the single-array kernel and the batched
// kernel.  The method and the layout are described in stft_phat.hip.
#pragma once
#include "device_common.hpp"
#include "fft_common.hpp"

namespace fcc {
namespace stft_core {

using namespace fft;

constexpr int kThreads = 256;

// PHAT of one bin: X / |X|, or 0 when |X|^2 is below the smallest normal
// float.  A real bin's PHAT is its sign.
__device__ __forceinline__ float2 phat_complex(float2 X) {
  const float n2 = X.x * X.x + X.y * X.y;
  if (n2 < 1.17549435e-38f) return make_float2(0.f, 0.f);
  const float s = rsqrtf(n2);
  return make_float2(X.x * s, X.y * s);
}
__device__ __forceinline__ float phat_real(float x) {
  if (x * x < 1.17549435e-38f) return 0.f;
  return x > 0.f ? 1.f : -1.f;
}

template <int N>
struct StftShape {
  static constexpr int NH = N / 2;
  using RD = Radices<NH>;
  static constexpr int LF = RD::LF;                       // lanes per transform
  static constexpr int FPB = kThreads / LF;               // transforms per block
  static constexpr int NHP = NH + NH / 16;                // padded buffer length
  static constexpr int P1 = RD::R0, P2 = RD::R0 * RD::R1;
  static constexpr int T1 = RD::R1 > 1 ? RD::R1 * P1 : 1; // twiddle table sizes of the LDS passes
  static constexpr int T2 = RD::R2 > 1 ? RD::R2 * P2 : 1;
  static constexpr int lds_float2 = N + T1 + T2 + FPB * NHP;
};

// Block-wide: the full-circle twiddles (and, through their cosines, the
// window) and the per-pass twiddle tables into LDS.
template <int N>
__device__ __forceinline__ void load_tables(float2* tw, float2* tw1, float2* tw2, const float2* __restrict__ twiddle) {
  using Sh = StftShape<N>;
  using RD = typename Sh::RD;
  for (int f = threadIdx.x; f < N; f += kThreads) tw[f] = twiddle[f];
  if constexpr (RD::R1 > 1)
    for (int e = threadIdx.x; e < Sh::T1; e += kThreads) {
      const int r = e / Sh::P1, k = e % Sh::P1;
      tw1[e] = twiddle[r * k * (N / (Sh::P1 * RD::R1))];
    }
  if constexpr (RD::R2 > 1)
    for (int e = threadIdx.x; e < Sh::T2; e += kThreads) {
      const int r = e / Sh::P2, k = e % Sh::P2;
      tw2[e] = twiddle[r * k * (N / (Sh::P2 * RD::R2))];
    }
}

// Block-wide: the FPB transforms lblk * FPB .. + FPB - 1 (transform b is
// microphone b % M of frame b / M; those at or past nfft idle).  Tables in
// LDS already; `data` is the block's transform scratch.
template <int N, class S, bool RAW>
__device__ __forceinline__ void transforms(const float2* tw, const float2* tw1, const float2* tw2, float2* data,
                                           const float* __restrict__ x, int64_t ld, int M, int hop, int64_t nfft,
                                           typename S::T* __restrict__ out, int64_t lblk) {
  using Sh = StftShape<N>;
  using RD = typename Sh::RD;
  constexpr int NH = Sh::NH, LF = Sh::LF, FPB = Sh::FPB, NHP = Sh::NHP, P1 = Sh::P1, P2 = Sh::P2;
  const int slot = threadIdx.x / LF, lf = threadIdx.x % LF;
  const int64_t b = lblk * FPB + slot;   // = t * M + m
  const bool active = b < nfft;
  float2* buf = data + slot * NHP;
  // first pass straight from memory: radix R0, no twiddles (p = 1)
  {
    constexpr int R = RD::R0, NB = NH / R;
    float2 u[R];
    if (active) {
      const int mic = (int)(b % M);
      const int64_t t = b / M;
      const float* src = x + (int64_t)mic * ld + t * hop;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int n = lf + r * NB;
        const float w0 = 0.5f - 0.5f * tw[2 * n].x;          // periodic Hann
        const float w1 = 0.5f - 0.5f * tw[2 * n + 1].x;
        u[r] = make_float2(w0 * src[2 * n], w1 * src[2 * n + 1]);
      }
      Dft<R>::run(u);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pidx(lf * R + r)] = u[r];
    }
    __syncthreads();
  }
  if constexpr (RD::R1 > 1) lds_pass<RD::R1, P1, NH, LF>(buf, tw1, lf, active);
  if constexpr (RD::R2 > 1) lds_pass<RD::R2, P2, NH, LF>(buf, tw2, lf, active);

  if (!active) return;
  // Real split: E = (Z(f) + Z*(NH - f)) / 2, O = (Z(f) - Z*(NH - f)) / 2j,
  // X(f) = E + W^f O and X(NH - f) = conj(E - W^f O).  PHAT is blind to a
  // common factor, so the halves are dropped unless the raw X is wanted.
  // Lane lf takes f = lf, lf + LF, ... < NH / 2 (the same number of bins on
  // every lane); f = 0 is the DC / Nyquist slot, and its lane also takes the
  // centre bin NH / 2, which is its own mirror.
  constexpr float h = RAW ? 0.5f : 1.f;
  typename S::T* dst = out + b * NH;
  for (int f = lf; f < NH / 2; f += LF) {
    if (f == 0) {
      // X(0) = Re Z(0) + Im Z(0), X(N/2) = Re Z(0) - Im Z(0); both real
      const float2 z0 = buf[0];
      if (RAW) dst[0] = spec_encode<S>(make_float2(z0.x + z0.y, z0.x - z0.y));
      else dst[0] = spec_encode<S>(make_float2(phat_real(z0.x + z0.y), phat_real(z0.x - z0.y)));
      // centre: E = Re Z(NH/2), O = Im Z(NH/2), X = E + W^(NH/2) O
      const float2 zc = buf[pidx(NH / 2)];
      const float2 wc = tw[NH / 2];
      const float2 Xc = make_float2(zc.x + wc.x * zc.y, wc.y * zc.y);
      dst[NH / 2] = spec_encode<S>(RAW ? Xc : phat_complex(Xc));
      continue;
    }
    const float2 zf = buf[pidx(f)];
    const float2 zr = buf[pidx(NH - f)];
    const float2 e = make_float2(h * (zf.x + zr.x), h * (zf.y - zr.y));
    const float2 o = make_float2(h * (zf.y + zr.y), -h * (zf.x - zr.x));
    const float2 wo = cmul(tw[f], o);
    const float2 Xa = cadd(e, wo);
    const float2 Xb = make_float2(e.x - wo.x, wo.y - e.y);
    dst[f] = spec_encode<S>(RAW ? Xa : phat_complex(Xa));
    dst[NH - f] = spec_encode<S>(RAW ? Xb : phat_complex(Xb));
  }
}

}  // namespace stft_core
}  // namespace fcc
