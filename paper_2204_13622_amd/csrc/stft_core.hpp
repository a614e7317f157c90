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
  // front table: NH window pairs (w(2n), w(2n + 1)), then W^f for f = 0 .. NH / 2
  static constexpr int TW = NH + NH / 2 + 1;
  static constexpr int lds_float2 = TW + T1 + T2 + FPB * NHP;
};

// Block-wide: the periodic Hann window and the split twiddles (from the
// full-circle FP64-computed twiddles) and the per-pass twiddle tables into LDS.
template <int N>
__device__ __forceinline__ void load_tables(float2* tw, float2* tw1, float2* tw2, const float2* __restrict__ twiddle) {
  using Sh = StftShape<N>;
  using RD = typename Sh::RD;
  constexpr int NH = Sh::NH;
  for (int n = threadIdx.x; n < NH; n += kThreads)      // w[n] = 0.5 - 0.5 cos(2 pi n / N)
    tw[n] = make_float2(0.5f - 0.5f * twiddle[2 * n].x, 0.5f - 0.5f * twiddle[2 * n + 1].x);
  for (int f = threadIdx.x; f <= NH / 2; f += kThreads) tw[NH + f] = twiddle[f];
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

// PHAT scale of one bin from its squared magnitude: 1 / |X|, or 0 below the
// smallest normal float
__device__ __forceinline__ float phat_scale(float n2) {
  const float s = rsqrtf(n2);
  return n2 < 1.17549435e-38f ? 0.f : s;
}

// The R0 sample pairs lane lf of transform b needs for the first pass:
// (x[2n], x[2n + 1]) for n = lf + r NB, unwindowed (b < nfft < 2^31).
template <int N>
__device__ __forceinline__ void load_samples_at(float2 (&u)[StftShape<N>::RD::R0], const float* __restrict__ src,
                                                int lf) {
  using RD = typename StftShape<N>::RD;
  constexpr int R = RD::R0, NB = StftShape<N>::NH / R;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int n = lf + r * NB;
    u[r] = make_float2(src[2 * n], src[2 * n + 1]);
  }
}
template <int N>
__device__ __forceinline__ void load_samples(float2 (&u)[StftShape<N>::RD::R0], const float* __restrict__ x,
                                             int64_t ld, int M, int hop, uint32_t b, int lf) {
  const uint32_t t = b / (uint32_t)M;
  const int mic = (int)(b - t * (uint32_t)M);
  load_samples_at<N>(u, x + (int64_t)mic * ld + (int64_t)t * hop, lf);
}

// One lane's share of one transform, given the first pass's samples of this
// lane in `u` (ignored where inactive): window, first pass in registers, the
// LDS passes in the transform's scratch `buf`, then the real split and, unless
// RAW, PHAT.  `between` runs on every lane once the first pass has stored its
// outputs (a persistent caller issues its next loads there); `emit(f, X)`
// takes each output slot f of this lane, slot 0 packing the real bins 0 and
// N/2.  Inactive lanes only take part in the wavefront-scope orderings (a
// transform's lanes share a wavefront).
template <int N, bool RAW, class Between, class Emit>
__device__ __forceinline__ void transform_lane(const float2* tw, const float2* tw1, const float2* tw2, float2* buf,
                                               float2 (&u)[StftShape<N>::RD::R0], bool active, int lf,
                                               Between&& between, Emit&& emit) {
  using Sh = StftShape<N>;
  using RD = typename Sh::RD;
  constexpr int NH = Sh::NH, LF = Sh::LF, P1 = Sh::P1, P2 = Sh::P2;
  const float2* win = tw;                          // window pairs
  const float2* wsp = tw + NH;                     // W^f, f = 0 .. NH / 2
  // first pass: radix R0 on the windowed samples, no twiddles (p = 1)
  {
    constexpr int R = RD::R0, NB = NH / R;
    if (active) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float2 w = win[lf + r * NB];         // periodic Hann at 2n, 2n + 1
        u[r] = make_float2(w.x * u[r].x, w.y * u[r].y);
      }
      Dft<R>::run(u);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pidx(lf * R + r)] = u[r];
    }
    between();
    exchange_sync<true>();
  }
  if constexpr (RD::R1 > 1) lds_pass<RD::R1, P1, NH, LF, true>(buf, tw1, lf, active);
  if constexpr (RD::R2 > 1) lds_pass<RD::R2, P2, NH, LF, true>(buf, tw2, lf, active);

  if (!active) return;
  // Real split: E = (Z(f) + Z*(NH - f)) / 2, O = (Z(f) - Z*(NH - f)) / 2j,
  // X(f) = E + W^f O and X(NH - f) = conj(E - W^f O).  PHAT is blind to a
  // common factor, so the halves are dropped unless the raw X is wanted.
  // Lane lf takes f = lf, lf + LF, ... < NH / 2 (the same number of bins on
  // every lane); f = 0 is the DC / Nyquist slot, done after the loop by the
  // lanes with lf = 0, which also take the centre bin NH / 2 (its own mirror).
  constexpr float h = RAW ? 0.5f : 1.f;
  constexpr int kIters = (NH / 2 + LF - 1) / LF;
#pragma unroll
  for (int k = 0; k < kIters; ++k) {
    const int f = lf + k * LF;
    if (f == 0 || f >= NH / 2) continue;
    const float2 zf = buf[pidx(f)];
    const float2 zr = buf[pidx(NH - f)];
    const float2 e = make_float2(h * (zf.x + zr.x), h * (zf.y - zr.y));
    const float2 o = make_float2(h * (zf.y + zr.y), -h * (zf.x - zr.x));
    const float2 wo = cmul(wsp[f], o);
    const float2 Xa = cadd(e, wo);
    const float2 Xb = make_float2(e.x - wo.x, wo.y - e.y);
    if (RAW) {
      emit(f, Xa);
      emit(NH - f, Xb);
    } else {
      const float sa = phat_scale(Xa.x * Xa.x + Xa.y * Xa.y);
      const float sb = phat_scale(Xb.x * Xb.x + Xb.y * Xb.y);
      emit(f, make_float2(Xa.x * sa, Xa.y * sa));
      emit(NH - f, make_float2(Xb.x * sb, Xb.y * sb));
    }
  }
  if (lf == 0) {
    // X(0) = Re Z(0) + Im Z(0), X(N/2) = Re Z(0) - Im Z(0); both real
    const float2 z0 = buf[0];
    if (RAW) emit(0, make_float2(z0.x + z0.y, z0.x - z0.y));
    else emit(0, make_float2(phat_real(z0.x + z0.y), phat_real(z0.x - z0.y)));
    // centre: E = Re Z(NH/2), O = Im Z(NH/2), X = E + W^(NH/2) O
    const float2 zc = buf[pidx(NH / 2)];
    const float2 wc = wsp[NH / 2];
    const float2 Xc = make_float2(zc.x + wc.x * zc.y, wc.y * zc.y);
    emit(NH / 2, RAW ? Xc : phat_complex(Xc));
  }
}

// Block-wide: the FPB transforms lblk * FPB .. + FPB - 1 (transform b is
// microphone b % M of frame b / M; those at or past nfft idle; nfft < 2^31),
// given the first pass's samples of this lane's transform in `u` (loaded by
// load_samples; ignored where inactive).  Tables in LDS already; `data` is
// the block's transform scratch.  `between` runs after the first pass has
// stored its outputs (a persistent caller issues its next loads there).
template <int N, class S, bool RAW, class Between>
__device__ __forceinline__ void transform_samples(const float2* tw, const float2* tw1, const float2* tw2,
                                                  float2* data, float2 (&u)[StftShape<N>::RD::R0], int64_t nfft,
                                                  typename S::T* __restrict__ out, int64_t lblk,
                                                  Between&& between) {
  using Sh = StftShape<N>;
  constexpr int NH = Sh::NH, LF = Sh::LF, FPB = Sh::FPB, NHP = Sh::NHP;
  const int slot = threadIdx.x / LF, lf = threadIdx.x % LF;
  const uint32_t b = (uint32_t)lblk * FPB + slot;   // = t * M + m
  typename S::T* dst = out + (int64_t)b * NH;
  transform_lane<N, RAW>(tw, tw1, tw2, data + slot * NHP, u, b < (uint64_t)nfft, lf, between,
                         [&](int f, float2 v) { dst[f] = spec_encode<S>(v); });
}

// Block-wide: the FPB transforms lblk * FPB .. + FPB - 1, samples loaded here.
template <int N, class S, bool RAW>
__device__ __forceinline__ void transforms(const float2* tw, const float2* tw1, const float2* tw2, float2* data,
                                           const float* __restrict__ x, int64_t ld, int M, int hop, int64_t nfft,
                                           typename S::T* __restrict__ out, int64_t lblk) {
  using Sh = StftShape<N>;
  const int slot = threadIdx.x / Sh::LF, lf = threadIdx.x % Sh::LF;
  const uint32_t b = (uint32_t)lblk * Sh::FPB + slot;
  float2 u[Sh::RD::R0];
  if (b < (uint64_t)nfft) load_samples<N>(u, x, ld, M, hop, b, lf);
  transform_samples<N, S, RAW>(tw, tw1, tw2, data, u, nfft, out, lblk, [] {});
}

}  // namespace stft_core
}  // namespace fcc
