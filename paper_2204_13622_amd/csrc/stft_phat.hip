// Front end of the TDoA path (Sec. 2): framing, periodic Hann window, real
// DFT of every frame of every microphone, and per-microphone PHAT.
//
// At alpha = 1 the PHAT of a pair's cross-spectrum factorises,
//   R_ij / |R_ij| = (X_i / |X_i|) (X_j / |X_j|)^*,
// so each bin is normalised once per microphone here instead of once per pair.
//
// The N real samples of a frame are packed as N/2 complex values
// z[n] = w[2n] x[2n] + j w[2n+1] x[2n+1] and transformed by a mixed-radix
// Stockham FFT: radix-16 butterflies held in registers, one LDS exchange per
// pass (two passes for N = 512), in a buffer padded by one slot every 16.  A
// transform uses N/32 lanes (one for N <= 32);
// a 256-thread block runs 256 / lanes transforms over consecutive
// (frame, microphone) pairs, so for M = 16 and N = 512 a block is one frame.
// The split Z -> X(f) = E(f) + W^f O(f) of the real transform follows, then the
// normalisation.  Twiddles (and the window, through its cosine) come from a
// full-circle FP64-computed table staged in LDS.
//
// With recursive smoothing (alpha < 1) the PHAT belongs to each pair's
// smoothed cross-spectrum, so the raw spectra X are written instead (FP32).
//
// Output layout ("packed real spectrum"): N/2 complex slots per microphone;
// slot 0 holds (e(0), e(N/2)), both real, slot f holds e(f) for 0 < f < N/2.
#include "device_common.hpp"
#include "fft_common.hpp"
#include "kernels.hpp"

namespace fcc {
namespace {

using namespace fft;

constexpr int kThreads = 256;
constexpr unsigned kXcds = 8;       // accelerator complex dies of an MI355X

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

template <int N, class S, bool RAW>
__global__ __launch_bounds__(kThreads) void stft_phat_kernel(
    const float* __restrict__ x, int64_t ld, int M, int hop, int64_t nfft,
    const float2* __restrict__ twiddle, typename S::T* __restrict__ out) {
  constexpr int NH = N / 2;
  using RD = Radices<NH>;
  constexpr int LF = RD::LF;
  constexpr int FPB = kThreads / LF;                // transforms per block
  constexpr int NHP = NH + NH / 16;                 // padded buffer length
  constexpr int P1 = RD::R0, P2 = RD::R0 * RD::R1;
  constexpr int T1 = RD::R1 > 1 ? RD::R1 * P1 : 1;  // twiddle table sizes of the LDS passes
  constexpr int T2 = RD::R2 > 1 ? RD::R2 * P2 : 1;
  __shared__ float2 tw[N];
  __shared__ float2 tw1[T1];
  __shared__ float2 tw2[T2];
  __shared__ float2 data[FPB * NHP];

  // Workgroups are dealt to the 8 XCDs round-robin; give each XCD one
  // contiguous run of transforms so the 4x overlap of neighbouring frames is
  // served from that XCD's L2 instead of HBM.
  const unsigned nblk = gridDim.x;
  const unsigned xcd = blockIdx.x % kXcds, local = blockIdx.x / kXcds;
  const unsigned per = nblk / kXcds, extra = nblk % kXcds;     // blocks per XCD (first `extra` get one more)
  const unsigned lblk = xcd * per + (xcd < extra ? xcd : extra) + local;
  const int slot = threadIdx.x / LF, lf = threadIdx.x % LF;
  const int64_t b = (int64_t)lblk * FPB + slot;   // = t * M + m
  const bool active = b < nfft;
  for (int f = threadIdx.x; f < N; f += kThreads) tw[f] = twiddle[f];
  if constexpr (RD::R1 > 1)
    for (int e = threadIdx.x; e < T1; e += kThreads) {
      const int r = e / P1, k = e % P1;
      tw1[e] = twiddle[r * k * (N / (P1 * RD::R1))];
    }
  if constexpr (RD::R2 > 1)
    for (int e = threadIdx.x; e < T2; e += kThreads) {
      const int r = e / P2, k = e % P2;
      tw2[e] = twiddle[r * k * (N / (P2 * RD::R2))];
    }
  __syncthreads();

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
  // X(f) = E + W^f O and X(NH - f) = conj(E - W^f O).
  typename S::T* dst = out + b * NH;
  for (int f = lf; f <= NH / 2; f += LF) {
    if (f == 0) {
      // X(0) = Re Z(0) + Im Z(0), X(N/2) = Re Z(0) - Im Z(0); both real
      const float2 z0 = buf[0];
      if (RAW) dst[0] = spec_encode<S>(make_float2(z0.x + z0.y, z0.x - z0.y));
      else dst[0] = spec_encode<S>(make_float2(phat_real(z0.x + z0.y), phat_real(z0.x - z0.y)));
      continue;
    }
    const float2 zf = buf[pidx(f)];
    const float2 zr = buf[pidx(NH - f)];
    const float2 e = make_float2(0.5f * (zf.x + zr.x), 0.5f * (zf.y - zr.y));
    const float2 o = make_float2(0.5f * (zf.y + zr.y), -0.5f * (zf.x - zr.x));
    const float2 wo = cmul(tw[f], o);
    const float2 Xa = cadd(e, wo);
    const float2 Xb = make_float2(e.x - wo.x, wo.y - e.y);
    dst[f] = spec_encode<S>(RAW ? Xa : phat_complex(Xa));
    if (f != NH - f) dst[NH - f] = spec_encode<S>(RAW ? Xb : phat_complex(Xb));
  }
}

template <int N, class S, bool RAW>
hipError_t launch_n(const StftArgs& a) {
  constexpr int FPB = kThreads / Radices<N / 2>::LF;
  const int64_t nfft = a.T * a.M;
  const int64_t blocks = (nfft + FPB - 1) / FPB;
  hipLaunchKernelGGL((stft_phat_kernel<N, S, RAW>), dim3((unsigned)blocks), dim3(kThreads), 0, a.stream,
                     a.x, a.ld, a.M, a.hop, nfft, a.twiddle, static_cast<typename S::T*>(a.out));
  return hipGetLastError();
}

template <class S, bool RAW = false>
hipError_t launch_s(const StftArgs& a) {
  switch (a.N) {
    case 16: return launch_n<16, S, RAW>(a);
    case 32: return launch_n<32, S, RAW>(a);
    case 64: return launch_n<64, S, RAW>(a);
    case 128: return launch_n<128, S, RAW>(a);
    case 256: return launch_n<256, S, RAW>(a);
    case 512: return launch_n<512, S, RAW>(a);
    case 1024: return launch_n<1024, S, RAW>(a);
    case 2048: return launch_n<2048, S, RAW>(a);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_stft_phat(const StftArgs& a) {
  if (a.T == 0) return hipSuccess;
  if (a.raw) return a.precision == FCC_FP32 ? launch_s<SpecF32, true>(a) : hipErrorInvalidValue;
  switch (a.precision) {
    case FCC_FP32: return launch_s<SpecF32>(a);
    case FCC_BF16: return launch_s<SpecBF16>(a);
    case FCC_FP16: return launch_s<SpecF16>(a);
    case FCC_FP8_E4M3: return launch_s<SpecE4M3>(a);
  }
  return hipErrorInvalidValue;
}

}  // namespace fcc
