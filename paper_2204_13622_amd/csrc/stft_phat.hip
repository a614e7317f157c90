// Front end of the TDoA path (Sec. 2): framing, periodic Hann window, real
// DFT of every frame of every microphone, and per-microphone PHAT.
//
// At alpha = 1 the PHAT of a pair's cross-spectrum factorises,
//   R_ij / |R_ij| = (X_i / |X_i|) (X_j / |X_j|)^*,
// so each bin is normalised once per microphone here instead of once per pair.
//
// One wavefront transforms one (frame, microphone): the N real samples are
// packed as N/2 complex values z[n] = x[2n] + j x[2n+1], transformed by a
// radix-2 Stockham FFT in LDS, and split into the N/2 + 1 bins of the real
// transform.  Twiddles come from the plan's FP64-computed table.
//
// Output layout ("packed real spectrum"): N/2 complex slots per microphone;
// slot 0 holds (e(0), e(N/2)), both real, slot f holds e(f) for 0 < f < N/2.
#include "device_common.hpp"
#include "kernels.hpp"

namespace fcc {
namespace {

// PHAT of a real bin: its sign, or 0 (the squared-magnitude rule of the
// complex bins, applied to a real value).
__device__ __forceinline__ float phat_real(float x) {
  if (x * x < 1.17549435e-38f) return 0.f;
  return x > 0.f ? 1.f : -1.f;
}

template <int N, class S>
__global__ __launch_bounds__(64) void stft_phat_kernel(
    const float* __restrict__ x, int64_t ld, int M, int hop,
    const float* __restrict__ window, const float2* __restrict__ twiddle,
    typename S::T* __restrict__ out) {
  constexpr int NH = N / 2;
  constexpr int F = NH + 1;
  __shared__ float2 buf[2][NH];
  __shared__ float2 tw[F];
  const int lane = threadIdx.x;
  const int64_t bid = blockIdx.x;                 // = t * M + m
  const int mic = (int)(bid % M);
  const int64_t t = bid / M;
  const float* src = x + (int64_t)mic * ld + t * hop;

  for (int f = lane; f < F; f += 64) tw[f] = twiddle[f];
  for (int n = lane; n < NH; n += 64) {
    const float a = src[2 * n] * window[2 * n];
    const float b = src[2 * n + 1] * window[2 * n + 1];
    buf[0][n] = make_float2(a, b);
  }
  __syncthreads();

  int cur = 0;
#pragma unroll 1
  for (int p = 1; p < NH; p <<= 1) {
    const int tstride = N / (2 * p);
    for (int i = lane; i < NH / 2; i += 64) {
      const int k = i & (p - 1);
      const float2 u0 = buf[cur][i];
      const float2 u1 = cmul(buf[cur][i + NH / 2], tw[k * tstride]);
      const int j = 2 * i - k;
      buf[cur ^ 1][j] = cadd(u0, u1);
      buf[cur ^ 1][j + p] = csub(u0, u1);
    }
    cur ^= 1;
    __syncthreads();
  }

  // X(f) = E(f) + W^f O(f), E = (Z(f) + Z*(NH - f)) / 2, O = (Z(f) - Z*(NH - f)) / 2j
  typename S::T* dst = out + bid * NH;
  for (int f = lane; f < NH; f += 64) {
    float2 v;
    if (f == 0) {
      // X(0) = Re Z(0) + Im Z(0), X(N/2) = Re Z(0) - Im Z(0); both real
      const float2 z0 = buf[cur][0];
      v = make_float2(phat_real(z0.x + z0.y), phat_real(z0.x - z0.y));
    } else {
      const float2 zf = buf[cur][f];
      const float2 zr = buf[cur][NH - f];
      const float2 e = make_float2(0.5f * (zf.x + zr.x), 0.5f * (zf.y - zr.y));
      const float2 o = make_float2(0.5f * (zf.y + zr.y), -0.5f * (zf.x - zr.x));  // (Z - Z*) / 2j
      const float2 X = cadd(e, cmul(tw[f], o));
      const float n2 = X.x * X.x + X.y * X.y;
      v = make_float2(0.f, 0.f);
      if (n2 >= 1.17549435e-38f) {
        const float s = rsqrtf(n2);
        v = make_float2(X.x * s, X.y * s);
      }
    }
    dst[f] = spec_encode<S>(v);
  }
}

template <int N, class S>
hipError_t launch_n(const StftArgs& a) {
  const int64_t blocks = a.T * a.M;
  hipLaunchKernelGGL((stft_phat_kernel<N, S>), dim3((unsigned)blocks), dim3(64), 0, a.stream,
                     a.x, a.ld, a.M, a.hop, a.window, a.twiddle,
                     static_cast<typename S::T*>(a.out));
  return hipGetLastError();
}

template <class S>
hipError_t launch_s(const StftArgs& a) {
  switch (a.N) {
    case 16: return launch_n<16, S>(a);
    case 32: return launch_n<32, S>(a);
    case 64: return launch_n<64, S>(a);
    case 128: return launch_n<128, S>(a);
    case 256: return launch_n<256, S>(a);
    case 512: return launch_n<512, S>(a);
    case 1024: return launch_n<1024, S>(a);
    case 2048: return launch_n<2048, S>(a);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_stft_phat(const StftArgs& a) {
  if (a.T == 0) return hipSuccess;
  switch (a.precision) {
    case FCC_FP32: return launch_s<SpecF32>(a);
    case FCC_BF16: return launch_s<SpecBF16>(a);
    case FCC_FP16: return launch_s<SpecF16>(a);
    case FCC_FP8_E4M3: return launch_s<SpecE4M3>(a);
  }
  return hipErrorInvalidValue;
}

}  // namespace fcc
