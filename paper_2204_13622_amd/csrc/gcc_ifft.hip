// GCC-PHAT comparator through a full inverse DFT (Sec. 2, eq. 2; the
// FFT-based baseline that Sec. 3 and Table 1 measure FCC against).
//
// For a pair the Hermitian spectrum of eq. (2) is
//   S(0) = 2 R(0),  S(N/2) = 2 R(N/2),  S(f) = R(f),  S(N - f) = R(f)^*  (0 < f < N/2)
// with R = e_i e_j^* (PHAT already applied per microphone), and
// y(tau) = sum_n S(n) exp(+j 2 pi n tau / N), read at tau mod N for
// tau = -tau_max .. tau_max.  y is real, so two pairs A and B share one
// complex transform: Z = S_A + j S_B gives z = y_A + j y_B.  The inverse is
// taken as the conjugate of a forward FFT of conj(Z).
//
// One workgroup per frame: the frame's M spectra are decoded to FP32 bins
// 0 .. N/2 in LDS; each group of N/16 lanes runs one N-point Stockham FFT
// (a radix-16 pass whose inputs are formed straight from the spectra, then
// one or two LDS passes), and the first lane of the group scans the 2 tau_max + 1
// wanted outputs for the first-index argmax of both pairs.
#include "fft_common.hpp"
#include "kernels.hpp"

namespace fcc {
namespace {

using namespace fft;

constexpr int kThreads = 256;

template <int N>
struct GccShape {
  using RD = Radices<N>;
  static constexpr int LF = RD::LF;                      // lanes per transform
  static constexpr int FPB = kThreads / LF;              // transforms per pass over the block
  static constexpr int NP = N + N / 16;                  // padded transform buffer
  static constexpr int P1 = RD::R0, P2 = RD::R0 * RD::R1;
  static constexpr int T1 = RD::R1 > 1 ? RD::R1 * P1 : 1;
  static constexpr int T2 = RD::R2 > 1 ? RD::R2 * P2 : 1;
  static size_t lds_bytes(int M) {
    return sizeof(float2) * (size_t(M) * (N / 2 + 1) + size_t(FPB) * NP + T1 + T2);
  }
};

template <int N, class S, bool WRITE_Y>
__global__ __launch_bounds__(kThreads) void gcc_ifft_kernel(
    const typename S::T* __restrict__ spec, int M, int P, int I, int tau_max,
    const uint8_t* __restrict__ pairs, const float2* __restrict__ twiddle,
    int32_t* __restrict__ tdoa, float* __restrict__ yout) {
  using G = GccShape<N>;
  using RD = typename G::RD;
  constexpr int NH = N / 2, F = NH + 1, LF = G::LF, FPB = G::FPB, NP = G::NP;
  extern __shared__ float2 lds[];
  float2* sp = lds;                          // [M][F]
  float2* data = sp + M * F;                 // [FPB][NP]
  float2* tw1 = data + FPB * NP;             // [T1]
  float2* tw2 = tw1 + G::T1;                 // [T2]

  const int64_t t = blockIdx.x;
  const typename S::T* src = spec + t * (int64_t)M * NH;
  for (int i = threadIdx.x; i < M * NH; i += kThreads) {
    const int mic = i / NH, f = i - mic * NH;
    const float2 v = spec_decode<S>(src[i]);
    if (f == 0) {
      sp[mic * F] = make_float2(v.x, 0.f);
      sp[mic * F + NH] = make_float2(v.y, 0.f);
    } else {
      sp[mic * F + f] = v;
    }
  }
  if constexpr (RD::R1 > 1)
    for (int e = threadIdx.x; e < G::T1; e += kThreads) {
      const int r = e / G::P1, k = e % G::P1;
      tw1[e] = twiddle[r * k * (N / (G::P1 * RD::R1))];
    }
  if constexpr (RD::R2 > 1)
    for (int e = threadIdx.x; e < G::T2; e += kThreads) {
      const int r = e / G::P2, k = e % G::P2;
      tw2[e] = twiddle[r * k * (N / (G::P2 * RD::R2))];
    }
  __syncthreads();

  const int slot = threadIdx.x / LF, lf = threadIdx.x % LF;
  float2* buf = data + slot * NP;
  const int transforms = (P + 1) / 2;
  for (int base = 0; base < transforms; base += FPB) {
    const int q = base + slot;
    const bool active = q < transforms;
    const int pa = 2 * q, pb = 2 * q + 1;
    const bool has_b = pb < P;
    // first pass: radix 16 over the inputs n = lf + 16-stride, no twiddles
    {
      constexpr int R = RD::R0, NB = N / R;
      float2 u[R];
      if (active) {
        const float2* ai = sp + pairs[2 * pa] * F;
        const float2* aj = sp + pairs[2 * pa + 1] * F;
        const float2* bi = sp + (has_b ? pairs[2 * pb] : 0) * F;
        const float2* bj = sp + (has_b ? pairs[2 * pb + 1] : 0) * F;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int n = lf + r * NB;
          const int f = n <= NH ? n : N - n;
          const float2 ra = cmul_conj(ai[f], aj[f]);
          float2 rb = cmul_conj(bi[f], bj[f]);
          if (!has_b) rb = make_float2(0.f, 0.f);
          float2 z;
          if (n == 0 || n == NH) {
            z = make_float2(2.f * ra.x, 2.f * rb.x);                 // both bins are real
          } else if (n < NH) {
            z = make_float2(ra.x - rb.y, ra.y + rb.x);               // R_A + j R_B
          } else {
            z = make_float2(ra.x + rb.y, rb.x - ra.y);               // R_A^* + j R_B^*
          }
          u[r] = make_float2(z.x, -z.y);                             // conj: inverse by a forward FFT
        }
        Dft<R>::run(u);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[pidx(lf * R + r)] = u[r];
      }
      __syncthreads();
    }
    if constexpr (RD::R1 > 1) lds_pass<RD::R1, G::P1, N, LF>(buf, tw1, lf, active);
    if constexpr (RD::R2 > 1) lds_pass<RD::R2, G::P2, N, LF>(buf, tw2, lf, active);

    // natural-order output w = FFT(conj Z); z = conj(w): y_A = Re w, y_B = -Im w
    if (active && lf == 0) {
      float best_a = 0.f, best_b = 0.f;
      int ia = 0, ib = 0;
      for (int ii = 0; ii < I; ++ii) {
        int n = ii - tau_max;
        n += n < 0 ? N : 0;
        const float2 w = buf[pidx(n)];
        const float ya = w.x, yb = -w.y;
        if (ii == 0 || ya > best_a) { best_a = ya; ia = ii; }
        if (ii == 0 || yb > best_b) { best_b = yb; ib = ii; }
        if (WRITE_Y) {
          yout[(t * P + pa) * I + ii] = ya;
          if (has_b) yout[(t * P + pb) * I + ii] = yb;
        }
      }
      if (!WRITE_Y) {
        tdoa[t * P + pa] = ia - tau_max;
        if (has_b) tdoa[t * P + pb] = ib - tau_max;
      }
    }
    __syncthreads();
  }
}

template <int N, class S>
hipError_t launch_n(const PairArgs& a) {
  const size_t lds = GccShape<N>::lds_bytes(a.M);
  auto k = a.y ? gcc_ifft_kernel<N, S, true> : gcc_ifft_kernel<N, S, false>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)a.T), dim3(kThreads), lds, a.stream,
                     static_cast<const typename S::T*>(a.spec), a.M, a.P, a.I, a.tau_max, a.pairs, a.twiddle,
                     a.tdoa, a.y);
  return hipGetLastError();
}

template <class S>
hipError_t launch_s(const PairArgs& a) {
  switch (a.N) {
    case 16: return launch_n<16, S>(a);
    case 32: return launch_n<32, S>(a);
    case 64: return launch_n<64, S>(a);
    case 128: return launch_n<128, S>(a);
    case 256: return launch_n<256, S>(a);
    case 512: return launch_n<512, S>(a);
    case 1024: return launch_n<1024, S>(a);
    case 2048: return launch_n<2048, S>(a);
  }
  return hipErrorInvalidValue;
}

size_t lds_for(int N, int M) {
  switch (N) {
    case 16: return GccShape<16>::lds_bytes(M);
    case 32: return GccShape<32>::lds_bytes(M);
    case 64: return GccShape<64>::lds_bytes(M);
    case 128: return GccShape<128>::lds_bytes(M);
    case 256: return GccShape<256>::lds_bytes(M);
    case 512: return GccShape<512>::lds_bytes(M);
    case 1024: return GccShape<1024>::lds_bytes(M);
    case 2048: return GccShape<2048>::lds_bytes(M);
  }
  return ~size_t(0);
}

}  // namespace

bool gcc_ifft_supported(const PairArgs& a) {
  return a.method == FCC_METHOD_GCC && a.twiddle != nullptr && a.I <= a.N && lds_for(a.N, a.M) <= 160 * 1024;
}

hipError_t launch_gcc_ifft(const PairArgs& a) {
  if (a.T == 0) return hipSuccess;
  if (!gcc_ifft_supported(a) || (!a.tdoa && !a.y)) return hipErrorInvalidValue;
  switch (a.precision) {
    case FCC_FP32: return launch_s<SpecF32>(a);
    case FCC_BF16: return launch_s<SpecBF16>(a);
    case FCC_FP16: return launch_s<SpecF16>(a);
    case FCC_FP8_E4M3: return launch_s<SpecE4M3>(a);
  }
  return hipErrorInvalidValue;
}

}  // namespace fcc
