// GCC-PHAT comparator through a full inverse DFT (Sec. 2, eq. 2; the
// FFT-based baseline that Sec. 3 and Table 1 measure FCC against).
//
// For a pair the Hermitian spectrum of eq. (2), zero-padded to L = r N points
// for a lag grid of 1/r sample (Sec. 3), is
//   S(0) = 2 R(0),  S(f) = R(f),  S(L - f) = R(f)^*  (0 < f <= N/2),  0 elsewhere
// (for r = 1 the two Nyquist terms land on one index, S(N/2) = 2 R(N/2)),
// with R = e_i e_j^* (PHAT already applied per microphone), and
// y(i / r - tau_max) = sum_n S(n) exp(+j 2 pi n (i - r tau_max) / L).  y is
// real, so two pairs A and B share one complex transform: Z = S_A + j S_B
// gives z = y_A + j y_B.  The inverse is taken as the conjugate of a forward
// FFT of conj(Z).
//
// One workgroup per frame: the frame's M spectra are decoded to FP32 bins
// 0 .. N/2 in LDS; each group of L/16 lanes runs one L-point Stockham FFT
// (a radix-16 pass whose inputs are formed straight from the spectra, then
// one to three LDS passes), and the first lane of the group scans the
// 2 r tau_max + 1 wanted outputs for the first-index argmax of both pairs.
#include "fft_common.hpp"
#include "kernels.hpp"

namespace fcc {
namespace {

using namespace fft;

constexpr int kThreads = 256;

// a transform of L points: radix 16, then up to three LDS passes
template <int L>
struct GccShape {
  static constexpr int R0 = 16;
  static constexpr int R1 = L / 16 >= 16 ? 16 : L / 16;
  static constexpr int R2 = L / 256 >= 16 ? 16 : (L / 256 > 1 ? L / 256 : 1);
  static constexpr int R3 = L / (R0 * R1 * R2);
  static_assert(R0 * R1 * R2 * R3 == L && R3 <= 16, "transform size");
  static constexpr int LF = L / 16;                      // lanes per transform
  static constexpr int FPB = kThreads / LF;              // transforms per pass over the block
  static constexpr int NP = L + L / 16;                  // padded transform buffer
  static constexpr int P1 = R0, P2 = R0 * R1, P3 = R0 * R1 * R2;
  static constexpr int T1 = R1 > 1 ? R1 * P1 : 1;
  static constexpr int T2 = R2 > 1 ? R2 * P2 : 1;
  static constexpr int T3 = R3 > 1 ? R3 * P3 : 1;
  static size_t lds_bytes(int M, int NH) {
    return sizeof(float2) * (size_t(M) * (NH + 1) + size_t(FPB) * NP + T1 + T2 + T3);
  }
};

template <int L, class S, bool WRITE_Y>
__global__ __launch_bounds__(kThreads) void gcc_ifft_kernel(
    const typename S::T* __restrict__ spec, int M, int P, int NH, int I, int lag0,
    const uint8_t* __restrict__ pairs, const float2* __restrict__ twiddle /*[L]*/,
    int32_t* __restrict__ tdoa, float* __restrict__ yout) {
  using G = GccShape<L>;
  constexpr int LF = G::LF, FPB = G::FPB, NP = G::NP;
  const int F = NH + 1;
  const bool single = 2 * NH == L;           // r = 1: both Nyquist terms on index N/2
  extern __shared__ float2 lds[];
  float2* sp = lds;                          // [M][F]
  float2* data = sp + M * F;                 // [FPB][NP]
  float2* tw1 = data + FPB * NP;             // [T1]
  float2* tw2 = tw1 + G::T1;                 // [T2]
  float2* tw3 = tw2 + G::T2;                 // [T3]

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
  if constexpr (G::R1 > 1)
    for (int e = threadIdx.x; e < G::T1; e += kThreads) {
      const int r = e / G::P1, k = e % G::P1;
      tw1[e] = twiddle[r * k * (L / (G::P1 * G::R1))];
    }
  if constexpr (G::R2 > 1)
    for (int e = threadIdx.x; e < G::T2; e += kThreads) {
      const int r = e / G::P2, k = e % G::P2;
      tw2[e] = twiddle[r * k * (L / (G::P2 * G::R2))];
    }
  if constexpr (G::R3 > 1)
    for (int e = threadIdx.x; e < G::T3; e += kThreads) {
      const int r = e / G::P3, k = e % G::P3;
      tw3[e] = twiddle[r * k * (L / (G::P3 * G::R3))];
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
    // first pass: radix 16 over the inputs n = lf + r L/16, no twiddles
    {
      constexpr int R = G::R0, NB = L / R;
      float2 u[R];
      if (active) {
        const float2* ai = sp + pairs[2 * pa] * F;
        const float2* aj = sp + pairs[2 * pa + 1] * F;
        const float2* bi = sp + (has_b ? pairs[2 * pb] : 0) * F;
        const float2* bj = sp + (has_b ? pairs[2 * pb + 1] : 0) * F;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int n = lf + r * NB;
          const int f = n <= L / 2 ? n : L - n;
          float2 z = make_float2(0.f, 0.f);                          // zero padding beyond N/2
          if (f <= NH) {
            const float2 ra = cmul_conj(ai[f], aj[f]);
            float2 rb = cmul_conj(bi[f], bj[f]);
            if (!has_b) rb = make_float2(0.f, 0.f);
            if (n == 0 || (single && n == NH)) {
              z = make_float2(2.f * ra.x, 2.f * rb.x);               // both bins are real
            } else if (n <= NH) {
              z = make_float2(ra.x - rb.y, ra.y + rb.x);             // R_A + j R_B
            } else {
              z = make_float2(ra.x + rb.y, rb.x - ra.y);             // R_A^* + j R_B^*
            }
          }
          u[r] = make_float2(z.x, -z.y);                             // conj: inverse by a forward FFT
        }
        Dft<R>::run(u);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[pidx(lf * R + r)] = u[r];
      }
      __syncthreads();
    }
    if constexpr (G::R1 > 1) lds_pass<G::R1, G::P1, L, LF>(buf, tw1, lf, active);
    if constexpr (G::R2 > 1) lds_pass<G::R2, G::P2, L, LF>(buf, tw2, lf, active);
    if constexpr (G::R3 > 1) lds_pass<G::R3, G::P3, L, LF>(buf, tw3, lf, active);

    // natural-order output w = FFT(conj Z); z = conj(w): y_A = Re w, y_B = -Im w
    if (active && lf == 0) {
      float best_a = 0.f, best_b = 0.f;
      int ia = 0, ib = 0;
      for (int ii = 0; ii < I; ++ii) {
        int n = ii - lag0;
        n += n < 0 ? L : 0;
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
        tdoa[t * P + pa] = ia - lag0;                  // units of 1/r sample
        if (has_b) tdoa[t * P + pb] = ib - lag0;
      }
    }
    __syncthreads();
  }
}

template <int L, class S>
hipError_t launch_n(const PairArgs& a) {
  const size_t lds = GccShape<L>::lds_bytes(a.M, a.N / 2);
  auto k = a.y ? gcc_ifft_kernel<L, S, true> : gcc_ifft_kernel<L, S, false>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)a.T), dim3(kThreads), lds, a.stream,
                     static_cast<const typename S::T*>(a.spec), a.M, a.P, a.N / 2, a.I, a.lag0, a.pairs,
                     a.twiddle_r, a.tdoa, a.y);
  return hipGetLastError();
}

template <class S>
hipError_t launch_s(const PairArgs& a) {
  switch (a.r * a.N) {
    case 16: return launch_n<16, S>(a);
    case 32: return launch_n<32, S>(a);
    case 64: return launch_n<64, S>(a);
    case 128: return launch_n<128, S>(a);
    case 256: return launch_n<256, S>(a);
    case 512: return launch_n<512, S>(a);
    case 1024: return launch_n<1024, S>(a);
    case 2048: return launch_n<2048, S>(a);
    case 4096: return launch_n<4096, S>(a);
  }
  return hipErrorInvalidValue;
}

size_t lds_for(int L, int M, int NH) {
  switch (L) {
    case 16: return GccShape<16>::lds_bytes(M, NH);
    case 32: return GccShape<32>::lds_bytes(M, NH);
    case 64: return GccShape<64>::lds_bytes(M, NH);
    case 128: return GccShape<128>::lds_bytes(M, NH);
    case 256: return GccShape<256>::lds_bytes(M, NH);
    case 512: return GccShape<512>::lds_bytes(M, NH);
    case 1024: return GccShape<1024>::lds_bytes(M, NH);
    case 2048: return GccShape<2048>::lds_bytes(M, NH);
    case 4096: return GccShape<4096>::lds_bytes(M, NH);
  }
  return ~size_t(0);
}

}  // namespace

bool gcc_ifft_supported(const PairArgs& a) {
  return a.method == FCC_METHOD_GCC && a.twiddle_r != nullptr && a.I <= a.r * a.N &&
         lds_for(a.r * a.N, a.M, a.N / 2) <= 160 * 1024;
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
