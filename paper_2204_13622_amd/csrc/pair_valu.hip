// Pair stage, plain FP32 vector-ALU form (Sec. 4): the reference GPU
// implementation of the low-rank path, and the direct eq. (2) comparator.
//
// One workgroup per frame.  The frame's M whitened spectra (packed real
// layout: slot 0 carries the DC and Nyquist bins) are decoded to FP32 bins
// 0 .. N/2 in LDS, together with the cropped bases p_hat (eq. 7).  One thread per
// pair forms R(f) = e_i(f) e_j(f)^* on the fly, folds it into x_s / x_d
// (eq. 8), accumulates the coefficients z_k of eq. (9) in chunks of eight
// components, adds each chunk's share of y = 2 Re{U z} to I registers, and
// keeps the first index of the largest value.
#include "device_common.hpp"
#include "kernels.hpp"

namespace fcc {
namespace {

constexpr int kThreads = 256;

template <class S, int IMAX, bool WRITE_Y, bool GCC>
__global__ __launch_bounds__(kThreads) void pair_valu_kernel(
    const typename S::T* __restrict__ spec, int M, int P, int N, int I, int D, int lag0,
    const uint8_t* __restrict__ pairs, const float* __restrict__ basis,
    const float* __restrict__ dict, const float2* __restrict__ lagw,
    int32_t* __restrict__ tdoa, float* __restrict__ yout) {
  extern __shared__ float smem[];
  const int F = N / 2 + 1, m = N / 4, Bs = m + 1;
  float2* sp = reinterpret_cast<float2*>(smem);
  float* bs = smem + 2 * M * F;
  const int64_t t = blockIdx.x;
  const int NH = N / 2;
  const typename S::T* src = spec + t * (int64_t)M * NH;
  // packed real spectrum: slot 0 = (e(0), e(N/2)), slot f = e(f)
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
  if (!GCC)
    for (int i = threadIdx.x; i < D * Bs; i += kThreads) bs[i] = basis[i];
  __syncthreads();

  for (int p = threadIdx.x; p < P; p += kThreads) {
    const float2* ei = sp + pairs[2 * p] * F;
    const float2* ej = sp + pairs[2 * p + 1] * F;
    float y[IMAX];
#pragma unroll
    for (int ii = 0; ii < IMAX; ++ii) y[ii] = 0.f;
    if (GCC) {
      // eq. (2): y(tau) = 2 Re{ sum_f R(f) exp(j 2 pi f tau / N) }
      for (int f = 0; f < F; ++f) {
        const float2 r = cmul_conj(ei[f], ej[f]);
#pragma unroll
        for (int ii = 0; ii < IMAX; ++ii) {
          if (ii < I) {
            const float2 w = lagw[ii * F + f];
            y[ii] += 2.f * (r.x * w.x - r.y * w.y);
          }
        }
      }
    } else {
      for (int k0 = 0; k0 < D; k0 += 8) {
        float a[8], b[8];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) a[kk] = b[kk] = 0.f;
        for (int f = 0; f < m; ++f) {
          const float2 r1 = cmul_conj(ei[f], ej[f]);
          const float2 r2 = cmul_conj(ei[N / 2 - f], ej[N / 2 - f]);
          const float2 xs = cadd(r1, r2), xd = csub(r1, r2);
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) {
            if (k0 + kk < D) {
              const float w = bs[(k0 + kk) * Bs + f];
              const float2 xv = (kk % 2 == 0) ? xs : xd;   // k0 is even: even kk symmetric
              a[kk] += w * xv.x;
              b[kk] += w * xv.y;
            }
          }
        }
        const float2 rc = cmul_conj(ei[m], ej[m]);
#pragma unroll
        for (int kk = 0; kk < 8; kk += 2) {
          if (k0 + kk < D) {
            const float w = bs[(k0 + kk) * Bs + m];
            a[kk] += w * rc.x;
            b[kk] += w * rc.y;
          }
        }
#pragma unroll
        for (int ii = 0; ii < IMAX; ++ii) {
          if (ii < I) {
            float acc = 0.f;
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
              if (k0 + kk < D) {
                acc += dict[ii * 2 * D + 2 * (k0 + kk)] * a[kk] +
                       dict[ii * 2 * D + 2 * (k0 + kk) + 1] * b[kk];
              }
            }
            y[ii] += acc;
          }
        }
      }
    }
    const int64_t row = t * P + p;
    if (WRITE_Y) {
      for (int ii = 0; ii < I; ++ii) yout[row * I + ii] = y[ii];
    } else {
      float best = y[0];
      int bi = 0;
#pragma unroll
      for (int ii = 1; ii < IMAX; ++ii) {
        if (ii < I && y[ii] > best) { best = y[ii]; bi = ii; }
      }
      tdoa[row] = bi - lag0;
    }
  }
}

template <class S, int IMAX, bool WY, bool GCC>
hipError_t launch4(const PairArgs& a, size_t lds) {
  auto k = pair_valu_kernel<S, IMAX, WY, GCC>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)a.T), dim3(kThreads), lds, a.stream,
                     static_cast<const typename S::T*>(a.spec), a.M, a.P, a.N, a.I, a.D,
                     a.lag0, a.pairs, a.basis32, a.dict, a.lagw, a.tdoa, a.y);
  return hipGetLastError();
}

template <class S, int IMAX>
hipError_t launch3(const PairArgs& a, size_t lds) {
  const bool wy = a.y != nullptr, gcc = a.method == FCC_METHOD_GCC;
  if (wy) return gcc ? launch4<S, IMAX, true, true>(a, lds) : launch4<S, IMAX, true, false>(a, lds);
  return gcc ? launch4<S, IMAX, false, true>(a, lds) : launch4<S, IMAX, false, false>(a, lds);
}

template <class S>
hipError_t launch2(const PairArgs& a, size_t lds) {
  if (a.I <= 16) return launch3<S, 16>(a, lds);
  if (a.I <= 32) return launch3<S, 32>(a, lds);
  if (a.I <= 64) return launch3<S, 64>(a, lds);
  return hipErrorInvalidValue;
}

}  // namespace

size_t pair_valu_lds_bytes(int M, int N, int D) {
  return sizeof(float2) * size_t(M) * (N / 2 + 1) + sizeof(float) * size_t(D) * (N / 4 + 1);
}

bool pair_valu_supported(const PairArgs& a) {
  return a.I <= 64 && pair_valu_lds_bytes(a.M, a.N, a.method == FCC_METHOD_GCC ? 0 : a.D) <= 160 * 1024;
}

hipError_t launch_pair_valu(const PairArgs& a) {
  if (a.T == 0) return hipSuccess;
  const size_t lds = pair_valu_lds_bytes(a.M, a.N, a.method == FCC_METHOD_GCC ? 0 : a.D);   // GCC stages no basis
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  switch (a.precision) {
    case FCC_FP32: return launch2<SpecF32>(a, lds);
    case FCC_BF16: return launch2<SpecBF16>(a, lds);
    case FCC_FP16: return launch2<SpecF16>(a, lds);
    case FCC_FP8_E4M3: return launch2<SpecE4M3>(a, lds);
  }
  return hipErrorInvalidValue;
}

}  // namespace fcc
