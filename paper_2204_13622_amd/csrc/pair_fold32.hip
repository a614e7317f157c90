// Pair stage in FP32 on the vector ALU, in the folded form of the paper
// (Sec. 4: eq. 8 fold, eq. 9 projection, y = 2 Re{U z}, argmax of Sec. 2).
//
// One workgroup per frame.  The frame's whitened spectra are unpacked to
// FP32 bins in LDS as folded pairs: for the folded bins f of a chunk, one
// row per microphone holds e(f), then e(N/2 - f), then the centre bin N/4.
// Lanes own pairs; the folded bins f < N/4 of each chunk are split between
// two groups of wavefronts, so within a wavefront every lane visits the same
// bin and the basis values p_hat_k(f) are wavefront-uniform (one scalar load
// of a contiguous row of the transposed table, no LDS traffic).  A frame is
// staged in chunks of folded bins, one after the other, so the LDS holds a
// part of it and more workgroups share a CU.  Per bin a lane forms
//   R(f) = e_i(f) e_j(f)^*,  R(N/2 - f),  x_s = R(f) + R(N/2 - f),  x_d = R(f) - R(N/2 - f)
// and accumulates z_k += p_hat_k(f) x_s (symmetric k) or p_hat_k(f) x_d
// (antisymmetric k).  The second group leaves its partial coefficients in
// LDS; the first adds them and the centre bin.  Outputs, by mode: the
// coefficients (a_k, b_k) themselves (optionally together with the
// interpolated lag, in one pass); or the expansion to the I lags through
// the dictionary (2 Dc, -2 Ds) followed by the first-index argmax, written as
// the integer lag, as the lag refined by quadratic interpolation around the
// maximum (Sec. 2), or as the correlation y itself.
//
// Storage types other than FP32 are decoded to FP32 while staging, so every
// precision can produce coefficients and interpolated lags.
#include "device_common.hpp"
#include "kernels.hpp"

namespace fcc {
namespace {

constexpr int kThreads = 256;
constexpr int kOutLag = 0, kOutCorr = 1, kOutCoef = 2, kOutParabolic = 3, kOutCoefParabolic = 4;

template <class S, int DB, int OUT, int NC>
__global__ __launch_bounds__(kThreads) void pair_fold32_kernel(
    const typename S::T* __restrict__ spec, int M, int P, int N, int I, int lag0, float inv_r, int overlay,
    const uint8_t* __restrict__ pairs, const float* __restrict__ pfold /*[N/4+1][DB]*/,
    const float* __restrict__ dict /*[I][2D]*/, int D, int32_t* __restrict__ tdoa,
    float* __restrict__ fout, float* __restrict__ fcoef) {
  extern __shared__ float smem[];
  const int NH = N / 2, m = N / 4;
  const int mc = m / NC, Fc = 2 * mc + 1;                 // folded bins per chunk, row length
  float2* sp = reinterpret_cast<float2*>(smem);          // [M][Fc]: e(f0 + q), e(NH - f0 - q), e(m)
  // [128][2 DB] partial sums of the second group: over the spectra when the
  // launch asks for it (one round of pairs covers the frame, so the spectra
  // have been read for the last time before)
  const bool one_round = overlay != 0;
  float* part = one_round ? smem : smem + 2 * M * Fc;
  const int64_t t = blockIdx.x;
  const typename S::T* src = spec + t * (int64_t)M * NH;
  // chunk c: folded bins f0 = c mc .. f0 + mc - 1 (the packed slot 0 holds
  // the real bins 0 and N/2)
  auto stage = [&](int c) {
    const int f0 = c * mc;
    const int lg = 31 - __builtin_clz(mc);               // mc is a power of two
    for (int x = threadIdx.x; x < M * mc; x += kThreads) {
      const int mic = x >> lg, q = x & (mc - 1), f = f0 + q;
      const typename S::T* row = src + mic * NH;
      float2 lo = spec_decode<S>(row[f]);
      float2 hi = spec_decode<S>(row[f == 0 ? 0 : NH - f]);
      if (f == 0) {
        lo.y = 0.f;
        hi = make_float2(hi.y, 0.f);
      }
      sp[mic * Fc + q] = lo;
      sp[mic * Fc + mc + q] = hi;
    }
    for (int mic = threadIdx.x; mic < M; mic += kThreads) sp[mic * Fc + 2 * mc] = spec_decode<S>(src[mic * NH + m]);
  };
  if constexpr (NC == 1) {
    stage(0);
    __syncthreads();
  }

  // lanes of the two halves: wavefronts [0, W/2) take the first half of each
  // chunk's folded bins, the rest the second half
  constexpr int W = kThreads / 64;
  const int wave = threadIdx.x >> 6;
  const int half = __builtin_amdgcn_readfirstlane(wave >= W / 2 ? 1 : 0);   // wavefront-uniform
  const int lane_in_half = threadIdx.x - half * (kThreads / 2);
  const int q0 = half ? mc / 2 : 0, q1 = half ? mc : mc / 2;

  for (int pbase = 0; pbase < P; pbase += kThreads / 2) {
    const int p = pbase + lane_in_half;
    const bool active = p < P;
    const int i = active ? pairs[2 * p] : 0, j = active ? pairs[2 * p + 1] : 0;
    const float2* ei = sp + i * Fc;
    const float2* ej = sp + j * Fc;
    float a[DB], b[DB];
#pragma unroll
    for (int k = 0; k < DB; ++k) a[k] = b[k] = 0.f;
    for (int c = 0; c < NC; ++c) {
      if constexpr (NC > 1) {                               // one round of pairs (P <= 128)
        if (c > 0) __syncthreads();                         // every lane has read chunk c - 1
        stage(c);
        __syncthreads();
      }
      const float* pc = pfold + c * mc * DB;
#pragma unroll 2
      for (int q = q0; q < q1; ++q) {
        const float2 r1 = cmul_conj(ei[q], ej[q]);
        const float2 r2 = cmul_conj(ei[mc + q], ej[mc + q]);
        const float2 xs = cadd(r1, r2), xd = csub(r1, r2);
        const float* pf = pc + q * DB;                      // one contiguous, wavefront-uniform row
#pragma unroll
        for (int k = 0; k < DB; ++k) {
          const float w = pf[k];
          const float2 xv = (k % 2 == 0) ? xs : xd;         // eq. (6) order: k even symmetric
          a[k] += w * xv.x;
          b[k] += w * xv.y;
        }
      }
    }
    const float2 rc = cmul_conj(ei[2 * mc], ej[2 * mc]);    // centre bin, symmetric k only
    if (one_round) __syncthreads();                         // every lane has read the spectra
    if (half) {
      if (active)
#pragma unroll
        for (int k = 0; k < DB; ++k) {
          part[lane_in_half * 2 * DB + 2 * k] = a[k];
          part[lane_in_half * 2 * DB + 2 * k + 1] = b[k];
        }
    }
    __syncthreads();
    if (!half && active) {
#pragma unroll
      for (int k = 0; k < DB; ++k) {
        a[k] += part[lane_in_half * 2 * DB + 2 * k];
        b[k] += part[lane_in_half * 2 * DB + 2 * k + 1];
        if (k % 2 == 0) {
          const float w = pfold[m * DB + k];
          a[k] += w * rc.x;
          b[k] += w * rc.y;
        }
      }
      const int64_t row = t * P + p;
      if (OUT == kOutCoef || OUT == kOutCoefParabolic) {
        for (int k = 0; k < D && k < DB; ++k) {
          fcoef[row * 2 * D + 2 * k] = a[k];
          fcoef[row * 2 * D + 2 * k + 1] = b[k];
        }
      }
      if (OUT != kOutCoef) {
        float best = 0.f, prev = 0.f, y_lo = 0.f, y_hi = 0.f;
        int bi = 0;
        for (int ii = 0; ii < I; ++ii) {
          const float* dr = dict + ii * 2 * D;
          float y = 0.f;
#pragma unroll
          for (int k = 0; k < DB; ++k)
            if (k < D) y += dr[2 * k] * a[k] + dr[2 * k + 1] * b[k];
          if (OUT == kOutCorr) fout[row * I + ii] = y;
          if (ii == 0 || y > best) {
            best = y;
            bi = ii;
            y_lo = prev;
          }
          if (ii == bi + 1) y_hi = y;
          prev = y;
        }
        if (OUT == kOutLag) tdoa[row] = bi - lag0;                  // units of 1/r sample
        if (OUT == kOutParabolic || OUT == kOutCoefParabolic) {
          // vertex of the parabola through (-1, y_lo), (0, best), (1, y_hi);
          // no refinement at the window edges or on a flat top
          float d = 0.f;
          const float den = y_lo - 2.f * best + y_hi;
          if (bi > 0 && bi < I - 1 && den != 0.f) d = 0.5f * (y_lo - y_hi) / den;
          fout[row] = ((float)(bi - lag0) + d) * inv_r;              // samples
        }
      }
    }
    __syncthreads();
  }
}

// LDS of one workgroup: the FP32 bins of one chunk and the second group's
// partial sums.  With one round of pairs the partial sums can take the
// spectra's place once the last chunk has been read.
//
// Chunks: when one round of pairs covers the frame, its folded bins are
// staged in two or four chunks, one after the other, so a workgroup's LDS
// drops to about 20 KB and a CU runs up to eight workgroups instead of one
// (N = 1024, whose whole frame took 82 KB) or four (N = 512).
int fold32_chunks(int M, int N, int P, int DB) {
  const int halfw = kThreads / 2;
  if (P > halfw || N < 64) return 1;
  const size_t part = sizeof(float) * size_t(P) * 2 * DB;
  for (int nc : {1, 2, 4}) {
    const size_t spec = sizeof(float) * 2 * size_t(M) * (2 * (N / 4 / nc) + 1);
    if ((spec > part ? spec : part) <= 20 * 1024 || (N / 4 / nc) <= 16) return nc;
  }
  return 4;
}

static size_t fold32_spec_floats(int M, int N, int P, int DB) {
  return 2 * size_t(M) * (2 * (N / 4 / fold32_chunks(M, N, P, DB)) + 1);
}

bool fold32_overlay(int M, int N, int P, int DB) {
  const int halfw = kThreads / 2;
  const int pslots = P < halfw ? P : halfw;
  const size_t spec = fold32_spec_floats(M, N, P, DB), part = size_t(pslots) * 2 * DB;
  return P <= halfw && sizeof(float) * (spec + part) <= 80 * 1024;
}

size_t fold32_lds(int M, int N, int P, int DB) {
  const int halfw = kThreads / 2;
  const int pslots = P < halfw ? P : halfw;
  const size_t spec = fold32_spec_floats(M, N, P, DB), part = size_t(pslots) * 2 * DB;
  return sizeof(float) * (fold32_overlay(M, N, P, DB) ? (spec > part ? spec : part) : spec + part);
}

template <class S, int DB, int OUT, int NC>
hipError_t launch4(const PairArgs& a) {
  auto k = pair_fold32_kernel<S, DB, OUT, NC>;
  const size_t lds = fold32_lds(a.M, a.N, a.P, DB);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  float* fout = OUT == kOutCorr ? a.y : a.tau_frac;
  hipLaunchKernelGGL(k, dim3((unsigned)a.T), dim3(kThreads), lds, a.stream,
                     static_cast<const typename S::T*>(a.spec), a.M, a.P, a.N, a.I, a.lag0, 1.f / (float)a.r,
                     fold32_overlay(a.M, a.N, a.P, DB) ? 1 : 0,
                     a.pairs, a.pfold, a.dict, a.D, a.tdoa, fout, a.coef);
  return hipGetLastError();
}

template <class S, int DB, int OUT>
hipError_t launch3(const PairArgs& a) {
  switch (fold32_chunks(a.M, a.N, a.P, DB)) {
    case 4: return launch4<S, DB, OUT, 4>(a);
    case 2: return launch4<S, DB, OUT, 2>(a);
    default: return launch4<S, DB, OUT, 1>(a);
  }
}

template <class S, int DB>
hipError_t launch2(const PairArgs& a) {
  if (a.coef && a.tau_frac) return launch3<S, DB, kOutCoefParabolic>(a);
  if (a.coef) return launch3<S, DB, kOutCoef>(a);
  if (a.tau_frac) return launch3<S, DB, kOutParabolic>(a);
  if (a.y) return launch3<S, DB, kOutCorr>(a);
  return launch3<S, DB, kOutLag>(a);
}

template <class S>
hipError_t launch1(const PairArgs& a) {
  switch (a.Dfold) {
    case 4: return launch2<S, 4>(a);
    case 8: return launch2<S, 8>(a);
    case 12: return launch2<S, 12>(a);
    case 16: return launch2<S, 16>(a);
    case 24: return launch2<S, 24>(a);
    case 32: return launch2<S, 32>(a);
    case 48: return launch2<S, 48>(a);
    case 64: return launch2<S, 64>(a);
  }
  return hipErrorInvalidValue;
}

}  // namespace

bool pair_fold32_supported(const PairArgs& a) {
  return a.method == FCC_METHOD_FCC && a.N >= 16 && a.Dfold >= a.D &&
         (a.Dfold == 4 || a.Dfold == 8 || a.Dfold == 12 || a.Dfold == 16 || a.Dfold == 24 ||
          a.Dfold == 32 || a.Dfold == 48 || a.Dfold == 64) &&
         fold32_lds(a.M, a.N, a.P, a.Dfold) <= 160 * 1024;
}

hipError_t launch_pair_fold32(const PairArgs& a) {
  if (a.T == 0) return hipSuccess;
  if (!pair_fold32_supported(a)) return hipErrorInvalidValue;
  switch (a.precision) {
    case FCC_FP32: return launch1<SpecF32>(a);
    case FCC_BF16: return launch1<SpecBF16>(a);
    case FCC_FP16: return launch1<SpecF16>(a);
    case FCC_FP8_E4M3: return launch1<SpecE4M3>(a);
  }
  return hipErrorInvalidValue;
}

}  // namespace fcc
