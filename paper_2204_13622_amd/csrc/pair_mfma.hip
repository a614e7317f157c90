// Pair stage on the matrix cores (Sec. 4: eqs. 5-9 and the dictionary
// expansion), for up to 16 microphones, with FP16 operands and FP32
// accumulation.
//
// The projection of eq. (9) for all pairs of a frame at once.  With the
// full-length basis rows p_k(f), f = 0 .. N/2 (eq. 5; the cropped rows of
// eq. 7 mirrored by the symmetry of eq. 6),
//   z_k(i, j) = sum_f p_k(f) e_i(f) e_j(f)^*,      e = X / |X|.
// Writing a = Re e, b = Im e and rotating one operand, r_j = (1 + j) e_j =
// (a_j - b_j) + j (a_j + b_j),
//   H_k(i, j) = sum_f p_k(f) [a_i Re r_j + b_i Im r_j] = Re z_k(i,j) + Im z_k(i,j)
//   H_k(j, i) = Re z_k(i,j) - Im z_k(i,j)
// so every pair's coefficients come out of one real product (p_k . E) R^T
// whose K dimension runs over the interleaved (re, im) of the N/2 packed
// slots.  The pair products e_i e_j^* are formed inside the matrix core; the
// fold of eq. (8), which only halves scalar multiplications by p_k, has no
// work left to save here.  The expansion y = 2 Re{U z} becomes
//   y_ij(tau) = sum_k G(tau, k) H_k(i, j) + G(-tau, k) H_k(j, i),  G = Dc - Ds.
//
// Tiles: one wavefront per frame.  A 16x16x32 MFMA tile has rows
// (k, i) = (4 kb + row / 4, 4 ib + row % 4) and columns j = 0 .. 15, so its
// output register q of lane (g, col) holds H_{4kb+g}(4ib+q, col); that register
// is directly the B operand of a 16x16x4 FP32 MFMA over k, which applies G.
// The lag rows of every microphone go to LDS, where each pair adds its two
// halves and takes the first index of the largest value.
#include "device_common.hpp"
#include "kernels.hpp"

namespace fcc {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr int kWaves = 4;
constexpr int kYStride = 16 * 16 + 4;   // floats per lag row; the pad spreads LDS banks

// Four packed complex slots as eight FP16 values (re, im, re, im, ...).
template <class S> __device__ __forceinline__ h8 load8(const typename S::T* p);

template <> __device__ __forceinline__ h8 load8<SpecF16>(const uint32_t* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(h8, v);
}
template <> __device__ __forceinline__ h8 load8<SpecBF16>(const uint32_t* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  h8 out;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    out[2 * c] = (_Float16)__uint_as_float(w[c] << 16);
    out[2 * c + 1] = (_Float16)__uint_as_float(w[c] & 0xffff0000u);
  }
  return out;
}
template <> __device__ __forceinline__ h8 load8<SpecE4M3>(const uint16_t* p) {
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  h8 out;
  const f2 a = __builtin_amdgcn_cvt_pk_f32_fp8((int)v.x, false);
  const f2 b = __builtin_amdgcn_cvt_pk_f32_fp8((int)v.x, true);
  const f2 c = __builtin_amdgcn_cvt_pk_f32_fp8((int)v.y, false);
  const f2 d = __builtin_amdgcn_cvt_pk_f32_fp8((int)v.y, true);
  out[0] = (_Float16)a.x; out[1] = (_Float16)a.y;
  out[2] = (_Float16)b.x; out[3] = (_Float16)b.y;
  out[4] = (_Float16)c.x; out[5] = (_Float16)c.y;
  out[6] = (_Float16)d.x; out[7] = (_Float16)d.y;
  return out;
}

template <class S, int KB, int TT, bool WRITE_Y>
__global__ __launch_bounds__(64 * kWaves) void pair_mfma_kernel(
    const typename S::T* __restrict__ spec, int64_t T, int M, int P, int NH, int I, int tau_max,
    const uint32_t* __restrict__ prow16, const float* __restrict__ gexp,
    const uint8_t* __restrict__ pairs, int32_t* __restrict__ tdoa, float* __restrict__ yout) {
  extern __shared__ float ybuf_all[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;
  float* ybuf = ybuf_all + wave * I * kYStride;
  const int IB = (M + 3) >> 2;
  const int Dp = 4 * KB;

  // A operands of the expansion: G(tau = 16 tt + col, k = 4 kb + g)
  float gx[TT][KB];
#pragma unroll
  for (int tt = 0; tt < TT; ++tt)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) gx[tt][kb] = gexp[(16 * tt + col) * Dp + 4 * kb + g];

  const int64_t t = (int64_t)blockIdx.x * kWaves + wave;
  const bool active = t < T;
  if (active) {
    f4 acc[KB][4];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) acc[kb][ib] = f4{0.f, 0.f, 0.f, 0.f};

    const typename S::T* base = spec + t * (int64_t)M * NH;
    const int micA = col & 3;
    const h8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
    const h8 sgn = {-1, 1, -1, 1, -1, 1, -1, 1};
    for (int s = 0; s < NH / 16; ++s) {
      const int slot = 16 * s + 4 * g;
      const h8 raw = (col < M) ? load8<S>(base + col * NH + slot) : zero8;
      // B: the rotated spectrum (a - b, a + b) of microphone `col`; the packed
      // DC / Nyquist slot holds two real bins and enters unrotated.
      const h8 sw = __builtin_shufflevector(raw, raw, 1, 0, 3, 2, 5, 4, 7, 6);
      h8 B = raw + sw * sgn;
      if (s == 0 && g == 0) {
        B[0] = raw[0];
        B[1] = raw[1];
      }
      h8 Am[4];
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) {
        const int mic = 4 * ib + micA;
        Am[ib] = (ib < IB && mic < M) ? load8<S>(base + mic * NH + slot) : zero8;
      }
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const int k = 4 * kb + (col >> 2);
        const h8 pk = __builtin_bit_cast(h8, *reinterpret_cast<const uint4*>(prow16 + (size_t)k * NH + slot));
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
          if (ib < IB) acc[kb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Am[ib] * pk, B, acc[kb][ib], 0, 0, 0);
        }
      }
    }

    // expansion: Y_i(tau, j) = sum_k G(tau, k) H_k(i, j), one 16x16x4 chain per mic
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
      if (ib >= IB) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 4 * ib + q;
        if (i >= M) continue;
#pragma unroll
        for (int tt = 0; tt < TT; ++tt) {
          f4 Y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kb = 0; kb < KB; ++kb)
            Y = __builtin_amdgcn_mfma_f32_16x16x4f32(gx[tt][kb], acc[kb][ib][q], Y, 0, 0, 0);
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const int tau = 16 * tt + 4 * g + qq;
            if (tau < I) ybuf[tau * kYStride + i * 16 + col] = Y[qq];
          }
        }
      }
    }
  }
  __syncthreads();
  if (active) {
    for (int p = lane; p < P; p += 64) {
      const int i = pairs[2 * p], j = pairs[2 * p + 1];
      const int64_t row = t * P + p;
      float best = 0.f;
      int bi = 0;
      for (int tau = 0; tau < I; ++tau) {
        const float v = ybuf[tau * kYStride + i * 16 + j] + ybuf[(I - 1 - tau) * kYStride + j * 16 + i];
        if (WRITE_Y) yout[row * I + tau] = v;
        if (tau == 0 || v > best) {
          best = v;
          bi = tau;
        }
      }
      if (!WRITE_Y) tdoa[row] = bi - tau_max;
    }
  }
}

template <class S, int KB, int TT, bool WY>
hipError_t launch4(const PairArgs& a) {
  auto k = pair_mfma_kernel<S, KB, TT, WY>;
  const size_t lds = sizeof(float) * size_t(kWaves) * a.I * kYStride;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t blocks = (a.T + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * kWaves), lds, a.stream,
                     static_cast<const typename S::T*>(a.spec), a.T, a.M, a.P, a.N / 2, a.I,
                     a.tau_max, reinterpret_cast<const uint32_t*>(a.prow16), a.gexp, a.pairs,
                     a.tdoa, a.y);
  return hipGetLastError();
}

template <class S, int KB>
hipError_t launch3(const PairArgs& a) {
  const bool wy = a.y != nullptr;
  if (a.I <= 16) return wy ? launch4<S, KB, 1, true>(a) : launch4<S, KB, 1, false>(a);
  return wy ? launch4<S, KB, 2, true>(a) : launch4<S, KB, 2, false>(a);
}

template <class S>
hipError_t launch2(const PairArgs& a) {
  // the tables hold exactly Dpad = 4 KB rows (zero beyond D)
  switch (a.Dpad / 4) {
    case 1: return launch3<S, 1>(a);
    case 2: return launch3<S, 2>(a);
    case 3: return launch3<S, 3>(a);
    case 4: return launch3<S, 4>(a);
    case 6: return launch3<S, 6>(a);
    case 8: return launch3<S, 8>(a);
  }
  return hipErrorInvalidValue;
}

}  // namespace

bool pair_mfma_supported(const PairArgs& a) {
  const int kb = a.Dpad / 4;
  const bool kb_ok = a.Dpad % 4 == 0 && (kb == 1 || kb == 2 || kb == 3 || kb == 4 || kb == 6 || kb == 8);
  return a.method == FCC_METHOD_FCC && a.precision != FCC_FP32 && a.M <= 16 && a.N >= 32 &&
         a.D <= a.Dpad && kb_ok && a.I <= 32;
}

hipError_t launch_pair_mfma(const PairArgs& a) {
  if (a.T == 0) return hipSuccess;
  if (!pair_mfma_supported(a)) return hipErrorInvalidValue;
  switch (a.precision) {
    case FCC_FP16: return launch2<SpecF16>(a);
    case FCC_BF16: return launch2<SpecBF16>(a);
    case FCC_FP8_E4M3: return launch2<SpecE4M3>(a);
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace fcc
