// Device code of the pair stage on the matrix cores (Sec. 4: eqs. 5-9 and the dictionary
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
// Tiles: one wavefront per frame, which first stages the frame's spectra
// into its LDS slab as FP16 pairs.  A 16x16x32 MFMA tile has rows
// (k, i) = (4 kb + row / 4, 4 ib + row % 4) and columns j = 0 .. 15, so its
// output register q of lane (g, col) holds H_{4kb+g}(4ib+q, col); that register
// is directly the B operand of a 16x16x4 FP32 MFMA over k, which applies G.
// The lag rows of every microphone go to LDS, where each pair adds its two
// halves and takes the first index of the largest value.
#pragma once
#include <type_traits>
#include "device_common.hpp"
#include "kernels.hpp"

namespace fcc {
namespace pair_core {


typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

// Lag rows Y[tau][i][j] live at tau * kYStride + i * kYRow + j: rows of 17
// and a stride of 276 words keep both the writes (lanes over j) and the
// transposed reads (lanes over i) on distinct LDS banks.
constexpr int kYRow = 17;
constexpr int kYStride = 276;

// Four packed complex slots as four FP16 pairs (re, im), from storage.
template <class S> __device__ __forceinline__ uint4 load4(const typename S::T* p);

template <> __device__ __forceinline__ uint4 load4<SpecF16>(const uint32_t* p) {
  return *reinterpret_cast<const uint4*>(p);
}
__device__ __forceinline__ uint32_t pack_h2(float lo, float hi) {
  const _Float16 a = (_Float16)lo, b = (_Float16)hi;
  return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}
template <> __device__ __forceinline__ uint4 load4<SpecBF16>(const uint32_t* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  // bf16 -> f32 is a shift; f32 -> f16 is exact for the unit-modulus range
  auto cv = [](uint32_t w) { return pack_h2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u)); };
  return make_uint4(cv(v.x), cv(v.y), cv(v.z), cv(v.w));
}
template <> __device__ __forceinline__ uint4 load4<SpecE4M3>(const uint16_t* p) {
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  const f2 a = __builtin_amdgcn_cvt_pk_f32_fp8((int)v.x, false);
  const f2 b = __builtin_amdgcn_cvt_pk_f32_fp8((int)v.x, true);
  const f2 c = __builtin_amdgcn_cvt_pk_f32_fp8((int)v.y, false);
  const f2 d = __builtin_amdgcn_cvt_pk_f32_fp8((int)v.y, true);
  return make_uint4(pack_h2(a.x, a.y), pack_h2(b.x, b.y), pack_h2(c.x, c.y), pack_h2(d.x, d.y));
}

// Memory ordering between the lanes of one wavefront (LDS written by some
// lanes, then read by others): a scheduling barrier fenced at wavefront scope.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kPrefetch = 16;   // rounds of 16-byte chunks per lane in flight (16 KB per wavefront)

// 32-bit words of LDS shared by the workgroup: basis rows, G, pair list
__host__ __device__ __forceinline__ int shared_words(int Dp, int NH, int TT, int P) {
  return Dp * (NH + 4) + 16 * TT * Dp + P;
}

// Block-wide: the tables one array's frames need, staged into LDS.  The
// basis rows p_k (FP16 pairs per slot) are NH + 4 words apart so the four rows
// a wavefront reads at once fall on different banks; the dictionary G and the
// pair list also sit in LDS, so inside the frame loop the only global loads
// are the next frame's prefetch and no wait on the in-order load counter ever
// has to drain that prefetch early.
template <int KB, int TT>
__device__ __forceinline__ void stage_tables(uint32_t* lds_all, int NH, int P, const uint32_t* __restrict__ prow16,
                                             const float* __restrict__ gexp, const uint8_t* __restrict__ pairs,
                                             int nthreads) {
  constexpr int Dp = 4 * KB;
  const int prow_words = NH + 4;
  uint32_t* ptab = lds_all;
  float* gsh = reinterpret_cast<float*>(ptab + Dp * prow_words);        // [16 TT][Dp]
  uint32_t* psh = ptab + Dp * prow_words + 16 * TT * Dp;                // [P] = i | j << 8
  for (int c = threadIdx.x; c < Dp * NH / 4; c += nthreads) {
    const int k = c / (NH / 4), q = c - k * (NH / 4);
    *reinterpret_cast<uint4*>(ptab + k * prow_words + 4 * q) = reinterpret_cast<const uint4*>(prow16)[c];
  }
  for (int c = threadIdx.x; c < 16 * TT * Dp; c += nthreads) gsh[c] = gexp[c];
  for (int c = threadIdx.x; c < P; c += nthreads) psh[c] = pairs[2 * c] | (uint32_t(pairs[2 * c + 1]) << 8);
}

// 32-bit words, 16-byte aligned, before the first wavefront slab
__host__ __device__ __forceinline__ int head_words(int Dp, int NH, int TT, int P) {
  return (shared_words(Dp, NH, TT, P) + 3) & ~3;
}

// One wavefront runs the frames t = first, first + step, ... < end of one
// array (spectra `spec`, outputs `tdoa` / `yout` indexed t * P + p), with the
// array's tables already in LDS and `slab` its own LDS slab.
template <class S, int KB, int TT, bool WRITE_Y>
__device__ __forceinline__ void run_frames(const uint32_t* lds_all, uint32_t* slab, const typename S::T* __restrict__ spec,
                                           int M, int P, int NH, int I, int lag0, int64_t first, int64_t end,
                                           int64_t step, int32_t* __restrict__ tdoa, float* __restrict__ yout) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;
  constexpr int Dp = 4 * KB;
  const int prow_words = NH + 4;
  const uint32_t* ptab = lds_all;
  const float* gsh = reinterpret_cast<const float*>(ptab + Dp * prow_words);
  const uint32_t* psh = ptab + Dp * prow_words + 16 * TT * Dp;
  float* ybuf = reinterpret_cast<float*>(slab);
  const int row = NH + 4;
  const int64_t T = end, stride = step;
  int64_t t = first;
  // a frame is M * NH / 4 chunks of 16 bytes (4 slots); chunk c is slots
  // 4 (c % (NH/4)) .. +3 of microphone c / (NH/4)
  const int lg_row = 31 - __builtin_clz(NH / 4);
  const int chunks = M * (NH / 4);
  const int rounds = chunks >> 6;              // full rounds of 64 chunks

  uint4 pre[kPrefetch];                        // first kPrefetch rounds, in flight
  auto prefetch = [&](int64_t tf) {
    const typename S::T* base = spec + tf * (int64_t)M * NH;
    if (rounds >= kPrefetch) {                  // every slot in use: no guards
#pragma unroll
      for (int u = 0; u < kPrefetch; ++u) pre[u] = load4<S>(base + 4 * (lane + 64 * u));
    } else {
#pragma unroll
      for (int u = 0; u < kPrefetch; ++u)
        if (u < rounds) pre[u] = load4<S>(base + 4 * (lane + 64 * u));
    }
  };
  if (t < T) prefetch(t);

  const h8 sgn = {-1, 1, -1, 1, -1, 1, -1, 1};
  const int nsteps = NH / 16;
  const int nib = (M + 3) >> 2;                 // blocks of four microphones holding any microphone

  for (; t < T; t += stride) {
    // ---- stage the frame into the slab --------------------------------------
    const typename S::T* base = spec + t * (int64_t)M * NH;
    if (rounds >= kPrefetch) {                  // every prefetch slot holds data: no guards
#pragma unroll
      for (int u = 0; u < kPrefetch; ++u) {
        const int c = lane + 64 * u;
        const int mic = c >> lg_row, q = c & ((NH / 4) - 1);
        *reinterpret_cast<uint4*>(slab + mic * row + 4 * q) = pre[u];
      }
    } else {
#pragma unroll
      for (int u = 0; u < kPrefetch; ++u) {
        if (u < rounds) {
          const int c = lane + 64 * u;
          const int mic = c >> lg_row, q = c & ((NH / 4) - 1);
          *reinterpret_cast<uint4*>(slab + mic * row + 4 * q) = pre[u];
        }
      }
    }
    for (int c = lane + 64 * (rounds < kPrefetch ? rounds : kPrefetch); c < chunks; c += 64) {
      const uint4 v = load4<S>(base + 4 * c);
      const int mic = c >> lg_row, q = c & ((NH / 4) - 1);
      *reinterpret_cast<uint4*>(slab + mic * row + 4 * q) = v;
    }
    for (int c = M * row + lane * 4; c < 16 * row; c += 256)   // absent microphones
      *reinterpret_cast<uint4*>(slab + c) = make_uint4(0, 0, 0, 0);
    wave_sync();
    if (t + stride < T) prefetch(t + stride);   // next frame flies during this one

    // ---- projection: H_k = (p_k . E) R^T on 16x16x32 FP16 tiles ------------
    f4 acc[KB][4];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) acc[kb][ib] = f4{0.f, 0.f, 0.f, 0.f};

    const uint32_t* own = slab + col * row + 4 * g;
    const uint32_t* amic = slab + (col & 3) * row + 4 * g;
    const uint32_t* prow = ptab + (col >> 2) * prow_words + 4 * g;
    // one K step: 16 slots (32 interleaved re / im values).  ALL: every block
    // of four microphones holds one (all four blocks run, A rows loaded
    // first); otherwise only the blocks that hold any run (rows of absent
    // microphones are zero and have nothing to add).
    auto kstep = [&](auto all, int off, bool dc_slot) {
      const uint4 rw = *reinterpret_cast<const uint4*>(own + off);
      const h8 raw = __builtin_bit_cast(h8, rw);
      // B: the rotated spectrum (a - b, a + b) of microphone `col`; the packed
      // DC / Nyquist slot holds two real bins and enters unrotated.
      const h8 sw = __builtin_shufflevector(raw, raw, 1, 0, 3, 2, 5, 4, 7, 6);
      h8 B = raw + sw * sgn;
      if (dc_slot) {
        B[0] = raw[0];
        B[1] = raw[1];
      }
      if constexpr (decltype(all)::value) {
        h8 Am[4];
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
          Am[ib] = __builtin_bit_cast(h8, *reinterpret_cast<const uint4*>(amic + 4 * ib * row + off));
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const h8 pk = __builtin_bit_cast(h8, *reinterpret_cast<const uint4*>(prow + 4 * kb * prow_words + off));
#pragma unroll
          for (int ib = 0; ib < 4; ++ib)
            acc[kb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Am[ib] * pk, B, acc[kb][ib], 0, 0, 0);
        }
      } else {
        h8 pk[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
          pk[kb] = __builtin_bit_cast(h8, *reinterpret_cast<const uint4*>(prow + 4 * kb * prow_words + off));
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
          if (ib < nib) {
            const h8 Am = __builtin_bit_cast(h8, *reinterpret_cast<const uint4*>(amic + 4 * ib * row + off));
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
              acc[kb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Am * pk[kb], B, acc[kb][ib], 0, 0, 0);
          }
        }
      }
    };
    auto project = [&](auto all) {
      if (KB <= 3 && KB * TT <= 6 && nsteps >= 2) {   // two K steps per trip (nsteps = N/32 is a power
                                                      // of two); wider tiles have no registers to spare
        for (int s = 0; s < nsteps; s += 2) {
          kstep(all, 16 * s, s == 0 && g == 0);
          kstep(all, 16 * s + 16, false);
        }
      } else {
        kstep(all, 0, g == 0);
        for (int s = 1; s < nsteps; ++s) kstep(all, 16 * s, false);
      }
    };
    if (nib == 4)
      project(std::true_type{});
    else
      project(std::false_type{});
    wave_sync();   // every lane has read the spectra; the slab now takes Y

    // ---- expansion: Y_i(tau, j) = sum_k G(tau, k) H_k(i, j) --------------------
    // A operands: G(tau = 16 tt + col, k = 4 kb + g)
    float gx[TT][KB];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) gx[tt][kb] = gsh[(16 * tt + col) * Dp + 4 * kb + g];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
      if (ib >= nib) continue;                  // rows i >= M are never read
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 4 * ib + q;
#pragma unroll
        for (int tt = 0; tt < TT; ++tt) {
          f4 Y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kb = 0; kb < KB; ++kb)
            Y = __builtin_amdgcn_mfma_f32_16x16x4f32(gx[tt][kb], acc[kb][ib][q], Y, 0, 0, 0);
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {  // rows tau >= I are padding: all go to row I, never read
            const int tau = 16 * tt + 4 * g + qq;
            ybuf[(tau < I ? tau : I) * kYStride + i * kYRow + col] = Y[qq];
          }
        }
      }
    }
    wave_sync();

    // ---- per pair: y_ij(tau) = Y_i(tau, j) + Y_j(-tau, i); first-index argmax
    for (int p = lane; p < P; p += 64) {
      const uint32_t ij = psh[p];
      const int i = ij & 0xff, j = ij >> 8;
      const int64_t orow = t * P + p;
      const float* ya = ybuf + i * kYRow + j;
      const float* yb = ybuf + (I - 1) * kYStride + j * kYRow + i;
      // all lag reads issue together (compile-time bound, guarded), then the
      // first-index argmax
      float y[16 * TT];
#pragma unroll
      for (int tau = 0; tau < 16 * TT; ++tau)
        y[tau] = tau < I ? ya[tau * kYStride] + yb[-tau * kYStride] : 0.f;
      float best = y[0];
      int bi = 0;
#pragma unroll
      for (int tau = 1; tau < 16 * TT; ++tau) {
        if (tau < I && y[tau] > best) {
          best = y[tau];
          bi = tau;
        }
      }
      if (WRITE_Y) {
#pragma unroll
        for (int tau = 0; tau < 16 * TT; ++tau)
          if (tau < I) yout[orow * I + tau] = y[tau];
      } else {
        tdoa[orow] = bi - lag0;
      }
    }
    wave_sync();   // the slab is rewritten by the next frame
  }
}

}  // namespace pair_core
}  // namespace fcc
