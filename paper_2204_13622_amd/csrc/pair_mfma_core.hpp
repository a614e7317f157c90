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
//
// Operand types of the projection tiles (OP):
//   OpF16  every storage type widened to FP16 in the slab (exact for
//          unit-modulus values), FP16 basis rows, 16x16x32 f16 tiles;
//   OpBF16 BF16 spectra kept as stored, BF16 basis rows, the products p_k e_i
//          and the rotated spectra formed in FP32 and rounded to BF16,
//          16x16x32 bf16 tiles;
//   OpF8   e4m3 spectra kept as stored (two bytes per slot), FP16 basis rows
//          scaled per component by a power of two, the products p_k e_i and
//          the rotated spectra formed in FP16 and rounded to e4m3,
//          16x16x32 fp8 tiles; the expansion table carries the inverse scales.
#pragma once
#include <type_traits>
#include "device_common.hpp"
#include "kernels.hpp"

namespace fcc {
namespace pair_core {


typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef __bf16 b2 __attribute__((ext_vector_type(2)));
typedef short s2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

// operand types of the projection tiles; slot_bytes: one complex slot in the slab
struct OpF16 { static constexpr int slot_bytes = 4; };
struct OpBF16 { static constexpr int slot_bytes = 4; };
struct OpF8 { static constexpr int slot_bytes = 2; };

// Lag rows in LDS, one lag tile (I <= 15): Y_i(tau, j) for every microphone
// pair (i, j), ordered as row r = 16 i + j of 16 words.  Lag index t sits at
// position pos = t + lag_shift(I, 1), which puts the mirrored lag I - 1 - t
// at 14 - pos (I is odd), so each pair reads its two rows with 16-byte loads
// and combines them at compile-time positions.  The groups of four positions
// of row r = 16 a + b are swizzled by ((b >> 1) ^ a) & 3 against bank
// conflicts, both where lanes run over b (expansion stores, Y_i(., j) reads)
// and where they run over a (the transposed Y_j(., i) reads).
__host__ __device__ constexpr int lag_shift(int I, int TT) { return TT == 1 ? (16 * TT - 1 - I) / 2 : 0; }
__host__ __device__ constexpr int lag_row_words(int TT) { return 16 * TT; }
__device__ __forceinline__ int lag_group(int r, int G) { return G ^ (((r >> 1) ^ (r >> 4)) & 3); }
// Two or three lag tiles: Y[tau][i][j] at tau * kYStride + i * kYRow + j; rows
// of 17 and a stride of 276 words keep both the writes (lanes over j) and the
// transposed reads (lanes over i) on distinct LDS banks.  This layout holds
// only the I lags (and one row taking the padding), which leaves room for
// more wavefronts at I < 32 than whole 16-position tiles would.
constexpr int kYRow = 17;
constexpr int kYStride = 276;
// 32-bit words of the lag rows
__host__ __device__ constexpr int lag_words(int I, int TT) {
  return TT == 1 ? 256 * lag_row_words(1) : (I + 1) * kYStride;
}

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

// One 16-byte slab chunk from storage: four slots widened to FP16 pairs
// (OpF16), or 16 / slot_bytes slots as stored (OpBF16, OpF8).
template <class S, class OP>
__device__ __forceinline__ uint4 load_chunk(const typename S::T* p) {
  if constexpr (std::is_same<OP, OpF16>::value) return load4<S>(p);
  else return *reinterpret_cast<const uint4*>(p);
}
// storage slots per slab chunk
template <class OP> constexpr int chunk_slots() { return 16 / OP::slot_bytes; }

// two FP32 values rounded to a BF16 pair (hardware round to nearest even)
__device__ __forceinline__ uint32_t pk_bf16(float lo, float hi) {
  const b2 v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}
// a BF16 pair word as two FP32 values
__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
// four e4m3 values (one word) as two FP16 pairs, and back
__device__ __forceinline__ h2 f8_lo(uint32_t w) { return __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w, 1.0f, false); }
__device__ __forceinline__ h2 f8_hi(uint32_t w) { return __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w, 1.0f, true); }
__device__ __forceinline__ uint32_t pk_f8(h2 lo, h2 hi) {
  s2 r = {0, 0};
  r = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(r, lo, 1.0f, false);
  r = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(r, hi, 1.0f, true);
  return __builtin_bit_cast(uint32_t, r);
}

// Memory ordering between the lanes of one wavefront (LDS written by some
// lanes, then read by others): a scheduling barrier fenced at wavefront scope.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// rounds of 16-byte chunks per lane in flight: a whole 16-microphone frame
// of N = 512 (16 KB per wavefront with 4-byte slots, 8 KB with e4m3 slots)
template <class OP> constexpr int prefetch_rounds() { return OP::slot_bytes == 4 ? 16 : 8; }

// 32-bit words of one microphone row of the slab (16-byte aligned, padded by
// four words so rows start on different banks)
template <class OP> __host__ __device__ constexpr int slab_row_words(int NH) {
  return NH * OP::slot_bytes / 4 + 4;
}

// 32-bit words of one basis row in LDS: FP16 pairs (p_k(f), p_k(f)) per slot
// (slot 0: (p_k(0), p_k(N/2))), or, compact (HALF), one FP16 value p_k(f) per
// slot with p_k(N/2) in the word after the row; four padding words keep the
// rows 16-byte aligned and on different banks
__host__ __device__ constexpr int prow_words_of(int NH, bool half) { return half ? NH / 2 + 4 : NH + 4; }

// 32-bit words of LDS shared by the workgroup: basis rows, G, pair list
__host__ __device__ __forceinline__ int shared_words(int Dp, int NH, int TT, int P, bool half = false) {
  return Dp * prow_words_of(NH, half) + 16 * TT * Dp + P;
}

// Block-wide: the tables one array's frames need, staged into LDS.  The
// basis rows p_k are prow_words_of(NH) words apart so the four rows a
// wavefront reads at once fall on different banks; the dictionary G and the
// pair list also sit in LDS, so inside the frame loop the only global loads
// are the next frame's prefetch and no wait on the in-order load counter ever
// has to drain that prefetch early.  HALF keeps each basis value once (half
// the table), for frame sizes whose slabs need the room.
template <int KB, int TT, bool HALF = false>
__device__ __forceinline__ void stage_tables(uint32_t* lds_all, int NH, int P, int I,
                                             const uint32_t* __restrict__ prow16, const float* __restrict__ gexp,
                                             const uint8_t* __restrict__ pairs, int nthreads) {
  constexpr int Dp = 4 * KB;
  const int prow_words = prow_words_of(NH, HALF);
  uint32_t* ptab = lds_all;
  float* gsh = reinterpret_cast<float*>(ptab + Dp * prow_words);        // [16 TT][Dp]
  uint32_t* psh = ptab + Dp * prow_words + 16 * TT * Dp;                // [P] = i | j << 8
  if constexpr (HALF) {
    for (int c = threadIdx.x; c < Dp * (NH / 2); c += nthreads) {      // two slots' p_k(f) per word
      const int k = c / (NH / 2), q = c - k * (NH / 2);
      const uint32_t w0 = prow16[k * NH + 2 * q], w1 = prow16[k * NH + 2 * q + 1];
      ptab[k * prow_words + q] = (w0 & 0xffffu) | (w1 << 16);
    }
    for (int k = threadIdx.x; k < Dp; k += nthreads) ptab[k * prow_words + NH / 2] = prow16[k * NH] >> 16;
  } else {
    for (int c = threadIdx.x; c < Dp * NH / 4; c += nthreads) {
      const int k = c / (NH / 4), q = c - k * (NH / 4);
      *reinterpret_cast<uint4*>(ptab + k * prow_words + 4 * q) = reinterpret_cast<const uint4*>(prow16)[c];
    }
  }
  // G row of lag index t at position t + lag_shift (zero rows elsewhere; no
  // shift for two or three lag tiles)
  const int sh = lag_shift(I, TT);
  for (int c = threadIdx.x; c < 16 * TT * Dp; c += nthreads) {
    const int tl = c / Dp - sh;
    gsh[c] = (tl >= 0 && tl < I) ? gexp[c - sh * Dp] : 0.f;
  }
  for (int c = threadIdx.x; c < P; c += nthreads) psh[c] = pairs[2 * c] | (uint32_t(pairs[2 * c + 1]) << 8);
}

// 32-bit words, 16-byte aligned, before the first wavefront slab
__host__ __device__ __forceinline__ int head_words(int Dp, int NH, int TT, int P, bool half = false) {
  return (shared_words(Dp, NH, TT, P, half) + 3) & ~3;
}

// The FP16 pairs of basis row 4 kb + col / 4 at a lane's four slots of K
// step offset poff: prow points at the lane's slots of row col / 4, prow_n2
// at that row's p(N/2) (compact rows only, where slot 0 pairs p(0) with it).
template <bool HALF>
__device__ __forceinline__ h8 basis_pairs(const uint32_t* prow, const _Float16* prow_n2, int prow_words, int kb,
                                          int poff, bool dc_slot) {
  if constexpr (HALF) {
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    const h4 v = __builtin_bit_cast(h4, *reinterpret_cast<const uint2*>(prow + 4 * kb * prow_words + poff));
    h8 r = __builtin_shufflevector(v, v, 0, 0, 1, 1, 2, 2, 3, 3);
    if (dc_slot) r[1] = prow_n2[2 * 4 * kb * prow_words];
    return r;
  } else {
    return __builtin_bit_cast(h8, *reinterpret_cast<const uint4*>(prow + 4 * kb * prow_words + poff));
  }
}

// One K step of the projection with FP16 operands: 16 slots (32 interleaved
// re / im values) of every microphone.  own: this lane's four slots of
// microphone `col` (the B operand); amic: the A rows' slots of microphone
// (col & 3) in block 0, blocks 4 rows apart; pk(kb): the FP16 pairs of basis
// row 4 kb + col / 4 at the lane's four slots.  ALL: every block of four
// microphones holds one (all four run, A rows loaded first); otherwise only
// blocks ib < nib run (rows of absent microphones have nothing to add).
// dc_slot: the lane's first slot is the packed DC / Nyquist slot, whose two
// real bins enter unrotated.
template <int KB, bool ALL, class PK>
__device__ __forceinline__ void kstep_f16(f4 (&acc)[KB][4], const uint32_t* own, const uint32_t* amic, int row,
                                          int nib, bool dc_slot, PK&& pk_of) {
  const h8 sgn = {-1, 1, -1, 1, -1, 1, -1, 1};
  const h8 raw = __builtin_bit_cast(h8, *reinterpret_cast<const uint4*>(own));
  // B: the rotated spectrum (a - b, a + b) of microphone `col`
  const h8 sw = __builtin_shufflevector(raw, raw, 1, 0, 3, 2, 5, 4, 7, 6);
  h8 B = __builtin_elementwise_fma(sw, sgn, raw);   // exact product by -1 / 1: one rounding
  if (dc_slot) {
    B[0] = raw[0];
    B[1] = raw[1];
  }
  if constexpr (ALL) {
    h8 Am[4];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) Am[ib] = __builtin_bit_cast(h8, *reinterpret_cast<const uint4*>(amic + 4 * ib * row));
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const h8 pk = pk_of(kb);
#pragma unroll
      for (int ib = 0; ib < 4; ++ib)
        acc[kb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Am[ib] * pk, B, acc[kb][ib], 0, 0, 0);
    }
  } else {
    h8 pk[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) pk[kb] = pk_of(kb);
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
      if (ib < nib) {
        const h8 Am = __builtin_bit_cast(h8, *reinterpret_cast<const uint4*>(amic + 4 * ib * row));
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
          acc[kb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Am * pk[kb], B, acc[kb][ib], 0, 0, 0);
      }
    }
  }
}

// Expansion of one block of four microphones: Y_i(tau, j) = sum_k G(tau, k)
// H_k(i, j) for i = 4 ib + q.  h[kb] holds the block's projection tile kb
// (register q of lane (g, col): H_{4kb+g}(4ib+q, col)), gx the A operands
// G(position 16 tt + col, k = 4 kb + g); the outputs of lane (g, col) are
// positions 16 tt + 4 g .. + 3 of row 16 i + col of the lag rows in ybuf.
template <int KB, int TT>
__device__ __forceinline__ void expand_block(const f4 (&h)[KB], const float (&gx)[TT][KB], float* ybuf, int ib,
                                             int g, int col, int I) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 16 * (4 * ib + q) + col;
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
      f4 Y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) Y = __builtin_amdgcn_mfma_f32_16x16x4f32(gx[tt][kb], h[kb][q], Y, 0, 0, 0);
      if constexpr (TT == 1) {
        *reinterpret_cast<f4*>(ybuf + r * lag_row_words(1) + 4 * lag_group(r, g)) = Y;
      } else {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {  // rows tau >= I are padding: all go to row I, never read
          const int tau = 16 * tt + 4 * g + qq;
          ybuf[(tau < I ? tau : I) * kYStride + (4 * ib + q) * kYRow + col] = Y[qq];
        }
      }
    }
  }
}

// One pair (i, j) of output row `orow`: y_ij(t) = Y_i(t, j) + Y_j(I - 1 - t, i)
// from the lag rows, then the first index of the largest value (tdoa, as a
// lag relative to lag0) or every lag (yout).
template <int TT, bool WRITE_Y>
__device__ __forceinline__ void pair_peak(const float* ybuf, uint32_t ij, int I, int lag0, int64_t orow,
                                          int32_t* __restrict__ tdoa, float* __restrict__ yout) {
  const int i = ij & 0xff, j = ij >> 8;
  if constexpr (TT == 1) {
    const int sh = lag_shift(I, 1);
    const int r1 = 16 * i + j, r2 = 16 * j + i;
    float v1[16], v2[16];
#pragma unroll
    for (int G = 0; G < 4; ++G) {
      const f4 a = *reinterpret_cast<const f4*>(ybuf + r1 * lag_row_words(1) + 4 * lag_group(r1, G));
      const f4 c = *reinterpret_cast<const f4*>(ybuf + r2 * lag_row_words(1) + 4 * lag_group(r2, G));
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v1[4 * G + e] = a[e];
        v2[4 * G + e] = c[e];
      }
    }
    float best = -__builtin_inff();
    int bi = 0;
#pragma unroll
    for (int pos = 0; pos < 15; ++pos) {
      const float y = v1[pos] + v2[14 - pos];
      const bool valid = pos >= sh && pos < sh + I;
      if (valid && y > best) {
        best = y;
        bi = pos;
      }
      if (WRITE_Y && valid) yout[orow * I + (pos - sh)] = y;
    }
    if (!WRITE_Y) tdoa[orow] = bi - sh - lag0;
  } else {
    const float* ya = ybuf + i * kYRow + j;
    const float* yb = ybuf + (I - 1) * kYStride + j * kYRow + i;
    // all lag reads issue together (compile-time bound, guarded), then the
    // first-index argmax
    float y[16 * TT];
#pragma unroll
    for (int tau = 0; tau < 16 * TT; ++tau) y[tau] = tau < I ? ya[tau * kYStride] + yb[-tau * kYStride] : 0.f;
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
}

// One wavefront runs the frames t = first, first + step, ... < end of one
// array (spectra `spec`, outputs `tdoa` / `yout` indexed t * P + p), with the
// array's tables already in LDS and `slab` its own LDS slab.
template <class S, int KB, int TT, bool WRITE_Y, class OP = OpF16, bool HALF = false>
__device__ __forceinline__ void run_frames(const uint32_t* lds_all, uint32_t* slab, const typename S::T* __restrict__ spec,
                                           int M, int P, int NH, int I, int lag0, int64_t first, int64_t end,
                                           int64_t step, int32_t* __restrict__ tdoa, float* __restrict__ yout) {
  constexpr bool kF16 = std::is_same<OP, OpF16>::value;
  constexpr bool kBF16 = std::is_same<OP, OpBF16>::value;
  constexpr int kPre = prefetch_rounds<OP>();
  constexpr int CS = chunk_slots<OP>();          // storage slots per 16-byte chunk
  static_assert(!HALF || kF16, "compact basis rows are built for FP16 operands");
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;
  constexpr int Dp = 4 * KB;
  const int prow_words = prow_words_of(NH, HALF);
  const uint32_t* ptab = lds_all;
  const float* gsh = reinterpret_cast<const float*>(ptab + Dp * prow_words);
  const uint32_t* psh = ptab + Dp * prow_words + 16 * TT * Dp;
  float* ybuf = reinterpret_cast<float*>(slab);
  const int row = slab_row_words<OP>(NH);
  const int64_t T = end, stride = step;
  int64_t t = first;
  // a frame is M * NH / CS chunks of 16 bytes; chunk c is slots
  // CS (c % (NH/CS)) .. +CS-1 of microphone c / (NH/CS)
  const int lg_row = 31 - __builtin_clz(NH / CS);
  const int chunks = M * (NH / CS);
  const int rounds = chunks >> 6;              // full rounds of 64 chunks

  uint4 pre[kPre];                             // first kPre rounds, in flight
  auto prefetch = [&](int64_t tf) {
    const typename S::T* base = spec + tf * (int64_t)M * NH;
    if (rounds >= kPre) {                       // every slot in use: no guards
#pragma unroll
      for (int u = 0; u < kPre; ++u) pre[u] = load_chunk<S, OP>(base + CS * (lane + 64 * u));
    } else {
#pragma unroll
      for (int u = 0; u < kPre; ++u)
        if (u < rounds) pre[u] = load_chunk<S, OP>(base + CS * (lane + 64 * u));
    }
  };
  if (t < T) prefetch(t);

  const h2 sgn2 = {-1, 1};
  const int nsteps = NH / 16;
  const int nib = (M + 3) >> 2;                 // blocks of four microphones holding any microphone
  // words of one K step (16 slots) in the slab, and a lane's offset inside it
  constexpr int step_words = 4 * OP::slot_bytes;
  constexpr int lane_words = OP::slot_bytes;   // four slots per lane: 4 * slot_bytes / 4 words
  constexpr int pstep = HALF ? 8 : 16;          // words of one K step in a basis row

  for (; t < T; t += stride) {
    // ---- stage the frame into the slab --------------------------------------
    const typename S::T* base = spec + t * (int64_t)M * NH;
    if (rounds >= kPre && lg_row == 6) {        // one round per microphone row (1 KB rows of
                                                // 260 words): microphone u, immediate offsets
#pragma unroll
      for (int u = 0; u < kPre; ++u) *reinterpret_cast<uint4*>(slab + 4 * lane + 260 * u) = pre[u];
    } else if (rounds >= kPre) {                // every prefetch slot holds data: no guards
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int c = lane + 64 * u;
        const int mic = c >> lg_row, q = c & ((NH / CS) - 1);
        *reinterpret_cast<uint4*>(slab + mic * row + 4 * q) = pre[u];
      }
    } else {
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        if (u < rounds) {
          const int c = lane + 64 * u;
          const int mic = c >> lg_row, q = c & ((NH / CS) - 1);
          *reinterpret_cast<uint4*>(slab + mic * row + 4 * q) = pre[u];
        }
      }
    }
    for (int c = lane + 64 * (rounds < kPre ? rounds : kPre); c < chunks; c += 64) {
      const uint4 v = load_chunk<S, OP>(base + CS * c);
      const int mic = c >> lg_row, q = c & ((NH / CS) - 1);
      *reinterpret_cast<uint4*>(slab + mic * row + 4 * q) = v;
    }
    for (int c = M * row + lane * 4; c < 16 * row; c += 256)   // absent microphones
      *reinterpret_cast<uint4*>(slab + c) = make_uint4(0, 0, 0, 0);
    wave_sync();
    if (t + stride < T) prefetch(t + stride);   // next frame flies during this one

    // ---- projection: H_k = (p_k . E) R^T on 16x16x32 tiles -------------------
    f4 acc[KB][4];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) acc[kb][ib] = f4{0.f, 0.f, 0.f, 0.f};

    const uint32_t* own = slab + col * row + lane_words * g;
    const uint32_t* amic = slab + (col & 3) * row + lane_words * g;
    const uint32_t* prow = ptab + (col >> 2) * prow_words + (HALF ? 2 : 4) * g;
    const _Float16* prow_n2 = reinterpret_cast<const _Float16*>(ptab + (col >> 2) * prow_words + NH / 2);
    auto load_pk = [&](int kb, int poff, bool dc_slot) -> h8 {
      return basis_pairs<HALF>(prow, prow_n2, prow_words, kb, poff, dc_slot);
    };
    // one K step: 16 slots (32 interleaved re / im values).  ALL: every block
    // of four microphones holds one (all four blocks run, A rows loaded
    // first); otherwise only the blocks that hold any run (rows of absent
    // microphones are zero and have nothing to add).  soff: the step's word
    // offset in the slab, poff in the basis rows (FP16 or BF16 pairs).
    auto kstep = [&](auto all, int soff, int poff, bool dc_slot) {
      if constexpr (kF16) {
        kstep_f16<KB, decltype(all)::value>(acc, own + soff, amic + soff, row, nib, dc_slot,
                                            [&](int kb) { return load_pk(kb, poff, dc_slot); });
      } else if constexpr (kBF16) {
        // BF16 pairs: the rotation and the products in FP32, rounded to BF16
        const uint4 rw = *reinterpret_cast<const uint4*>(own + soff);
        const uint32_t w[4] = {rw.x, rw.y, rw.z, rw.w};
        uint32_t bw[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float a = bf_lo(w[u]), b = bf_hi(w[u]);
          bw[u] = (u == 0 && dc_slot) ? w[u] : pk_bf16(a - b, a + b);
        }
        const b8 B = __builtin_bit_cast(b8, make_uint4(bw[0], bw[1], bw[2], bw[3]));
        float pf[KB][8];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const uint4 pw = *reinterpret_cast<const uint4*>(prow + 4 * kb * prow_words + poff);
          const uint32_t pv[4] = {pw.x, pw.y, pw.z, pw.w};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            pf[kb][2 * u] = bf_lo(pv[u]);
            pf[kb][2 * u + 1] = bf_hi(pv[u]);
          }
        }
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
          if (decltype(all)::value || ib < nib) {
            const uint4 aw = *reinterpret_cast<const uint4*>(amic + 4 * ib * row + soff);
            const uint32_t av[4] = {aw.x, aw.y, aw.z, aw.w};
            float ef[8];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              ef[2 * u] = bf_lo(av[u]);
              ef[2 * u + 1] = bf_hi(av[u]);
            }
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
              uint32_t A[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) A[u] = pk_bf16(ef[2 * u] * pf[kb][2 * u], ef[2 * u + 1] * pf[kb][2 * u + 1]);
              acc[kb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  __builtin_bit_cast(b8, make_uint4(A[0], A[1], A[2], A[3])), B, acc[kb][ib], 0, 0, 0);
            }
          }
        }
      } else {
        // e4m3 slots: decoded to FP16 pairs, rotation and products in FP16,
        // rounded back to e4m3 for the fp8 tiles
        const uint2 rw = *reinterpret_cast<const uint2*>(own + soff);
        h2 e[4] = {f8_lo(rw.x), f8_hi(rw.x), f8_lo(rw.y), f8_hi(rw.y)};   // slots 4g .. 4g + 3
        h2 r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const h2 sw = __builtin_shufflevector(e[u], e[u], 1, 0);
          r[u] = e[u] + sw * sgn2;
        }
        if (dc_slot) r[0] = e[0];
        const long B = (long)pk_f8(r[0], r[1]) | ((long)pk_f8(r[2], r[3]) << 32);
        h2 pk[KB][4];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const uint4 pw = *reinterpret_cast<const uint4*>(prow + 4 * kb * prow_words + poff);
          pk[kb][0] = __builtin_bit_cast(h2, pw.x);
          pk[kb][1] = __builtin_bit_cast(h2, pw.y);
          pk[kb][2] = __builtin_bit_cast(h2, pw.z);
          pk[kb][3] = __builtin_bit_cast(h2, pw.w);
        }
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
          if (decltype(all)::value || ib < nib) {
            const uint2 aw = *reinterpret_cast<const uint2*>(amic + 4 * ib * row + soff);
            const h2 a[4] = {f8_lo(aw.x), f8_hi(aw.x), f8_lo(aw.y), f8_hi(aw.y)};
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
              const long A = (long)pk_f8(a[0] * pk[kb][0], a[1] * pk[kb][1]) |
                             ((long)pk_f8(a[2] * pk[kb][2], a[3] * pk[kb][3]) << 32);
              acc[kb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(A, B, acc[kb][ib], 0, 0, 0);
            }
          }
        }
      }
    };
    auto project = [&](auto all) {
      if (kF16 && KB <= 3 && KB * TT <= 6 && nsteps >= 2) {   // two K steps per trip (nsteps = N/32 is a
                                                            // power of two); wider tiles have no registers to spare
        for (int s = 0; s < nsteps; s += 2) {
          kstep(all, step_words * s, pstep * s, s == 0 && g == 0);
          kstep(all, step_words * s + step_words, pstep * s + pstep, false);
        }
      } else {
        kstep(all, 0, 0, g == 0);
        for (int s = 1; s < nsteps; ++s) kstep(all, step_words * s, pstep * s, false);
      }
    };
    if (nib == 4)
      project(std::true_type{});
    else
      project(std::false_type{});
    wave_sync();   // every lane has read the spectra; the slab now takes Y

    // ---- expansion: Y_i(tau, j) = sum_k G(tau, k) H_k(i, j) --------------------
    // A operands: G(position 16 tt + col, k = 4 kb + g); the output registers
    // of lane (g, col) hold positions 16 tt + 4 g .. + 3 of row 16 i + col
    float gx[TT][KB];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) gx[tt][kb] = gsh[(16 * tt + col) * Dp + 4 * kb + g];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
      if (ib >= nib) continue;                  // rows i >= M are never read
      f4 h[KB];
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) h[kb] = acc[kb][ib];
      expand_block<KB, TT>(h, gx, ybuf, ib, g, col, I);
    }
    wave_sync();

    // ---- per pair: y_ij(t) = Y_i(t, j) + Y_j(I - 1 - t, i); first-index argmax
    for (int p = lane; p < P; p += 64) pair_peak<TT, WRITE_Y>(ybuf, psh[p], I, lag0, t * P + p, tdoa, yout);
    wave_sync();   // the slab is rewritten by the next frame
  }
}

}  // namespace pair_core
}  // namespace fcc
