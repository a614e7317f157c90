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
// Tiles: one wavefront per frame, which first stages the frame's spectra
// into its LDS slab as FP16 pairs.  A 16x16x32 MFMA tile has rows
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

template <class S, int KB, int TT, bool WRITE_Y, int kWaves>
__global__ __launch_bounds__(64 * kWaves, 2) void pair_mfma_kernel(
    const typename S::T* __restrict__ spec, int64_t T, int M, int P, int NH, int I, int lag0,
    int slab_words, const uint32_t* __restrict__ prow16, const float* __restrict__ gexp,
    const uint8_t* __restrict__ pairs, int32_t* __restrict__ tdoa, float* __restrict__ yout) {
  extern __shared__ uint32_t lds_all[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;
  constexpr int Dp = 4 * KB;
  // block-wide: the basis rows p_k (FP16 pairs per slot), then one slab per
  // wavefront holding first the frame's spectra as FP16 pairs (16 rows of
  // NH + 4 slots; rows of absent microphones are zero; the pad spreads rows
  // over the LDS banks) and, after the projection, the lag rows Y
  // basis rows are NH + 4 words apart so the four rows a wavefront reads at
  // once fall on different LDS banks
  // The dictionary G and the pair list also sit in LDS: inside the frame loop
  // the only global loads are the next frame's prefetch, so no wait on the
  // in-order load counter ever has to drain that prefetch early.
  const int prow_words = NH + 4;
  uint32_t* ptab = lds_all;
  float* gsh = reinterpret_cast<float*>(ptab + Dp * prow_words);        // [16 TT][Dp]
  uint32_t* psh = ptab + Dp * prow_words + 16 * TT * Dp;                // [P] = i | j << 8
  uint32_t* slab = lds_all + ((shared_words(Dp, NH, TT, P) + 3) & ~3) + wave * slab_words;   // 16-byte aligned
  float* ybuf = reinterpret_cast<float*>(slab);
  const int row = NH + 4;
  for (int c = threadIdx.x; c < Dp * NH / 4; c += 64 * kWaves) {
    const int k = c / (NH / 4), q = c - k * (NH / 4);
    *reinterpret_cast<uint4*>(ptab + k * prow_words + 4 * q) = reinterpret_cast<const uint4*>(prow16)[c];
  }
  for (int c = threadIdx.x; c < 16 * TT * Dp; c += 64 * kWaves) gsh[c] = gexp[c];
  for (int c = threadIdx.x; c < P; c += 64 * kWaves) psh[c] = pairs[2 * c] | (uint32_t(pairs[2 * c + 1]) << 8);
  __syncthreads();

  // a frame is M * NH / 4 chunks of 16 bytes (4 slots); chunk c is slots
  // 4 (c % (NH/4)) .. +3 of microphone c / (NH/4)
  const int lg_row = 31 - __builtin_clz(NH / 4);
  const int chunks = M * (NH / 4);
  const int rounds = chunks >> 6;              // full rounds of 64 chunks
  const int64_t stride = (int64_t)gridDim.x * kWaves;
  int64_t t = (int64_t)blockIdx.x * kWaves + wave;

  uint4 pre[kPrefetch];                        // first kPrefetch rounds, in flight
  auto prefetch = [&](int64_t tf) {
    const typename S::T* base = spec + tf * (int64_t)M * NH;
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u)
      if (u < rounds) pre[u] = load4<S>(base + 4 * (lane + 64 * u));
  };
  if (t < T) prefetch(t);

  const h8 sgn = {-1, 1, -1, 1, -1, 1, -1, 1};
  const int micA = col & 3;
  const int nsteps = NH / 16;

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
    const uint32_t* amic = slab + micA * row + 4 * g;
    const uint32_t* prow = ptab + (col >> 2) * prow_words + 4 * g;
    // one K step: 16 slots (32 interleaved re / im values); every tile of
    // four microphone blocks runs (rows of absent microphones are zero)
    auto kstep = [&](int off, bool dc_slot) {
      const h8 raw = __builtin_bit_cast(h8, *reinterpret_cast<const uint4*>(own + off));
      // B: the rotated spectrum (a - b, a + b) of microphone `col`; the packed
      // DC / Nyquist slot holds two real bins and enters unrotated.
      const h8 sw = __builtin_shufflevector(raw, raw, 1, 0, 3, 2, 5, 4, 7, 6);
      h8 B = raw + sw * sgn;
      if (dc_slot) {
        B[0] = raw[0];
        B[1] = raw[1];
      }
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
    };
    kstep(0, g == 0);
    for (int s = 1; s < nsteps; ++s) kstep(16 * s, false);
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
      float best = ya[0] + yb[0];
      int bi = 0;
      if (WRITE_Y) yout[orow * I] = best;
      for (int tau = 1; tau < I; ++tau) {
        const float v = ya[tau * kYStride] + yb[-tau * kYStride];
        if (WRITE_Y) yout[orow * I + tau] = v;
        if (v > best) {
          best = v;
          bi = tau;
        }
      }
      if (!WRITE_Y) tdoa[orow] = bi - lag0;
    }
    wave_sync();   // the slab is rewritten by the next frame
  }
}

// 32-bit words of LDS one wavefront needs: the staged spectra or the lag rows
int slab_words(const PairArgs& a) {
  const int spec_words = 16 * (a.N / 2 + 4);
  const int y_words = (a.I + 1) * kYStride;   // I lag rows and one row taking the padding
  return spec_words > y_words ? spec_words : y_words;
}

int lag_tiles(const PairArgs& a) { return a.I <= 16 ? 1 : (a.I <= 32 ? 2 : 3); }

size_t lds_bytes(const PairArgs& a, int waves) {
  // slabs hold uint4 rows: keep them 16-byte aligned
  const size_t head = (size_t(shared_words(a.Dpad, a.N / 2, lag_tiles(a), a.P)) + 3) & ~size_t(3);
  return sizeof(uint32_t) * (head + size_t(waves) * slab_words(a));
}

// wavefronts per block: four when the block's LDS fits, else two
int block_waves(const PairArgs& a) {
  if (lds_bytes(a, 4) <= 160 * 1024) return 4;
  if (lds_bytes(a, 2) <= 160 * 1024) return 2;
  return 0;
}

template <class S, int KB, int TT, bool WY, int WV>
hipError_t launch5(const PairArgs& a) {
  auto k = pair_mfma_kernel<S, KB, TT, WY, WV>;
  const size_t lds = lds_bytes(a, WV);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  // persistent wavefronts: enough blocks to fill the chip twice over, each
  // wavefront walking the frames with a grid-sized stride
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  const int64_t need = (a.T + WV - 1) / WV;
  const int64_t cap = int64_t(2) * cus * (4 / WV);
  const int64_t blocks = need < cap ? need : cap;
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * WV), lds, a.stream,
                     static_cast<const typename S::T*>(a.spec), a.T, a.M, a.P, a.N / 2, a.I,
                     a.lag0, slab_words(a), reinterpret_cast<const uint32_t*>(a.prow16), a.gexp,
                     a.pairs, a.tdoa, a.y);
  return hipGetLastError();
}

template <class S, int KB, int TT, bool WY>
hipError_t launch4(const PairArgs& a) {
  return block_waves(a) == 4 ? launch5<S, KB, TT, WY, 4>(a) : launch5<S, KB, TT, WY, 2>(a);
}

template <class S, int KB>
hipError_t launch3(const PairArgs& a) {
  const bool wy = a.y != nullptr;
  if (a.I <= 16) return wy ? launch4<S, KB, 1, true>(a) : launch4<S, KB, 1, false>(a);
  if (a.I <= 32) return wy ? launch4<S, KB, 2, true>(a) : launch4<S, KB, 2, false>(a);
  return wy ? launch4<S, KB, 3, true>(a) : launch4<S, KB, 3, false>(a);
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
         (reinterpret_cast<uintptr_t>(a.spec) % 16) == 0 &&
         a.D <= a.Dpad && kb_ok && a.I <= 48 && block_waves(a) > 0;
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
