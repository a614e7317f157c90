// Launch templates of the pair stage on the matrix cores, single array: a
// persistent grid whose wavefronts walk the frames with a grid-sized stride.
// The method and the tiling are described in pair_mfma_core.hpp.  Each
// (storage, operand) combination is instantiated in a translation unit of its
// own (pair_mfma_<combination>.hip); pair_mfma.hip dispatches.
#pragma once
#include "pair_mfma_core.hpp"

namespace fcc {
namespace pair_mfma_detail {

using namespace pair_core;

template <class S, class OP, int KB, int TT, bool WRITE_Y, int kWaves, bool HALF>
__global__ __launch_bounds__(64 * kWaves, 2) void pair_mfma_kernel(
    const typename S::T* __restrict__ spec, int64_t T, int M, int P, int NH, int I, int lag0,
    int slab_words, const uint32_t* __restrict__ prow16, const float* __restrict__ gexp,
    const uint8_t* __restrict__ pairs, int32_t* __restrict__ tdoa, float* __restrict__ yout) {
  extern __shared__ uint32_t lds_all[];
  const int wave = threadIdx.x >> 6;
  stage_tables<KB, TT, HALF>(lds_all, NH, P, I, prow16, gexp, pairs, 64 * kWaves);
  __syncthreads();
  // one slab per wavefront: first the frame's spectra as FP16 pairs (16 rows
  // of NH + 4 slots, absent microphones zero), after the projection the lag rows
  uint32_t* slab = lds_all + head_words(4 * KB, NH, TT, P, HALF) + wave * slab_words;
  run_frames<S, KB, TT, WRITE_Y, OP, HALF>(lds_all, slab, spec, M, P, NH, I, lag0,
                                           (int64_t)blockIdx.x * kWaves + wave, T, (int64_t)gridDim.x * kWaves,
                                           tdoa, yout);
}

// operand types in use: FP16 for every storage type, or the storage type's own
inline bool native_operands(const PairArgs& a) {
  return a.operands == FCC_OPERANDS_STORAGE && a.precision != FCC_FP16;
}

inline int lag_tiles(const PairArgs& a) { return a.I <= 16 ? 1 : (a.I <= 32 ? 2 : 3); }

// 32-bit words of LDS one wavefront needs: the staged spectra or the lag rows
inline int slab_words(const PairArgs& a) {
  const int row = (native_operands(a) && a.precision == FCC_FP8_E4M3) ? slab_row_words<OpF8>(a.N / 2)
                                                                      : slab_row_words<OpF16>(a.N / 2);
  const int spec_words = 16 * row;
  const int y_words = lag_words(a.I, lag_tiles(a));   // lag rows of every microphone pair
  return spec_words > y_words ? spec_words : y_words;
}


inline size_t lds_bytes(const PairArgs& a, int waves, bool half = false) {
  return sizeof(uint32_t) *
         (size_t(head_words(a.Dpad, a.N / 2, lag_tiles(a), a.P, half)) + size_t(waves) * slab_words(a));
}

// Workgroup shape: four wavefronts when the block's LDS fits; else four with
// the basis rows kept once (FP16 operands); else three, else two.
struct BlockShape {
  int waves;
  bool half;
};
inline BlockShape block_shape(const PairArgs& a) {
  if (lds_bytes(a, 4) <= 160 * 1024) return {4, false};
  if (!native_operands(a) && lds_bytes(a, 4, true) <= 160 * 1024) return {4, true};
  for (int w : {3, 2})
    if (lds_bytes(a, w) <= 160 * 1024) return {w, false};
  return {0, false};
}
inline int block_waves(const PairArgs& a) { return block_shape(a).waves; }

template <class S, class OP, int KB, int TT, bool WY, int WV, bool HALF = false>
hipError_t launch5(const PairArgs& a) {
  auto k = pair_mfma_kernel<S, OP, KB, TT, WY, WV, HALF>;
  const size_t lds = lds_bytes(a, WV, HALF);
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
  const int64_t cap = int64_t(2) * cus * (WV == 2 ? 2 : 1);
  const int64_t blocks = need < cap ? need : cap;
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * WV), lds, a.stream,
                     static_cast<const typename S::T*>(a.spec), a.T, a.M, a.P, a.N / 2, a.I,
                     a.lag0, slab_words(a),
                     reinterpret_cast<const uint32_t*>(std::is_same<OP, OpF16>::value ? a.prow16 : a.prow_op),
                     std::is_same<OP, OpF16>::value ? a.gexp : a.gexp_op, a.pairs, a.tdoa, a.y);
  return hipGetLastError();
}

template <class S, class OP, int KB, int TT, bool WY>
hipError_t launch4(const PairArgs& a) {
  const BlockShape sh = block_shape(a);
  if constexpr (std::is_same<OP, OpF16>::value)
    if (sh.waves == 4 && sh.half) return launch5<S, OP, KB, TT, WY, 4, true>(a);
  switch (sh.waves) {
    case 4: return launch5<S, OP, KB, TT, WY, 4>(a);
    case 3: return launch5<S, OP, KB, TT, WY, 3>(a);
    default: return launch5<S, OP, KB, TT, WY, 2>(a);
  }
}

template <class S, class OP, int KB>
hipError_t launch3(const PairArgs& a) {
  const bool wy = a.y != nullptr;
  if (a.I <= 16) return wy ? launch4<S, OP, KB, 1, true>(a) : launch4<S, OP, KB, 1, false>(a);
  if (a.I <= 32) return wy ? launch4<S, OP, KB, 2, true>(a) : launch4<S, OP, KB, 2, false>(a);
  return wy ? launch4<S, OP, KB, 3, true>(a) : launch4<S, OP, KB, 3, false>(a);
}

template <class S, class OP = OpF16>
hipError_t launch2(const PairArgs& a) {
  // the tables hold exactly Dpad = 4 KB rows (zero beyond D)
  switch (a.Dpad / 4) {
    case 1: return launch3<S, OP, 1>(a);
    case 2: return launch3<S, OP, 2>(a);
    case 3: return launch3<S, OP, 3>(a);
    case 4: return launch3<S, OP, 4>(a);
    case 6: return launch3<S, OP, 6>(a);
    case 8: return launch3<S, OP, 8>(a);
  }
  return hipErrorInvalidValue;
}

}  // namespace pair_mfma_detail

// the launcher of one (storage, operand) combination
hipError_t launch_pair_mfma_f16(const PairArgs& a);
hipError_t launch_pair_mfma_bf16(const PairArgs& a);
hipError_t launch_pair_mfma_e4m3(const PairArgs& a);
hipError_t launch_pair_mfma_bf16_native(const PairArgs& a);
hipError_t launch_pair_mfma_e4m3_native(const PairArgs& a);

}  // namespace fcc
