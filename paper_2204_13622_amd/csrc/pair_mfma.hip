// Pair stage on the matrix cores, single array: a persistent grid whose
// wavefronts walk the frames with a grid-sized stride.  The method and the
// tiling are described in pair_mfma_core.hpp.
#include "pair_mfma_core.hpp"

namespace fcc {
namespace {

using namespace pair_core;

template <class S, int KB, int TT, bool WRITE_Y, int kWaves>
__global__ __launch_bounds__(64 * kWaves, 2) void pair_mfma_kernel(
    const typename S::T* __restrict__ spec, int64_t T, int M, int P, int NH, int I, int lag0,
    int slab_words, const uint32_t* __restrict__ prow16, const float* __restrict__ gexp,
    const uint8_t* __restrict__ pairs, int32_t* __restrict__ tdoa, float* __restrict__ yout) {
  extern __shared__ uint32_t lds_all[];
  const int wave = threadIdx.x >> 6;
  stage_tables<KB, TT>(lds_all, NH, P, prow16, gexp, pairs, 64 * kWaves);
  __syncthreads();
  // one slab per wavefront: first the frame's spectra as FP16 pairs (16 rows
  // of NH + 4 slots, absent microphones zero), after the projection the lag rows
  uint32_t* slab = lds_all + head_words(4 * KB, NH, TT, P) + wave * slab_words;
  run_frames<S, KB, TT, WRITE_Y>(lds_all, slab, spec, M, P, NH, I, lag0, (int64_t)blockIdx.x * kWaves + wave, T,
                                 (int64_t)gridDim.x * kWaves, tdoa, yout);
}

// 32-bit words of LDS one wavefront needs: the staged spectra or the lag rows
int slab_words(const PairArgs& a) {
  const int spec_words = 16 * (a.N / 2 + 4);
  const int y_words = (a.I + 1) * kYStride;   // I lag rows and one row taking the padding
  return spec_words > y_words ? spec_words : y_words;
}

int lag_tiles(const PairArgs& a) { return a.I <= 16 ? 1 : (a.I <= 32 ? 2 : 3); }

size_t lds_bytes(const PairArgs& a, int waves) {
  return sizeof(uint32_t) * (size_t(head_words(a.Dpad, a.N / 2, lag_tiles(a), a.P)) + size_t(waves) * slab_words(a));
}

// wavefronts per block: four when the block's LDS fits, else three, else two
int block_waves(const PairArgs& a) {
  for (int w : {4, 3, 2})
    if (lds_bytes(a, w) <= 160 * 1024) return w;
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
  const int64_t cap = int64_t(2) * cus * (WV == 2 ? 2 : 1);
  const int64_t blocks = need < cap ? need : cap;
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * WV), lds, a.stream,
                     static_cast<const typename S::T*>(a.spec), a.T, a.M, a.P, a.N / 2, a.I,
                     a.lag0, slab_words(a), reinterpret_cast<const uint32_t*>(a.prow16), a.gexp,
                     a.pairs, a.tdoa, a.y);
  return hipGetLastError();
}

template <class S, int KB, int TT, bool WY>
hipError_t launch4(const PairArgs& a) {
  switch (block_waves(a)) {
    case 4: return launch5<S, KB, TT, WY, 4>(a);
    case 3: return launch5<S, KB, TT, WY, 3>(a);
    default: return launch5<S, KB, TT, WY, 2>(a);
  }
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
