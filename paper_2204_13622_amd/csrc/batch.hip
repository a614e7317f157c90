// Many independent arrays of uneven microphone count, aperture, sample rate,
// frame size and rank in one pass.  Every array keeps its own plan tables
// (its slice of the batch image) and its own spectra and outputs; the work is
// cut into items that persistent workgroups take from atomic queues:
//   - front end: one launch for every array; an item is one block of
//     transforms (microphone-frames) of one array, handed out in chunks of
//     consecutive items so overlapping frames meet in the same L1 / L2;
//     the transform size is dispatched per item;
//   - pair stage: one launch per class of arrays that share the matrix-core
//     tile shape (components in blocks of four, lags in tiles of 16); an item
//     is a tile of consecutive frames of one array, whose tables the
//     workgroup stages into LDS when the array changes.
// The queues are counters in the workspace, cleared by a fill kernel, so the
// whole sequence can be captured in one graph.
#include "kernels.hpp"
#include "pair_mfma_core.hpp"
#include "stft_core.hpp"

namespace fcc {
namespace {

template <int N, class S>
__device__ __forceinline__ void stft_item(float2* lds, int& cur_N, const BatchArray& d, const unsigned char* image,
                                          const float* audio, unsigned char* spec_base, int64_t lblk) {
  using Sh = stft_core::StftShape<N>;
  float2* tw = lds;
  float2* tw1 = tw + N;
  float2* tw2 = tw1 + Sh::T1;
  float2* data = tw2 + Sh::T2;
  if (cur_N != N) {                 // the tables depend on N only
    stft_core::load_tables<N>(tw, tw1, tw2, reinterpret_cast<const float2*>(image + d.img_off + d.tab_twiddle));
    __syncthreads();
    cur_N = N;
  }
  stft_core::transforms<N, S, false>(tw, tw1, tw2, data, audio + d.audio_off, d.L, d.M, d.hop, d.T * d.M,
                                     reinterpret_cast<typename S::T*>(spec_base + d.spec_off), lblk);
}

template <class S>
__global__ __launch_bounds__(stft_core::kThreads) void batch_stft_kernel(
    const BatchArray* __restrict__ arrays, int n, int64_t total_items, int chunk,
    const unsigned char* __restrict__ image, const float* __restrict__ audio, unsigned char* __restrict__ spec_base,
    int* __restrict__ queue) {
  extern __shared__ float2 lds2[];
  __shared__ long long item_sh;
  int cur_N = 0;
  for (;;) {
    if (threadIdx.x == 0) item_sh = (long long)atomicAdd(queue, 1) * chunk;
    __syncthreads();
    const int64_t first = item_sh;
    __syncthreads();                                   // read before thread 0 takes the next chunk
    if (first >= total_items) break;                   // the same for every thread of the block
    const int64_t last = first + chunk < total_items ? first + chunk : total_items;
    for (int64_t it = first; it < last; ++it) {
      int lo = 0, hi = n - 1;                          // last array whose first item is <= it
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (arrays[mid].stft_first <= it) lo = mid;
        else hi = mid - 1;
      }
      const BatchArray& d = arrays[lo];
      const int64_t lblk = it - d.stft_first;
#define FCC_ITEM(NN)                                                    \
  case NN:                                                              \
    stft_item<NN, S>(lds2, cur_N, d, image, audio, spec_base, lblk);    \
    break;
      switch (d.N) {
        FCC_ITEM(16) FCC_ITEM(32) FCC_ITEM(64) FCC_ITEM(128) FCC_ITEM(256) FCC_ITEM(512) FCC_ITEM(1024)
        FCC_ITEM(2048)
      }
#undef FCC_ITEM
      __syncthreads();                                 // the scratch is reused by the next item
    }
  }
}

template <class S, int KB, int TT, int kWaves>
__global__ __launch_bounds__(64 * kWaves, 2) void batch_pair_kernel(
    const BatchArray* __restrict__ arrays, const int32_t* __restrict__ members, int n_members, int ft,
    const unsigned char* __restrict__ image, const unsigned char* __restrict__ spec_base,
    int32_t* __restrict__ tdoa_base, int* __restrict__ queue, int slab_words) {
  extern __shared__ uint32_t lds_all[];
  __shared__ int item_sh[3];
  const int wave = threadIdx.x >> 6;
  int cur = -1;
  for (;;) {
    if (threadIdx.x == 0) {
      // item -> (array, first frame, end frame): walk the class's arrays
      int rem = atomicAdd(queue, 1), a = -1, t0 = 0, t1 = 0;
      for (int c = 0; c < n_members; ++c) {
        const int m = members[c];
        const int64_t T = arrays[m].T;
        const int tiles = (int)((T + ft - 1) / ft);
        if (rem < tiles) {
          a = m;
          t0 = rem * ft;
          t1 = (int)(t0 + ft < T ? t0 + ft : T);
          break;
        }
        rem -= tiles;
      }
      item_sh[0] = a;
      item_sh[1] = t0;
      item_sh[2] = t1;
    }
    __syncthreads();
    const int a = item_sh[0], t0 = item_sh[1], t1 = item_sh[2];
    __syncthreads();                                   // read before thread 0 takes the next item
    if (a < 0) break;                                  // the same for every thread of the block
    const BatchArray& d = arrays[a];
    const int NH = d.N / 2;
    if (a != cur) {
      pair_core::stage_tables<KB, TT>(lds_all, NH, d.P,
                                      reinterpret_cast<const uint32_t*>(image + d.img_off + d.tab_prow16),
                                      reinterpret_cast<const float*>(image + d.img_off + d.tab_gexp),
                                      image + d.img_off + d.tab_pairs, 64 * kWaves);
      __syncthreads();
      cur = a;
    }
    uint32_t* slab = lds_all + pair_core::head_words(4 * KB, NH, TT, d.P) + wave * slab_words;
    pair_core::run_frames<S, KB, TT, false>(lds_all, slab,
                                            reinterpret_cast<const typename S::T*>(spec_base + d.spec_off), d.M,
                                            d.P, NH, d.I, d.lag0, (int64_t)t0 + wave, t1, kWaves,
                                            tdoa_base + d.tdoa_off, nullptr);
    __syncthreads();                                   // every wave is done before the tables change
  }
}

int num_cus() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  return cus;
}

size_t stft_lds_for(int N) {
  switch (N) {
    case 16: return sizeof(float2) * stft_core::StftShape<16>::lds_float2;
    case 32: return sizeof(float2) * stft_core::StftShape<32>::lds_float2;
    case 64: return sizeof(float2) * stft_core::StftShape<64>::lds_float2;
    case 128: return sizeof(float2) * stft_core::StftShape<128>::lds_float2;
    case 256: return sizeof(float2) * stft_core::StftShape<256>::lds_float2;
    case 512: return sizeof(float2) * stft_core::StftShape<512>::lds_float2;
    case 1024: return sizeof(float2) * stft_core::StftShape<1024>::lds_float2;
    case 2048: return sizeof(float2) * stft_core::StftShape<2048>::lds_float2;
  }
  return 0;
}

template <class S, int KB, int TT, int WV>
hipError_t launch_pair_class(const BatchRun& r, const BatchClass& c, int ft, int blocks_per_cu) {
  if (ft < 1 || blocks_per_cu < 1) return hipErrorInvalidValue;
  auto k = batch_pair_kernel<S, KB, TT, WV>;
  const size_t lds = sizeof(uint32_t) * (size_t(c.head_words_max) + size_t(WV) * c.slab_words_max);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t items = c.items(ft);
  int64_t blocks = (int64_t)num_cus() * blocks_per_cu * (4 / WV);
  if (blocks > items) blocks = items;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * WV), lds, r.stream, r.arrays, r.members + c.member_first,
                     c.member_count, ft, r.image, r.spec, r.tdoa, r.queue + 1 + c.index, c.slab_words_max);
  return hipGetLastError();
}

template <class S, int KB, int TT>
hipError_t launch_pair_waves(const BatchRun& r, const BatchClass& c, const PairTuning& t) {
  // four wavefronts per workgroup when their slabs fit in LDS, else two
  const size_t lds4 = sizeof(uint32_t) * (size_t(c.head_words_max) + 4 * size_t(c.slab_words_max));
  if (t.waves == 4 && lds4 <= 160 * 1024) return launch_pair_class<S, KB, TT, 4>(r, c, t.ft, t.blocks_per_cu);
  return launch_pair_class<S, KB, TT, 2>(r, c, t.ft, t.blocks_per_cu);
}

template <class S, int KB>
hipError_t launch_pair_tt(const BatchRun& r, const BatchClass& c, const PairTuning& t) {
  switch (c.tt) {
    case 1: return launch_pair_waves<S, KB, 1>(r, c, t);
    case 2: return launch_pair_waves<S, KB, 2>(r, c, t);
    case 3: return launch_pair_waves<S, KB, 3>(r, c, t);
  }
  return hipErrorInvalidValue;
}

template <class S>
hipError_t launch_pair_kb(const BatchRun& r, const BatchClass& c, const PairTuning& t) {
  switch (c.kb) {
    case 1: return launch_pair_tt<S, 1>(r, c, t);
    case 2: return launch_pair_tt<S, 2>(r, c, t);
    case 3: return launch_pair_tt<S, 3>(r, c, t);
    case 4: return launch_pair_tt<S, 4>(r, c, t);
    case 6: return launch_pair_tt<S, 6>(r, c, t);
    case 8: return launch_pair_tt<S, 8>(r, c, t);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int batch_head_words(int Dpad, int NH, int TT, int P) { return pair_core::head_words(Dpad, NH, TT, P); }
int batch_slab_words(int N, int I) {
  const int spec_words = 16 * (N / 2 + 4);
  const int y_words = (I + 1) * pair_core::kYStride;
  return spec_words > y_words ? spec_words : y_words;
}

int stft_transforms_per_block(int N) {
  switch (N) {
    case 16: return stft_core::StftShape<16>::FPB;
    case 32: return stft_core::StftShape<32>::FPB;
    case 64: return stft_core::StftShape<64>::FPB;
    case 128: return stft_core::StftShape<128>::FPB;
    case 256: return stft_core::StftShape<256>::FPB;
    case 512: return stft_core::StftShape<512>::FPB;
    case 1024: return stft_core::StftShape<1024>::FPB;
    case 2048: return stft_core::StftShape<2048>::FPB;
  }
  return 0;
}

int64_t BatchClass::items(int ft) const {
  int64_t n = 0;
  for (int64_t T : member_frames) n += (T + ft - 1) / ft;
  return n;
}

hipError_t launch_batch_stft(const BatchRun& r, const StftTuning& t) {
  if (r.stft_items == 0) return hipSuccess;
  if (t.chunk < 1 || t.blocks_per_cu < 1) return hipErrorInvalidValue;
  size_t lds = 0;
  for (int N : r.sizes) lds = stft_lds_for(N) > lds ? stft_lds_for(N) : lds;
  auto k = r.precision == FCC_BF16 ? batch_stft_kernel<SpecBF16> : batch_stft_kernel<SpecF16>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t chunks = (r.stft_items + t.chunk - 1) / t.chunk;
  int64_t blocks = (int64_t)num_cus() * t.blocks_per_cu;
  if (blocks > chunks) blocks = chunks;
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(stft_core::kThreads), lds, r.stream, r.arrays, r.n_arrays,
                     r.stft_items, t.chunk, r.image, r.audio, r.spec, r.queue);
  return hipGetLastError();
}

hipError_t launch_batch_pair(const BatchRun& r, const BatchClass& c, const PairTuning& t) {
  if (r.precision == FCC_BF16) return launch_pair_kb<SpecBF16>(r, c, t);
  if (r.precision == FCC_FP16) return launch_pair_kb<SpecF16>(r, c, t);
  return hipErrorInvalidValue;
}

}  // namespace fcc
