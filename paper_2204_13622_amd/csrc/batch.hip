// Many independent arrays of uneven microphone count, aperture, sample rate,
// frame size and rank in one pass.  Every array keeps its own plan tables
// (its slice of the batch image) and its own spectra and outputs:
//   - front end: one launch per frame size present, one workgroup per block
//     of transforms (microphone-frames) of one array; the items of a size are
//     numbered consecutively and a host-built table maps each to its array;
//   - pair stage: one persistent launch per class of arrays that share the
//     matrix-core tile shape (components in blocks of four, lags in tiles of
//     16); an item is a tile of consecutive frames of one array, taken from
//     an atomic queue; each workgroup stages the class's item prefix in LDS
//     once, and the array's tables when the array changes.
// The queues are counters in the workspace, cleared by a fill kernel, so the
// whole sequence can be captured in one graph.
#include "kernels.hpp"
#include "pair_mfma_core.hpp"
#include "stft_core.hpp"

namespace fcc {
namespace {

// Front end, one launch per frame size: one workgroup per block of
// transforms, exactly as the single-array kernel (tables staged per
// workgroup, XCD-contiguous order so a frame's 4x overlap with its neighbours
// is served by one L2); the item's array comes from a table built on the host.
template <int N, class S>
__global__ __launch_bounds__(stft_core::kThreads) void batch_stft_kernel(
    const BatchArray* __restrict__ arrays, const int32_t* __restrict__ item_array, int64_t first_item,
    const unsigned char* __restrict__ image, const float* __restrict__ audio, unsigned char* __restrict__ spec_base) {
  using Sh = stft_core::StftShape<N>;
  __shared__ float2 tw[N];
  __shared__ float2 tw1[Sh::T1];
  __shared__ float2 tw2[Sh::T2];
  __shared__ float2 data[Sh::FPB * Sh::NHP];
  constexpr unsigned kXcds = 8;
  const unsigned nblk = gridDim.x;
  const unsigned xcd = blockIdx.x % kXcds, local = blockIdx.x / kXcds;
  const unsigned per = nblk / kXcds, extra = nblk % kXcds;
  const int64_t it = first_item + (int64_t)(xcd * per + (xcd < extra ? xcd : extra) + local);
  const BatchArray& d = arrays[item_array[it]];
  stft_core::load_tables<N>(tw, tw1, tw2, reinterpret_cast<const float2*>(image + d.img_off + d.tab_twiddle));
  __syncthreads();
  stft_core::transforms<N, S, false>(tw, tw1, tw2, data, audio + d.audio_off, d.L, d.M, d.hop, d.T * d.M,
                                     reinterpret_cast<typename S::T*>(spec_base + d.spec_off), it - d.stft_first);
}

// Tiles of ft frames of member c start at item first[c]; first[n] is the
// class's item count.  Computed once per workgroup by wavefront 0: each lane
// sums a run of members, a 64-lane scan gives the runs' offsets.
__device__ __forceinline__ void tile_prefix(const BatchArray* __restrict__ arrays, const int32_t* __restrict__ members,
                                            int n, int ft, int* __restrict__ first) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x, run = (n + 63) / 64, c0 = lane * run, c1 = c0 + run < n ? c0 + run : n;
  int sum = 0;
  for (int c = c0; c < c1; ++c) sum += (int)((arrays[members[c]].T + ft - 1) / ft);
  int incl = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  int at = incl - sum;                           // items before this lane's run
  for (int c = c0; c < c1; ++c) {
    first[c] = at;
    at += (int)((arrays[members[c]].T + ft - 1) / ft);
  }
  if (lane == 63) first[n] = incl;
}

template <class S, int KB, int TT, int kWaves>
__global__ __launch_bounds__(64 * kWaves, 2) void batch_pair_kernel(
    const BatchArray* __restrict__ arrays, const int32_t* __restrict__ members, int n_members, int ft,
    const unsigned char* __restrict__ image, const unsigned char* __restrict__ spec_base,
    int32_t* __restrict__ tdoa_base, int* __restrict__ queue, int slab_words, int prefix_off) {
  extern __shared__ uint32_t lds_all[];
  __shared__ int item_sh[3];
  const int wave = threadIdx.x >> 6;
  // the item prefix lives past the largest table head and the slabs; prefix_off < 0: the class is
  // too large to stage it and thread 0 walks the member list instead
  const bool staged = prefix_off >= 0;
  int* first = reinterpret_cast<int*>(lds_all + (staged ? prefix_off : 0));
  if (staged) {
    tile_prefix(arrays, members, n_members, ft, first);
    __syncthreads();
  }
  int cur = -1;
  for (;;) {
    if (threadIdx.x == 0) {
      int rem = atomicAdd(queue, 1), a = -1, t0 = 0, t1 = 0;
      if (staged) {
        // item -> member: last c with first[c] <= rem
        if (rem < first[n_members]) {
          int lo = 0, hi = n_members - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (first[mid] <= rem) lo = mid;
            else hi = mid - 1;
          }
          a = members[lo];
          const int64_t T = arrays[a].T;
          t0 = (rem - first[lo]) * ft;
          t1 = (int)(t0 + ft < T ? t0 + ft : T);
        }
      } else {
        // walk the class's arrays
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

template <class S, int KB, int TT, int WV>
hipError_t launch_pair_class(const BatchRun& r, const BatchClass& c, int ft, int blocks_per_cu) {
  if (ft < 1 || blocks_per_cu < 1) return hipErrorInvalidValue;
  auto k = batch_pair_kernel<S, KB, TT, WV>;
  const size_t base_words = size_t(c.head_words_max) + size_t(WV) * c.slab_words_max;
  if (sizeof(uint32_t) * base_words > 160 * 1024) return hipErrorInvalidValue;
  // stage the class's item prefix when it fits beside the tables and slabs
  const size_t prefix_words = size_t(c.member_count) + 1;
  const bool staged = sizeof(uint32_t) * (base_words + prefix_words) <= 160 * 1024;
  const size_t lds = sizeof(uint32_t) * (base_words + (staged ? prefix_words : 0));
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
                     c.member_count, ft, r.image, r.spec, r.tdoa, r.queue + 1 + c.index, c.slab_words_max,
                     staged ? int(base_words) : -1);
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

namespace {

template <int N, class S>
hipError_t launch_stft_range(const BatchRun& r, int64_t first, int64_t count) {
  hipLaunchKernelGGL((batch_stft_kernel<N, S>), dim3((unsigned)count), dim3(stft_core::kThreads), 0, r.stream,
                     r.arrays, r.item_array, first, r.image, r.audio, r.spec);
  return hipGetLastError();
}

template <class S>
hipError_t launch_stft_size(const BatchRun& r, int N, int64_t first, int64_t count) {
  switch (N) {
    case 16: return launch_stft_range<16, S>(r, first, count);
    case 32: return launch_stft_range<32, S>(r, first, count);
    case 64: return launch_stft_range<64, S>(r, first, count);
    case 128: return launch_stft_range<128, S>(r, first, count);
    case 256: return launch_stft_range<256, S>(r, first, count);
    case 512: return launch_stft_range<512, S>(r, first, count);
    case 1024: return launch_stft_range<1024, S>(r, first, count);
    case 2048: return launch_stft_range<2048, S>(r, first, count);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_batch_stft(const BatchRun& r) {
  for (const BatchStftRange& g : r.stft_ranges) {
    if (g.count <= 0) continue;
    if (g.count > 0x7fffffff) return hipErrorInvalidValue;
    const hipError_t e = r.precision == FCC_BF16 ? launch_stft_size<SpecBF16>(r, g.N, g.first, g.count)
                                                 : launch_stft_size<SpecF16>(r, g.N, g.first, g.count);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_batch_pair(const BatchRun& r, const BatchClass& c, const PairTuning& t) {
  if (r.precision == FCC_BF16) return launch_pair_kb<SpecBF16>(r, c, t);
  if (r.precision == FCC_FP16) return launch_pair_kb<SpecF16>(r, c, t);
  return hipErrorInvalidValue;
}

}  // namespace fcc
