// Many independent arrays of uneven microphone count, aperture, sample rate,
// frame size and rank in one pass.  Every array keeps its own plan tables
// (its slice of the batch image) and its own spectra and outputs:
//   - front end: one launch per frame size present, one workgroup per block
//     of transforms (microphone-frames) of one array; the items of a size are
//     numbered consecutively and a host-built table maps each to its array;
//   - pair stage: one persistent launch per class of arrays that share the
//     matrix-core tile shape (components in blocks of four, lags in tiles of
//     16); each workgroup takes one contiguous run of the class's frames,
//     split by an estimated per-frame cost, and stages an array's tables
//     where its run enters that array.
// Nothing is counted at run time, so the whole sequence can be captured in
// one graph.
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
  __shared__ float2 tw[Sh::TW];
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

// Pair stage of one class: workgroup b takes the frames whose start lies in
// [W b / B, W (b + 1) / B) of the class's cost scale, where member c's frames
// weigh w_c each and start at wprefix[c] (W = wprefix[n]).  The runs are
// contiguous, so a workgroup stages an array's tables only where its run
// crosses into the next array and its wavefronts keep their next-frame
// prefetch going across the run, as in the single-array kernel.
template <class S, int KB, int TT, int kWaves>
__global__ __launch_bounds__(64 * kWaves, 2) void batch_pair_kernel(
    const BatchArray* __restrict__ arrays, const int32_t* __restrict__ members, int n_members,
    const int64_t* __restrict__ wprefix, const unsigned char* __restrict__ image,
    const unsigned char* __restrict__ spec_base, int32_t* __restrict__ tdoa_base, int slab_words) {
  extern __shared__ uint32_t lds_all[];
  __shared__ long long run_sh[3];
  const int wave = threadIdx.x >> 6;
  // thread 0 alone walks the runs: the member it is at and the cost range
  int c = 0;
  int64_t w0 = 0, w1 = 0;
  if (threadIdx.x == 0) {
    const int64_t W = wprefix[n_members];
    w0 = W * (int64_t)blockIdx.x / gridDim.x;
    w1 = W * ((int64_t)blockIdx.x + 1) / gridDim.x;
    int lo = 0, hi = n_members - 1;               // last member starting at or before w0
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (wprefix[mid] <= w0) lo = mid;
      else hi = mid - 1;
    }
    c = lo;
  }
  for (;;) {
    if (threadIdx.x == 0) {
      long long a = -1, tb = 0, te = 0;
      for (; c < n_members && wprefix[c] < w1; ++c) {
        const int m = members[c];
        const int64_t T = arrays[m].T;
        if (T <= 0) continue;
        const int64_t pre = wprefix[c], w = (wprefix[c + 1] - pre) / T;
        // frame t starts at pre + t w; this run keeps the starts in [w0, w1)
        const int64_t b0 = w0 > pre ? (w0 - pre + w - 1) / w : 0;
        int64_t b1 = (w1 - pre + w - 1) / w;
        if (b1 > T) b1 = T;
        if (b0 < b1) {
          a = m;
          tb = b0;
          te = b1;
          ++c;
          break;
        }
      }
      run_sh[0] = a;
      run_sh[1] = tb;
      run_sh[2] = te;
    }
    __syncthreads();
    const int a = (int)run_sh[0];
    const int64_t tb = run_sh[1], te = run_sh[2];
    __syncthreads();                                   // read before thread 0 writes the next run
    if (a < 0) break;                                  // the same for every thread of the block
    const BatchArray& d = arrays[a];
    const int NH = d.N / 2;
    pair_core::stage_tables<KB, TT>(lds_all, NH, d.P, d.I,
                                    reinterpret_cast<const uint32_t*>(image + d.img_off + d.tab_prow16),
                                    reinterpret_cast<const float*>(image + d.img_off + d.tab_gexp),
                                    image + d.img_off + d.tab_pairs, 64 * kWaves);
    __syncthreads();
    uint32_t* slab = lds_all + pair_core::head_words(4 * KB, NH, TT, d.P) + wave * slab_words;
    pair_core::run_frames<S, KB, TT, false>(lds_all, slab,
                                            reinterpret_cast<const typename S::T*>(spec_base + d.spec_off), d.M,
                                            d.P, NH, d.I, d.lag0, tb + wave, te, kWaves,
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
hipError_t launch_pair_class(const BatchRun& r, const BatchClass& c, int blocks_per_cu) {
  if (blocks_per_cu < 1) return hipErrorInvalidValue;
  auto k = batch_pair_kernel<S, KB, TT, WV>;
  const size_t lds = sizeof(uint32_t) * (size_t(c.head_words_max) + size_t(WV) * c.slab_words_max);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t blocks = c.workgroups(num_cus(), blocks_per_cu, WV);
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * WV), lds, r.stream, r.arrays, r.members + c.member_first,
                     c.member_count, reinterpret_cast<const int64_t*>(r.image + c.wprefix_off), r.image, r.spec,
                     r.tdoa, c.slab_words_max);
  return hipGetLastError();
}

template <class S, int KB, int TT>
hipError_t launch_pair_waves(const BatchRun& r, const BatchClass& c, const PairTuning& t) {
  switch (batch_pair_waves(c, t)) {
    case 4: return launch_pair_class<S, KB, TT, 4>(r, c, t.blocks_per_cu);
    case 3: return launch_pair_class<S, KB, TT, 3>(r, c, t.blocks_per_cu);
    default: return launch_pair_class<S, KB, TT, 2>(r, c, t.blocks_per_cu);
  }
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
  const int y_words = pair_core::lag_words(I, I <= 16 ? 1 : (I <= 32 ? 2 : 3));
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

// the wavefronts per workgroup asked for (2, 3 or 4), fewer where their slabs do not fit in LDS
int batch_pair_waves(const BatchClass& c, const PairTuning& t) {
  for (int w = t.waves < 4 ? t.waves : 4; w > 2; --w)
    if (sizeof(uint32_t) * (size_t(c.head_words_max) + size_t(w) * c.slab_words_max) <= 160 * 1024) return w;
  return 2;
}

int64_t batch_pair_workgroups(const BatchClass& c, const PairTuning& t) {
  return c.workgroups(num_cus(), t.blocks_per_cu, batch_pair_waves(c, t));
}

// workgroups of one class launch: persistent, at most one per frame
int64_t BatchClass::workgroups(int cus, int blocks_per_cu, int waves) const {
  int64_t frames = 0;
  for (int64_t T : member_frames) frames += T;
  int64_t blocks = int64_t(cus) * blocks_per_cu * (waves == 2 ? 2 : 1);
  return blocks < frames ? blocks : frames;
}

// cost of one frame on the class's cost scale: K steps of the projection plus
// a fixed share for staging, expansion and the argmax
int64_t pair_frame_weight(int N) { return N / 32 + 4; }

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
