// Front end of the TDoA path (Sec. 2): framing, periodic Hann window, real
// DFT of every frame of every microphone, and per-microphone PHAT.
//
// At alpha = 1 the PHAT of a pair's cross-spectrum factorises,
//   R_ij / |R_ij| = (X_i / |X_i|) (X_j / |X_j|)^*,
// so each bin is normalised once per microphone here instead of once per pair.
//
// The N real samples of a frame are packed as N/2 complex values
// z[n] = w[2n] x[2n] + j w[2n+1] x[2n+1] and transformed by a mixed-radix
// Stockham FFT: radix-16 butterflies held in registers, one LDS exchange per
// pass (two passes for N = 512), in a buffer padded by one slot every 16.  A
// transform uses N/32 lanes (one for N <= 32);
// a 256-thread block runs 256 / lanes transforms over consecutive
// (frame, microphone) pairs, so for M = 16 and N = 512 a block is one frame.
// The split Z -> X(f) = E(f) + W^f O(f) of the real transform follows, then the
// normalisation.  Twiddles (and the window, through its cosine) come from a
// full-circle FP64-computed table staged in LDS.
//
// With recursive smoothing (alpha < 1) the PHAT belongs to each pair's
// smoothed cross-spectrum, so the raw spectra X are written instead (FP32).
//
// Output layout ("packed real spectrum"): N/2 complex slots per microphone;
// slot 0 holds (e(0), e(N/2)), both real, slot f holds e(f) for 0 < f < N/2.
#include "stft_core.hpp"
#include "kernels.hpp"

namespace fcc {
namespace {

using namespace stft_core;

constexpr unsigned kXcds = 8;       // accelerator complex dies of an MI355X

template <int N, class S, bool RAW>
__global__ __launch_bounds__(kThreads) void stft_phat_kernel(
    const float* __restrict__ x, int64_t ld, int M, int hop, int64_t nfft,
    const float2* __restrict__ twiddle, typename S::T* __restrict__ out) {
  using Sh = StftShape<N>;
  __shared__ float2 tw[Sh::TW];
  __shared__ float2 tw1[Sh::T1];
  __shared__ float2 tw2[Sh::T2];
  __shared__ float2 data[Sh::FPB * Sh::NHP];

  // Persistent workgroups, dealt to the 8 XCDs round-robin: XCD x walks the
  // x-th contiguous run of the logical blocks (FPB transforms each), its
  // workgroups side by side, so the 4x overlap of neighbouring frames is
  // served from that XCD's L2 instead of HBM.  Each lane holds the next
  // block's samples in registers while the current block is transformed.
  const int64_t nblk = (nfft + Sh::FPB - 1) / Sh::FPB;
  const unsigned grid = gridDim.x;
  const unsigned xcd = blockIdx.x % kXcds, local = blockIdx.x / kXcds;
  const unsigned nx = grid / kXcds + (xcd < grid % kXcds ? 1u : 0u);    // workgroups on this XCD
  const int64_t per = nblk / kXcds, extra = nblk % kXcds;
  const int64_t begin = xcd * per + (xcd < extra ? xcd : extra);
  const int64_t end = begin + per + (xcd < extra ? 1 : 0);
  load_tables<N>(tw, tw1, tw2, twiddle);
  __syncthreads();
  const int slot = threadIdx.x / Sh::LF, lf = threadIdx.x % Sh::LF;
  // where a block holds whole frames (M divides its transforms), a lane keeps
  // its microphone and frame offset, and a block's first frame is uniform
  const bool whole = Sh::FPB % M == 0;
  const int fpb = whole ? Sh::FPB / M : 0;
  const int mic_in = whole ? slot % M : 0, t_in = whole ? slot / M : 0;
  const float* lane_x = x + (int64_t)mic_in * ld + (int64_t)t_in * hop;
  float2 u[Sh::RD::R0], nxt[Sh::RD::R0];
  auto fetch = [&](int64_t blk) {
    const uint64_t b = (uint64_t)blk * Sh::FPB + slot;
    if (b >= (uint64_t)nfft) return;
    if (whole) load_samples_at<N>(nxt, lane_x + blk * fpb * hop, lf);
    else load_samples<N>(nxt, x, ld, M, hop, (uint32_t)b, lf);
  };
  int64_t lblk = begin + local;
  if (lblk < end) fetch(lblk);
  for (; lblk < end; lblk += nx) {
#pragma unroll
    for (int r = 0; r < Sh::RD::R0; ++r) u[r] = nxt[r];
    const int64_t next = lblk + nx;
    transform_samples<N, S, RAW>(tw, tw1, tw2, data, u, nfft, out, lblk, [&] {
      if (next < end) fetch(next);
    });
    exchange_sync<true>();   // the next block's first pass rewrites this wavefront's scratch
  }
}

template <int N, class S, bool RAW>
hipError_t launch_n(const StftArgs& a) {
  constexpr int FPB = StftShape<N>::FPB;
  const int64_t nfft = a.T * a.M;
  const int64_t blocks = (nfft + FPB - 1) / FPB;
  // persistent grid: as many workgroups as the CUs hold at once (registers
  // and LDS decide), each walking its XCD's run of blocks
  int dev = 0, cus = 256, per_cu = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stft_phat_kernel<N, S, RAW>, kThreads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int64_t cap = int64_t(per_cu) * cus;
  const int64_t grid = blocks < cap ? blocks : cap;
  hipLaunchKernelGGL((stft_phat_kernel<N, S, RAW>), dim3((unsigned)grid), dim3(kThreads), 0, a.stream,
                     a.x, a.ld, a.M, a.hop, nfft, a.twiddle, static_cast<typename S::T*>(a.out));
  return hipGetLastError();
}

template <class S, bool RAW = false>
hipError_t launch_s(const StftArgs& a) {
  switch (a.N) {
    case 16: return launch_n<16, S, RAW>(a);
    case 32: return launch_n<32, S, RAW>(a);
    case 64: return launch_n<64, S, RAW>(a);
    case 128: return launch_n<128, S, RAW>(a);
    case 256: return launch_n<256, S, RAW>(a);
    case 512: return launch_n<512, S, RAW>(a);
    case 1024: return launch_n<1024, S, RAW>(a);
    case 2048: return launch_n<2048, S, RAW>(a);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_stft_phat(const StftArgs& a) {
  if (a.T == 0) return hipSuccess;
  if (a.raw) return a.precision == FCC_FP32 ? launch_s<SpecF32, true>(a) : hipErrorInvalidValue;
  switch (a.precision) {
    case FCC_FP32: return launch_s<SpecF32>(a);
    case FCC_BF16: return launch_s<SpecBF16>(a);
    case FCC_FP16: return launch_s<SpecF16>(a);
    case FCC_FP8_E4M3: return launch_s<SpecE4M3>(a);
  }
  return hipErrorInvalidValue;
}

}  // namespace fcc
