// Direction-of-arrival search over all pairs of an array: the step the paper
// names after TDoA estimation (Sec. 6), done as the steered response of the
// pairwise correlations.  For direction g and pair p the host table holds
// q[p][g], the fractional index on the lag grid of the TDoA that a far-field
// source from g produces; the score of g is the sum over pairs of y_p read at
// q[p][g] with linear interpolation, and the DoA is the first direction of
// largest score.
//
// One workgroup takes FB consecutive frames: their correlations [P][I] are
// staged in LDS, each lane walks directions g = lane, lane + 256, ...
// accumulating the FB scores of its direction (one table read serves FB
// frames), and a (value, index) reduction over the workgroup gives each
// frame's first best direction.
#include "device_common.hpp"
#include "kernels.hpp"

namespace fcc {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr size_t kLdsBudget = 48 * 1024;

__device__ __forceinline__ void better(float& v, int& i, float ov, int oi) {
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}

template <int FB>
__global__ __launch_bounds__(kThreads) void doa_kernel(const float* __restrict__ y, int64_t T, int P, int I,
                                                       const float* __restrict__ q, int G, int32_t* __restrict__ doa,
                                                       float* __restrict__ score) {
  extern __shared__ float ys[];                    // [FB][P * I]
  __shared__ float red_v[FB][kWaves];
  __shared__ int red_i[FB][kWaves];
  const int PI = P * I;
  const int64_t t0 = (int64_t)blockIdx.x * FB;
  const int nf = T - t0 < FB ? (int)(T - t0) : FB;
  for (int e = threadIdx.x; e < FB * PI; e += kThreads) ys[e] = e < nf * PI ? y[t0 * PI + e] : 0.f;
  __syncthreads();

  float best[FB];
  int bidx[FB];
#pragma unroll
  for (int f = 0; f < FB; ++f) {
    best[f] = -3.402823466e38f;
    bidx[f] = G;
  }
  for (int g = threadIdx.x; g < G; g += kThreads) {
    float s[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f) s[f] = 0.f;
    for (int p = 0; p < P; ++p) {
      const float qq = q[(int64_t)p * G + g];
      int i0 = (int)qq;
      i0 = i0 < I - 2 ? i0 : (I >= 2 ? I - 2 : 0);
      const int i1 = i0 + 1 < I ? i0 + 1 : i0;
      const float w = qq - (float)i0;
      const float* yr = ys + p * I;
#pragma unroll
      for (int f = 0; f < FB; ++f) {
        const float y0 = yr[f * PI + i0], y1 = yr[f * PI + i1];
        s[f] += y0 + w * (y1 - y0);
      }
    }
#pragma unroll
    for (int f = 0; f < FB; ++f) {
      if (f < nf) {
        if (score) score[(t0 + f) * G + g] = s[f];
        if (s[f] > best[f]) {              // g ascends per lane: strict > keeps the first
          best[f] = s[f];
          bidx[f] = g;
        }
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int f = 0; f < FB; ++f) {
    float v = best[f];
    int i = bidx[f];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) better(v, i, __shfl_xor(v, off), __shfl_xor(i, off));
    if (lane == 0) {
      red_v[f][wave] = v;
      red_i[f][wave] = i;
    }
  }
  __syncthreads();
  if (threadIdx.x < nf) {
    const int f = threadIdx.x;
    float v = red_v[f][0];
    int i = red_i[f][0];
    for (int w = 1; w < kWaves; ++w) better(v, i, red_v[f][w], red_i[f][w]);
    doa[t0 + f] = i;
  }
}

template <int FB>
hipError_t launch_fb(const DoaArgs& a) {
  const size_t lds = sizeof(float) * size_t(FB) * a.P * a.I;
  const unsigned blocks = (unsigned)((a.T + FB - 1) / FB);
  hipLaunchKernelGGL(doa_kernel<FB>, dim3(blocks), dim3(kThreads), lds, a.stream, a.y, a.T, a.P, a.I, a.table,
                     a.G, a.doa, a.score);
  return hipGetLastError();
}

}  // namespace

bool doa_supported(const DoaArgs& a) {
  return a.G >= 1 && a.P >= 1 && a.I >= 1 && sizeof(float) * size_t(a.P) * a.I <= kLdsBudget;
}

hipError_t launch_doa(const DoaArgs& a) {
  if (a.T == 0) return hipSuccess;
  if (!doa_supported(a)) return hipErrorInvalidValue;
  const size_t per = sizeof(float) * size_t(a.P) * a.I;     // one frame's correlations
  if (8 * per <= kLdsBudget) return launch_fb<8>(a);
  if (4 * per <= kLdsBudget) return launch_fb<4>(a);
  if (2 * per <= kLdsBudget) return launch_fb<2>(a);
  return launch_fb<1>(a);
}

}  // namespace fcc
