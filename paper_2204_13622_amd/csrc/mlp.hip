// Learned sub-sample TDoA: a small multilayer perceptron on the projection
// coefficients of eq. (9), with hand-written FP16 training and inference.
//
// Model (one row = one pair-frame):
//   u = c / ||c||_2                       c = (a_1, b_1, ..., a_D, b_D)
//   h1 = gelu(u W1 + b1),  h2 = gelu(h1 W2 + b2),  (mu, s) = h2 W3 + b3
// mu is the TDoA in samples; s, clipped to [-8, 8], the log-variance of a
// Gaussian error model, trained by the mean negative log-likelihood
//   L = (1/R) sum_r 0.5 (exp(-s_r) (mu_r - delta_r)^2 + s_r).
// gelu is the tanh form of Hendrycks and Gimpel (2016).
//
// Every matrix product runs on 16x16x32 FP16 MFMA tiles with FP32
// accumulation (operands are rounded to FP16 when staged in LDS); bias,
// activation, loss and the optimiser are FP32.  Backward products carry
// per-row derivatives of order one and the 1/R batch mean is applied in the
// FP32 epilogue, so small gradients do not underflow FP16.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace fcc {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr float kSClip = 8.f;
constexpr float kGeluC = 0.7978845608028654f;   // sqrt(2 / pi)
constexpr float kGeluA = 0.044715f;

__device__ __forceinline__ float gelu(float x) {
  return 0.5f * x * (1.f + tanhf(kGeluC * (x + kGeluA * x * x * x)));
}
__device__ __forceinline__ float gelu_grad(float x) {
  const float t = tanhf(kGeluC * (x + kGeluA * x * x * x));
  return 0.5f * (1.f + t) + 0.5f * x * (1.f - t * t) * kGeluC * (1.f + 3.f * kGeluA * x * x);
}

constexpr int kTile = 64, kKStep = 32, kLdsRow = kKStep + 8;   // halves per LDS row (pad: banks)

enum { kEpiStore = 0, kEpiBiasGelu = 1, kEpiBias = 2 };

// C[M x N] = alpha * op(A) op(B) (+ bias; + gelu into H).  op(A)(m, k) is
// A[k * lda + m] when TA, else A[m * lda + k]; op(B)(k, n) is B[n * ldb + k]
// when TB, else B[k * ldb + n].  One 64 x 64 output tile per 256-thread block.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void gemm_f16_kernel(const float* __restrict__ A, int lda,
                                                       const float* __restrict__ B, int ldb,
                                                       float* __restrict__ C, int ldc, int M, int N, int K,
                                                       float alpha, const float* __restrict__ bias,
                                                       float* __restrict__ H) {
  __shared__ __attribute__((aligned(16))) _Float16 As[kTile * kLdsRow];   // [m][k]
  __shared__ __attribute__((aligned(16))) _Float16 Bs[kTile * kLdsRow];   // [n][k]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, col = lane & 15;
  const int m0 = blockIdx.x * kTile, n0 = blockIdx.y * kTile;   // rows on x: no 65535 cap
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < K; k0 += kKStep) {
    for (int e = tid; e < kTile * kKStep; e += 256) {
      // walk the contiguous direction of each operand in memory
      int m, k;
      if (TA) { m = e % kTile; k = e / kTile; } else { k = e % kKStep; m = e / kKStep; }
      const int gm = m0 + m, gk = k0 + k;
      float v = 0.f;
      if (gm < M && gk < K) v = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
      As[m * kLdsRow + k] = (_Float16)v;
      int n;
      if (TB) { k = e % kKStep; n = e / kKStep; } else { n = e % kTile; k = e / kTile; }
      const int gn = n0 + n, gk2 = k0 + k;
      float w = 0.f;
      if (gn < N && gk2 < K) w = TB ? B[(size_t)gn * ldb + gk2] : B[(size_t)gk2 * ldb + gn];
      Bs[n * kLdsRow + k] = (_Float16)w;
    }
    __syncthreads();
    h8 a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = *reinterpret_cast<const h8*>(&As[(wm + 16 * t + col) * kLdsRow + 8 * g]);
      b[t] = *reinterpret_cast<const h8*>(&Bs[(wn + 16 * t + col) * kLdsRow + 8 * g]);
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = m0 + wm + 16 * mt + 4 * g + q, c = n0 + wn + 16 * nt + col;
        if (r < M && c < N) {
          float v = alpha * acc[mt][nt][q];
          if (EPI != kEpiStore) v += bias[c];
          C[(size_t)r * ldc + c] = v;
          if (EPI == kEpiBiasGelu) H[(size_t)r * ldc + c] = gelu(v);
        }
      }
}

template <bool TA, bool TB, int EPI>
hipError_t gemm(const float* A, int lda, const float* B, int ldb, float* C, int ldc, int M, int N, int K,
                float alpha, const float* bias, float* H, hipStream_t st) {
  const dim3 grid((M + kTile - 1) / kTile, (N + kTile - 1) / kTile);
  hipLaunchKernelGGL((gemm_f16_kernel<TA, TB, EPI>), grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K,
                     alpha, bias, H);
  return hipGetLastError();
}

__global__ void features_kernel(const float* __restrict__ c, float* __restrict__ u, int64_t R, int K) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  float n2 = 0.f;
  for (int k = 0; k < K; ++k) n2 += c[r * K + k] * c[r * K + k];
  const float s = n2 > 0.f ? rsqrtf(n2) : 0.f;
  for (int k = 0; k < K; ++k) u[r * K + k] = c[r * K + k] * s;
}

// (mu, s) from the raw head output; per-row derivative of the loss (not yet
// divided by R) and the summed loss
__global__ void head_kernel(const float* __restrict__ o, const float* __restrict__ delta,
                            float* __restrict__ out, float* __restrict__ dout, float* __restrict__ loss_sum,
                            int64_t R) {
  __shared__ float red[256];
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (r < R) {
    const float mu = o[2 * r], s_raw = o[2 * r + 1];
    const float s = fminf(fmaxf(s_raw, -kSClip), kSClip);
    out[2 * r] = mu;
    out[2 * r + 1] = s;
    if (delta) {
      const float e = mu - delta[r], w = expf(-s);
      l = 0.5f * (w * e * e + s);
      dout[2 * r] = w * e;
      dout[2 * r + 1] = (s_raw > -kSClip && s_raw < kSClip) ? 0.5f * (1.f - w * e * e) : 0.f;
    }
  }
  if (!delta) return;
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss_sum, red[0]);
}

__global__ void gelu_backward_kernel(float* __restrict__ dh, const float* __restrict__ z, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dh[i] *= gelu_grad(z[i]);
}

// out[n] = alpha * sum_r x[r][n]; one block per column, fixed summation order
__global__ void colsum_kernel(const float* __restrict__ x, int64_t R, int N, float alpha, float* __restrict__ out) {
  __shared__ float red[256];
  const int n = blockIdx.x;
  float s = 0.f;
  for (int64_t r = threadIdx.x; r < R; r += 256) s += x[r * N + n];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = alpha * red[0];
}

__global__ void adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// learned estimate where its confidence exp(-s/2) reaches the threshold,
// the fallback (interpolated FCC lag) elsewhere
__global__ void select_kernel(const float* __restrict__ out, const float* __restrict__ fallback, int64_t R,
                              float min_conf, float* __restrict__ tau, float* __restrict__ conf) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const float c = expf(-0.5f * out[2 * r + 1]);
  tau[r] = c >= min_conf ? out[2 * r] : fallback[r];
  if (conf) conf[r] = c;
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

struct Layout {
  int K0, H;
  size_t W1, b1, W2, b2, W3, b3, total;
};
__host__ __device__ Layout layout(int K0, int H) {
  Layout L{K0, H, 0, 0, 0, 0, 0, 0, 0};
  size_t o = 0;
  L.W1 = o; o += size_t(K0) * H;
  L.b1 = o; o += H;
  L.W2 = o; o += size_t(H) * H;
  L.b2 = o; o += H;
  L.W3 = o; o += size_t(H) * 2;
  L.b3 = o; o += 2;
  L.total = o;
  return L;
}

struct Work {
  float *U, *Z1, *H1, *Z2, *H2, *O, *dO, *dH2, *dH1;
};
Work carve(void* ws, int64_t R, int K0, int H) {
  float* p = static_cast<float*>(ws);
  Work w;
  w.U = p; p += R * K0;
  w.Z1 = p; p += R * H;
  w.H1 = p; p += R * H;
  w.Z2 = p; p += R * H;
  w.H2 = p; p += R * H;
  w.O = p; p += R * 2;
  w.dO = p; p += R * 2;
  w.dH2 = p; p += R * H;
  w.dH1 = p; p += R * H;
  return w;
}

#define FCC_TRY(x)                        \
  do {                                    \
    hipError_t e_ = (x);                  \
    if (e_ != hipSuccess) return e_;      \
  } while (0)

hipError_t forward_impl(const float* theta, int K0, int H, const float* x, int64_t R, float* out,
                        const float* delta, float* loss_sum, const Work& w, hipStream_t st) {
  const Layout L = layout(K0, H);
  hipLaunchKernelGGL(features_kernel, dim3(blocks_for(R, 256)), dim3(256), 0, st, x, w.U, R, K0);
  FCC_TRY(hipGetLastError());
  FCC_TRY((gemm<false, false, kEpiBiasGelu>(w.U, K0, theta + L.W1, H, w.Z1, H, (int)R, H, K0, 1.f,
                                            theta + L.b1, w.H1, st)));
  FCC_TRY((gemm<false, false, kEpiBiasGelu>(w.H1, H, theta + L.W2, H, w.Z2, H, (int)R, H, H, 1.f,
                                            theta + L.b2, w.H2, st)));
  FCC_TRY((gemm<false, false, kEpiBias>(w.H2, H, theta + L.W3, 2, w.O, 2, (int)R, 2, H, 1.f, theta + L.b3,
                                        nullptr, st)));
  hipLaunchKernelGGL(head_kernel, dim3(blocks_for(R, 256)), dim3(256), 0, st, w.O, delta, out, w.dO,
                     loss_sum, R);
  return hipGetLastError();
}

// ---- fused inference ---------------------------------------------------------
// Every wavefront takes 16 rows at a time through all three layers: the
// normalised coefficients go straight into the A-operand registers of the
// 16x16x32 FP16 MFMA, the layer outputs pass through a per-wavefront FP16
// row buffer in LDS (the C layout of one layer is not the A layout of the
// next), and the two head outputs are dot products on the vector ALU.  The
// weights sit in LDS, transposed ([n][k]) as the B operands want them.  The
// rounding points are those of the layer-by-layer path: operands of every
// product in FP16, accumulation, bias, GELU and head in FP32.

__device__ __forceinline__ float gelu_fast(float x) {
  // (1 + tanh(u)) / 2 = 1 / (1 + exp(-2u)): exact at both tails (exp over- and
  // underflow); the hardware reciprocal (about 1 ulp) stands in for a
  // correctly rounded division, whose result is rounded to FP16 anyway
  const float u = kGeluC * (x + kGeluA * x * x * x);
  return x * __builtin_amdgcn_rcpf(1.f + __expf(-2.f * u));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int K0P, int H>
struct InferLds {
  static constexpr int W1ROW = K0P + 8, W2ROW = H + 8, HROW = H + 8;   // halves; pads spread the banks
  static constexpr size_t bytes(int waves) {
    return sizeof(_Float16) * (size_t(H) * W1ROW + size_t(H) * W2ROW + size_t(waves) * 16 * HROW) +
           sizeof(float) * (3 * size_t(H) + 2 * size_t(H) + 4);
  }
};

// out: (mu, s) per row, or with `fallback` the learned lag where exp(-s/2) >=
// min_conf and the fallback elsewhere into tau, with exp(-s/2) into conf
template <int K0P, int H>
__global__ __launch_bounds__(256) void mlp_infer_kernel(const float* __restrict__ theta, int K0,
                                                        const float* __restrict__ x, int64_t R,
                                                        float* __restrict__ out, const float* __restrict__ fallback,
                                                        float min_conf, float* __restrict__ tau,
                                                        float* __restrict__ conf) {
  using LY = InferLds<K0P, H>;
  constexpr int kWaves = 4;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  _Float16* w1t = reinterpret_cast<_Float16*>(lds_raw);                  // [H][W1ROW]
  _Float16* w2t = w1t + H * LY::W1ROW;                                    // [H][W2ROW]
  _Float16* hb_all = w2t + H * LY::W2ROW;                                 // [waves][16][HROW]
  float* b1 = reinterpret_cast<float*>(hb_all + kWaves * 16 * LY::HROW);  // [H]
  float* b2 = b1 + H;                                                     // [H]
  float* w3 = b2 + H;                                                     // [H][2], FP16-rounded
  float* b3 = w3 + 2 * H;                                                 // [2]
  const Layout L = layout(K0, H);
  for (int e = threadIdx.x; e < H * K0P; e += 256) {
    const int n = e / K0P, k = e % K0P;
    w1t[n * LY::W1ROW + k] = (_Float16)(k < K0 ? theta[L.W1 + (size_t)k * H + n] : 0.f);
  }
  for (int e = threadIdx.x; e < H * H; e += 256) {
    const int n = e / H, k = e % H;
    w2t[n * LY::W2ROW + k] = (_Float16)theta[L.W2 + (size_t)k * H + n];
  }
  for (int e = threadIdx.x; e < H; e += 256) {
    b1[e] = theta[L.b1 + e];
    b2[e] = theta[L.b2 + e];
    w3[2 * e] = (float)(_Float16)theta[L.W3 + 2 * e];
    w3[2 * e + 1] = (float)(_Float16)theta[L.W3 + 2 * e + 1];
  }
  if (threadIdx.x < 2) b3[threadIdx.x] = theta[L.b3 + threadIdx.x];
  __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;
  _Float16* hb = hb_all + wave * 16 * LY::HROW;
  const int64_t groups = (R + 15) / 16;
  for (int64_t grp = (int64_t)blockIdx.x * kWaves + wave; grp < groups; grp += (int64_t)gridDim.x * kWaves) {
    const int64_t row = grp * 16 + col;                   // this lane's row as an A operand
    // features: u = c / ||c||, straight into the A layout (k = 8 g + 32 kk + i)
    float v[K0P / 32][8];
    float n2 = 0.f;
#pragma unroll
    for (int kk = 0; kk < K0P / 32; ++kk)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = 32 * kk + 8 * g + i;
        const float c = (row < R && k < K0) ? x[row * K0 + k] : 0.f;
        v[kk][i] = c;
        n2 += c * c;
      }
    n2 += __shfl_xor(n2, 16);
    n2 += __shfl_xor(n2, 32);
    const float sc = n2 > 0.f ? rsqrtf(n2) : 0.f;
    h8 a1[K0P / 32];
#pragma unroll
    for (int kk = 0; kk < K0P / 32; ++kk)
#pragma unroll
      for (int i = 0; i < 8; ++i) a1[kk][i] = (_Float16)(v[kk][i] * sc);

    // layer 1 -> hb
#pragma unroll
    for (int nt = 0; nt < H / 16; ++nt) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < K0P / 32; ++kk) {
        const h8 bw = *reinterpret_cast<const h8*>(w1t + (16 * nt + col) * LY::W1ROW + 32 * kk + 8 * g);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1[kk], bw, acc, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = 16 * nt + col;
        hb[(4 * g + q) * LY::HROW + n] = (_Float16)gelu_fast(acc[q] + b1[n]);
      }
    }
    wave_sync();
    h8 a2[H / 32];
#pragma unroll
    for (int kk = 0; kk < H / 32; ++kk) a2[kk] = *reinterpret_cast<const h8*>(hb + col * LY::HROW + 32 * kk + 8 * g);
    wave_sync();                                          // every lane holds its operands: hb takes layer 2
    // layer 2 -> hb
#pragma unroll
    for (int nt = 0; nt < H / 16; ++nt) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < H / 32; ++kk) {
        const h8 bw = *reinterpret_cast<const h8*>(w2t + (16 * nt + col) * LY::W2ROW + 32 * kk + 8 * g);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2[kk], bw, acc, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = 16 * nt + col;
        hb[(4 * g + q) * LY::HROW + n] = (_Float16)gelu_fast(acc[q] + b2[n]);
      }
    }
    wave_sync();
    // layer 3 and head: lane (row col, quarter g) sums a quarter of the hidden units
    float s0 = 0.f, s1 = 0.f;
#pragma unroll 8
    for (int k = g * (H / 4); k < (g + 1) * (H / 4); ++k) {
      const float h = (float)hb[col * LY::HROW + k];
      s0 += h * w3[2 * k];
      s1 += h * w3[2 * k + 1];
    }
    s0 += __shfl_xor(s0, 16);
    s1 += __shfl_xor(s1, 16);
    s0 += __shfl_xor(s0, 32);
    s1 += __shfl_xor(s1, 32);
    if (g == 0 && row < R) {
      const float mu = s0 + b3[0];
      const float s = fminf(fmaxf(s1 + b3[1], -kSClip), kSClip);
      if (fallback) {
        const float c = expf(-0.5f * s);
        tau[row] = c >= min_conf ? mu : fallback[row];
        if (conf) conf[row] = c;
      } else {
        out[2 * row] = mu;
        out[2 * row + 1] = s;
      }
    }
    wave_sync();                                          // hb is rewritten by the next group
  }
}

template <int K0P, int H>
hipError_t launch_infer(const float* theta, int K0, const float* x, int64_t R, float* out, const float* fallback,
                        float min_conf, float* tau, float* conf, hipStream_t st) {
  const size_t lds = InferLds<K0P, H>::bytes(4);
  auto k = mlp_infer_kernel<K0P, H>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  const int64_t groups = (R + 15) / 16;
  int64_t blocks = (groups + 3) / 4;
  if (blocks > 2 * (int64_t)cus) blocks = 2 * (int64_t)cus;    // persistent: two workgroups per CU
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(256), lds, st, theta, K0, x, R, out, fallback, min_conf, tau, conf);
  return hipGetLastError();
}

// the fused kernel's shapes: in_dim <= 64, hidden 32, 64 or 128
hipError_t infer_dispatch(const float* theta, int K0, int H, const float* x, int64_t R, float* out,
                          const float* fallback, float min_conf, float* tau, float* conf, hipStream_t st) {
  if (K0 <= 32) {
    if (H == 32) return launch_infer<32, 32>(theta, K0, x, R, out, fallback, min_conf, tau, conf, st);
    if (H == 64) return launch_infer<32, 64>(theta, K0, x, R, out, fallback, min_conf, tau, conf, st);
    if (H == 128) return launch_infer<32, 128>(theta, K0, x, R, out, fallback, min_conf, tau, conf, st);
  } else if (K0 <= 64) {
    if (H == 32) return launch_infer<64, 32>(theta, K0, x, R, out, fallback, min_conf, tau, conf, st);
    if (H == 64) return launch_infer<64, 64>(theta, K0, x, R, out, fallback, min_conf, tau, conf, st);
    if (H == 128) return launch_infer<64, 128>(theta, K0, x, R, out, fallback, min_conf, tau, conf, st);
  }
  return hipErrorNotSupported;
}

}  // namespace

bool mlp_fused_supported(int in_dim, int hidden) {
  return in_dim >= 1 && in_dim <= 64 && (hidden == 32 || hidden == 64 || hidden == 128);
}

hipError_t mlp_infer(const float* theta, int in_dim, int hidden, const float* x, int64_t rows, float* out,
                     hipStream_t st) {
  if (rows == 0) return hipSuccess;
  return infer_dispatch(theta, in_dim, hidden, x, rows, out, nullptr, 0.f, nullptr, nullptr, st);
}

hipError_t mlp_infer_select(const float* theta, int in_dim, int hidden, const float* x, int64_t rows,
                            const float* fallback, float min_conf, float* tau, float* conf, hipStream_t st) {
  if (rows == 0) return hipSuccess;
  return infer_dispatch(theta, in_dim, hidden, x, rows, nullptr, fallback, min_conf, tau, conf, st);
}

size_t mlp_num_params(int in_dim, int hidden) { return layout(in_dim, hidden).total; }

size_t mlp_workspace_floats(int in_dim, int hidden, int64_t rows) {
  return size_t(rows) * (size_t(in_dim) + 6 * size_t(hidden) + 4);
}

hipError_t mlp_forward(const float* theta, int in_dim, int hidden, const float* x, int64_t rows, float* out,
                       void* ws, hipStream_t st) {
  if (rows == 0) return hipSuccess;
  const Work w = carve(ws, rows, in_dim, hidden);
  return forward_impl(theta, in_dim, hidden, x, rows, out, nullptr, nullptr, w, st);
}

hipError_t mlp_backward(const float* theta, int in_dim, int hidden, const float* x, const float* delta,
                        int64_t rows, float* grad, float* loss_sum, float* out, void* ws, hipStream_t st) {
  if (rows == 0) return hipSuccess;
  const int K0 = in_dim, H = hidden;
  const Layout L = layout(K0, H);
  const Work w = carve(ws, rows, K0, H);
  const int R = (int)rows;
  const float inv = 1.f / float(rows);
  FCC_TRY(forward_impl(theta, K0, H, x, rows, out, delta, loss_sum, w, st));
  // layer 3: dW3 = H2^T dO / R, db3, dH2 = dO W3^T
  FCC_TRY((gemm<true, false, kEpiStore>(w.H2, H, w.dO, 2, grad + L.W3, 2, H, 2, R, inv, nullptr, nullptr, st)));
  hipLaunchKernelGGL(colsum_kernel, dim3(2), dim3(256), 0, st, w.dO, rows, 2, inv, grad + L.b3);
  FCC_TRY((gemm<false, true, kEpiStore>(w.dO, 2, theta + L.W3, 2, w.dH2, H, R, H, 2, 1.f, nullptr, nullptr, st)));
  hipLaunchKernelGGL(gelu_backward_kernel, dim3(blocks_for(rows * H, 256)), dim3(256), 0, st, w.dH2, w.Z2, rows * H);
  // layer 2
  FCC_TRY((gemm<true, false, kEpiStore>(w.H1, H, w.dH2, H, grad + L.W2, H, H, H, R, inv, nullptr, nullptr, st)));
  hipLaunchKernelGGL(colsum_kernel, dim3(H), dim3(256), 0, st, w.dH2, rows, H, inv, grad + L.b2);
  FCC_TRY((gemm<false, true, kEpiStore>(w.dH2, H, theta + L.W2, H, w.dH1, H, R, H, H, 1.f, nullptr, nullptr, st)));
  hipLaunchKernelGGL(gelu_backward_kernel, dim3(blocks_for(rows * H, 256)), dim3(256), 0, st, w.dH1, w.Z1, rows * H);
  // layer 1
  FCC_TRY((gemm<true, false, kEpiStore>(w.U, K0, w.dH1, H, grad + L.W1, H, K0, H, R, inv, nullptr, nullptr, st)));
  hipLaunchKernelGGL(colsum_kernel, dim3(H), dim3(256), 0, st, w.dH1, rows, H, inv, grad + L.b1);
  return hipGetLastError();
}

hipError_t mlp_select(const float* out, const float* fallback, int64_t rows, float min_conf, float* tau,
                      float* conf, hipStream_t st) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(select_kernel, dim3(blocks_for(rows, 256)), dim3(256), 0, st, out, fallback, rows, min_conf,
                     tau, conf);
  return hipGetLastError();
}

hipError_t mlp_adam(float* theta, float* m, float* v, const float* grad, int64_t n, float lr, float b1, float b2,
                    float eps, int step, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, theta, m, v, grad, n, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

}  // namespace fcc
