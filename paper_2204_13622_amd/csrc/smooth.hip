// Pair stage with recursive cross-spectrum smoothing, alpha < 1 (Sec. 2, eq. 1):
//   R(t, f) = (1 - alpha) R(t - 1, f) + alpha X_i(t, f) X_j(t, f)^*,
// then the PHAT R / |R| per pair (the per-microphone factorisation of the
// alpha = 1 path does not hold here), the fold of eq. (8), the projection of
// eq. (9), the expansion y = 2 Re{U z} and the first-index argmax, optionally
// refined by quadratic interpolation (Sec. 2).
//
// The recursion is linear, so it is scanned in chunks of frames in parallel
// and stitched exactly:
//   1. local scan: every (chunk, pair) runs the recursion from R = 0 over its
//      chunk and keeps only the final state S_c;
//   2. carry: per (pair, bin), R_in(0) = the caller's state and
//      R_in(c + 1) = beta^len(c) R_in(c) + S_c, beta = 1 - alpha;
//   3. every chunk reruns the recursion from R_in(c) and evaluates FCC on
//      each frame; the last chunk hands the final state back to the caller.
//
// Lane layout (passes 1 and 3): a 64-lane workgroup serves four pairs with
// 16 lanes each.  Lane l of a pair owns the folded bins f = l + 16 s
// (f < N/4) together with their mirrors N/2 - f, which is exactly what the
// fold needs, and lane 0 also owns the centre bin N/4.  The per-lane partial
// coefficients are summed over the 16 lanes by cross-lane shuffles; the lags
// are then spread over the 16 lanes (lag i on lane i mod 16) and the argmax is
// a 16-lane reduction on (value, index).
#include "device_common.hpp"
#include "kernels.hpp"

namespace fcc {
namespace {

constexpr int kGroup = 16;            // lanes per pair
constexpr int kPairsPerBlock = 4;
constexpr int kThreads = kGroup * kPairsPerBlock;
constexpr int kMaxLagSlots = 5;       // lags per lane: I <= 80

struct Chunking {
  int64_t len;      // frames per chunk (the last one may be shorter)
  int64_t count;    // chunks
};

Chunking chunking(int64_t T, int P) {
  const int64_t groups = (P + kPairsPerBlock - 1) / kPairsPerBlock;
  int64_t want = (8192 + groups - 1) / groups;       // aim at ~8k single-wave workgroups
  const int64_t most = (T + 7) / 8;                   // of at least 8 frames each
  if (want > most) want = most;
  if (want < 1) want = 1;
  Chunking c;
  c.len = (T + want - 1) / want;
  c.count = (T + c.len - 1) / c.len;
  return c;
}

// raw spectrum of one microphone in the packed layout: slot 0 = (X(0), X(N/2))
__device__ __forceinline__ void load_bins(const float2* __restrict__ x, int f, int NH, float2& lo, float2& hi) {
  if (f == 0) {
    const float2 v = x[0];
    lo = make_float2(v.x, 0.f);
    hi = make_float2(v.y, 0.f);
  } else {
    lo = x[f];
    hi = x[NH - f];
  }
}

__device__ __forceinline__ float2 smooth_step(float2 R, float2 a, float2 b, float alpha, float beta) {
  const float2 c = cmul_conj(a, b);
  return make_float2(beta * R.x + alpha * c.x, beta * R.y + alpha * c.y);
}

__device__ __forceinline__ float2 phat_pair(float2 R) {
  const float n2 = R.x * R.x + R.y * R.y;
  if (n2 < 1.17549435e-38f) return make_float2(0.f, 0.f);
  const float s = rsqrtf(n2);
  return make_float2(R.x * s, R.y * s);
}

// state index of bin b of pair p
__device__ __forceinline__ int64_t sidx(int p, int b, int F) { return (int64_t)p * F + b; }

// ---- pass 1: local scan of every chunk but the last ----------------------
template <int S>
__global__ __launch_bounds__(kThreads) void smooth_local_kernel(
    const float2* __restrict__ spec, int64_t T, int M, int P, int N, int64_t clen, int groups,
    const uint8_t* __restrict__ pairs, float alpha, float2* __restrict__ scratch) {
  const int NH = N / 2, m = N / 4, F = NH + 1;
  const int lane = threadIdx.x % kGroup, grp = threadIdx.x / kGroup;
  const int pg = blockIdx.x % groups;
  const int64_t c = blockIdx.x / groups;
  const int p = pg * kPairsPerBlock + grp;
  if (p >= P) return;                       // no cross-lane work in this pass
  const int i = pairs[2 * p], j = pairs[2 * p + 1];
  const float beta = 1.f - alpha;
  float2 lo[S], hi[S], ce = make_float2(0.f, 0.f);
#pragma unroll
  for (int s = 0; s < S; ++s) lo[s] = hi[s] = make_float2(0.f, 0.f);
  const int64_t t0 = c * clen, t1 = t0 + clen < T ? t0 + clen : T;
  for (int64_t t = t0; t < t1; ++t) {
    const float2* xi = spec + (t * M + i) * NH;
    const float2* xj = spec + (t * M + j) * NH;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int f = lane + kGroup * s;
      if (f < m) {
        float2 il, ih, jl, jh;
        load_bins(xi, f, NH, il, ih);
        load_bins(xj, f, NH, jl, jh);
        lo[s] = smooth_step(lo[s], il, jl, alpha, beta);
        hi[s] = smooth_step(hi[s], ih, jh, alpha, beta);
      }
    }
    if (lane == 0) ce = smooth_step(ce, xi[m], xj[m], alpha, beta);
  }
  float2* out = scratch + c * (int64_t)P * F;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int f = lane + kGroup * s;
    if (f < m) {
      out[sidx(p, f, F)] = lo[s];
      out[sidx(p, NH - f, F)] = hi[s];
    }
  }
  if (lane == 0) out[sidx(p, m, F)] = ce;
}

// ---- pass 2: carries across chunks, in place ------------------------------
// scratch[c] holds S_c (c < count - 1) on entry and R_in(c) on return.
__global__ void smooth_carry_kernel(const float2* __restrict__ state, float2* __restrict__ scratch,
                                    int64_t PF, int64_t count, float beta_len) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= PF) return;
  float2 st = state[e];
  for (int64_t c = 0; c < count; ++c) {
    float2* slot = scratch + c * PF + e;
    const float2 local = c + 1 < count ? *slot : make_float2(0.f, 0.f);
    *slot = st;
    st = make_float2(beta_len * st.x + local.x, beta_len * st.y + local.y);
  }
}

// ---- pass 3: rerun each chunk from its carry and evaluate FCC --------------
template <int S, int DB>
__global__ __launch_bounds__(kThreads) void smooth_fcc_kernel(
    const float2* __restrict__ spec, int64_t T, int M, int P, int N, int I, int D, int lag0, float inv_r,
    int64_t clen, int groups, const uint8_t* __restrict__ pairs, float alpha,
    const float* __restrict__ pfold /*[N/4 + 1][DB]*/, const float* __restrict__ dict /*[I][2D]*/,
    const float2* __restrict__ scratch, float2* __restrict__ state, int32_t* __restrict__ tdoa,
    float* __restrict__ tau, float* __restrict__ yout) {
  extern __shared__ float lds[];
  const int NH = N / 2, m = N / 4, F = NH + 1;
  constexpr int PW = DB + 1;                      // padded basis row: conflict-free across lanes
  float* pf = lds;                                // [m + 1][PW]
  float* dc = lds + (m + 1) * PW;                 // [I][2D]
  for (int e = threadIdx.x; e < (m + 1) * DB; e += kThreads) pf[(e / DB) * PW + e % DB] = pfold[e];
  for (int e = threadIdx.x; e < I * 2 * D; e += kThreads) dc[e] = dict[e];
  __syncthreads();

  const int lane = threadIdx.x % kGroup, grp = threadIdx.x / kGroup;
  const int pg = blockIdx.x % groups;
  const int64_t c = blockIdx.x / groups;
  const int pq = pg * kPairsPerBlock + grp;
  const bool active = pq < P;                     // idle groups mirror pair 0 so every shuffle is uniform
  const int p = active ? pq : 0;
  const int i = pairs[2 * p], j = pairs[2 * p + 1];
  const float beta = 1.f - alpha;
  const float2* in = scratch + c * (int64_t)P * F;
  float2 lo[S], hi[S], ce = make_float2(0.f, 0.f);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int f = lane + kGroup * s;
    lo[s] = hi[s] = make_float2(0.f, 0.f);
    if (f < m) {
      lo[s] = in[sidx(p, f, F)];
      hi[s] = in[sidx(p, NH - f, F)];
    }
  }
  if (lane == 0) ce = in[sidx(p, m, F)];

  const int64_t t0 = c * clen, t1 = t0 + clen < T ? t0 + clen : T;
  for (int64_t t = t0; t < t1; ++t) {
    const float2* xi = spec + (t * M + i) * NH;
    const float2* xj = spec + (t * M + j) * NH;
    float a[DB], b[DB];
#pragma unroll
    for (int k = 0; k < DB; ++k) a[k] = b[k] = 0.f;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int f = lane + kGroup * s;
      if (f < m) {
        float2 il, ih, jl, jh;
        load_bins(xi, f, NH, il, ih);
        load_bins(xj, f, NH, jl, jh);
        lo[s] = smooth_step(lo[s], il, jl, alpha, beta);
        hi[s] = smooth_step(hi[s], ih, jh, alpha, beta);
        const float2 el = phat_pair(lo[s]), eh = phat_pair(hi[s]);
        const float2 xs = cadd(el, eh), xd = csub(el, eh);            // eq. (8)
        const float* w = pf + f * PW;
#pragma unroll
        for (int k = 0; k < DB; ++k) {
          const float2 x = (k % 2 == 0) ? xs : xd;                      // eq. (6) order
          a[k] += w[k] * x.x;
          b[k] += w[k] * x.y;
        }
      }
    }
    if (lane == 0) {
      ce = smooth_step(ce, xi[m], xj[m], alpha, beta);
      const float2 ec = phat_pair(ce);
      const float* w = pf + m * PW;
#pragma unroll
      for (int k = 0; k < DB; k += 2) {                                 // centre bin: symmetric k only
        a[k] += w[k] * ec.x;
        b[k] += w[k] * ec.y;
      }
    }
    // sum the coefficients over the pair's 16 lanes; every lane ends with z
#pragma unroll
    for (int off = kGroup / 2; off > 0; off >>= 1)
#pragma unroll
      for (int k = 0; k < DB; ++k) {
        a[k] += __shfl_xor(a[k], off, kGroup);
        b[k] += __shfl_xor(b[k], off, kGroup);
      }
    // expansion to the lags of this lane and first-index argmax
    float y[kMaxLagSlots];
    float best = -3.4e38f;
    int bi = I;
#pragma unroll
    for (int q = 0; q < kMaxLagSlots; ++q) {
      const int ii = lane + kGroup * q;
      y[q] = 0.f;
      if (ii < I) {
        const float* dr = dc + ii * 2 * D;
        float v = 0.f;
#pragma unroll
        for (int k = 0; k < DB; ++k)
          if (k < D) v += dr[2 * k] * a[k] + dr[2 * k + 1] * b[k];
        y[q] = v;
        if (v > best) { best = v; bi = ii; }
      }
    }
#pragma unroll
    for (int off = kGroup / 2; off > 0; off >>= 1) {
      const float ov = __shfl_xor(best, off, kGroup);
      const int oi = __shfl_xor(bi, off, kGroup);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    const int64_t row = t * P + p;
    if (tau) {
      // neighbours of the maximum for the quadratic refinement
      const int il = bi > 0 ? bi - 1 : 0, ih = bi + 1 < I ? bi + 1 : I - 1;
      float sl = 0.f, sh = 0.f;
#pragma unroll
      for (int q = 0; q < kMaxLagSlots; ++q) {
        if (q == il / kGroup) sl = y[q];
        if (q == ih / kGroup) sh = y[q];
      }
      const float y_lo = __shfl(sl, il % kGroup, kGroup);
      const float y_hi = __shfl(sh, ih % kGroup, kGroup);
      if (active && lane == 0) {
        float d = 0.f;
        const float den = y_lo - 2.f * best + y_hi;
        if (bi > 0 && bi < I - 1 && den != 0.f) d = 0.5f * (y_lo - y_hi) / den;
        tau[row] = ((float)(bi - lag0) + d) * inv_r;
      }
    }
    if (active) {
      if (tdoa && lane == 0) tdoa[row] = bi - lag0;
      if (yout)
#pragma unroll
        for (int q = 0; q < kMaxLagSlots; ++q) {
          const int ii = lane + kGroup * q;
          if (ii < I) yout[row * I + ii] = y[q];
        }
    }
  }
  // the last chunk leaves R after the final frame for the next call
  if (active && t1 == T) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int f = lane + kGroup * s;
      if (f < m) {
        state[sidx(p, f, F)] = lo[s];
        state[sidx(p, NH - f, F)] = hi[s];
      }
    }
    if (lane == 0) state[sidx(p, m, F)] = ce;
  }
}

template <int S>
hipError_t launch_s(const SmoothArgs& a, const Chunking& ch) {
  const int groups = (a.P + kPairsPerBlock - 1) / kPairsPerBlock;
  if (ch.count > 1) {
    hipLaunchKernelGGL(smooth_local_kernel<S>, dim3((unsigned)((ch.count - 1) * groups)), dim3(kThreads), 0,
                       a.stream, a.spec, a.T, a.M, a.P, a.N, ch.len, groups, a.pairs, a.alpha, a.scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t PF = (int64_t)a.P * (a.N / 2 + 1);
  const float beta_len = powf(1.f - a.alpha, (float)ch.len);
  hipLaunchKernelGGL(smooth_carry_kernel, dim3((unsigned)((PF + 255) / 256)), dim3(256), 0, a.stream, a.state,
                     a.scratch, PF, ch.count, beta_len);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = sizeof(float) * (size_t(a.N / 4 + 1) * (a.Dfold + 1) + size_t(a.I) * 2 * a.D);
  const unsigned blocks = (unsigned)(ch.count * groups);
  const float inv_r = 1.f / (float)a.r;
#define FCC_SMOOTH_FCC(DB)                                                                                   \
  hipLaunchKernelGGL((smooth_fcc_kernel<S, DB>), dim3(blocks), dim3(kThreads), lds, a.stream, a.spec, a.T, \
                     a.M, a.P, a.N, a.I, a.D, a.lag0, inv_r, ch.len, groups, a.pairs, a.alpha, a.pfold,    \
                     a.dict, a.scratch, a.state, a.tdoa, a.tau, a.y)
  switch (a.Dfold) {
    case 4: FCC_SMOOTH_FCC(4); break;
    case 8: FCC_SMOOTH_FCC(8); break;
    case 12: FCC_SMOOTH_FCC(12); break;
    case 16: FCC_SMOOTH_FCC(16); break;
    case 24: FCC_SMOOTH_FCC(24); break;
    case 32: FCC_SMOOTH_FCC(32); break;
    default: return hipErrorInvalidValue;
  }
#undef FCC_SMOOTH_FCC
  return hipGetLastError();
}

__global__ void fill_zero_kernel(float* __restrict__ p, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = 0.f;
}

}  // namespace

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

size_t smooth_scratch_bytes(int64_t T, int P, int N) {
  if (T <= 0) return 0;
  const Chunking ch = chunking(T, P);
  return sizeof(float2) * size_t(ch.count) * size_t(P) * size_t(N / 2 + 1);
}

bool smooth_supported(const SmoothArgs& a) {
  const size_t lds = sizeof(float) * (size_t(a.N / 4 + 1) * (a.Dfold + 1) + size_t(a.I) * 2 * a.D);
  return a.N >= 16 && a.N <= 2048 && a.I <= kGroup * kMaxLagSlots && a.Dfold >= a.D &&
         (a.Dfold == 4 || a.Dfold == 8 || a.Dfold == 12 || a.Dfold == 16 || a.Dfold == 24 || a.Dfold == 32) &&
         lds <= 64 * 1024 && a.alpha > 0.f && a.alpha <= 1.f;
}

hipError_t launch_smooth(const SmoothArgs& a) {
  if (a.T == 0) return hipSuccess;
  if (!smooth_supported(a)) return hipErrorInvalidValue;
  const Chunking ch = chunking(a.T, a.P);
  switch (a.N) {        // folded-bin slots per lane: N/4 bins over 16 lanes
    case 16:
    case 32:
    case 64: return launch_s<1>(a, ch);
    case 128: return launch_s<2>(a, ch);
    case 256: return launch_s<4>(a, ch);
    case 512: return launch_s<8>(a, ch);
    case 1024: return launch_s<16>(a, ch);
    case 2048: return launch_s<32>(a, ch);
  }
  return hipErrorInvalidValue;
}

}  // namespace fcc
