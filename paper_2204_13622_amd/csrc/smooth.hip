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

// Every supported N >= 128 gives N/4 = 16 S folded bins, so each lane of a
// pair owns exactly S of them; only N <= 64 (S = 1) leaves lanes idle.
template <int S>
__device__ __forceinline__ bool owns_bin(int f, int m) { return S > 1 || f < m; }

// Where a lane reads its bins: bin f = lane + 16 s of a microphone sits at
// lo + 16 s and bin N/2 - f at hi - 16 s (for s >= 1; slot 0 of lane 0 is the
// packed (X(0), X(N/2)) pair of the spectrum layout).  The pointers step one
// frame at a time, so every load is a base plus a constant offset.
struct BinPtrs {
  const float2* lo;
  const float2* hi;
  __device__ __forceinline__ BinPtrs(const float2* row, int NH, int lane) : lo(row + lane), hi(row + NH - lane) {}
  __device__ __forceinline__ void advance(int64_t stride) {
    lo += stride;
    hi += stride;
  }
};

// Slot group of one frame, branch-free: bins f and N/2 - f of microphones i
// and j for slots s0 .. s0 + G - 1 of a lane.  The FCC pass (and the local
// scan for large N) loads and consumes a frame in groups of at most 4 slots,
// so that the loads in flight leave registers for three waves per SIMD.
constexpr int kSlotGroup = 4;

template <int S, int G>
struct SlotBins {
  float2 il[G], ih[G], jl[G], jh[G];
  __device__ __forceinline__ void load(const BinPtrs& pi, const BinPtrs& pj, int m, int lane, int s0) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int s = s0 + g;
      il[g] = ih[g] = jl[g] = jh[g] = make_float2(0.f, 0.f);
      if (owns_bin<S>(lane + 16 * s, m)) {
        il[g] = pi.lo[16 * s];
        jl[g] = pj.lo[16 * s];
        if (s > 0) {
          ih[g] = pi.hi[-16 * s];
          jh[g] = pj.hi[-16 * s];
        } else {
          // slot 0: bin N/2 - lane for lanes 1..15; lane 0 unpacks DC and Nyquist
          const bool dc = lane == 0;
          ih[g] = (dc ? pi.lo : pi.hi)[0];
          jh[g] = (dc ? pj.lo : pj.hi)[0];
          ih[g] = dc ? make_float2(il[g].y, 0.f) : ih[g];
          jh[g] = dc ? make_float2(jl[g].y, 0.f) : jh[g];
          il[g].y = dc ? 0.f : il[g].y;
          jl[g].y = dc ? 0.f : jl[g].y;
        }
      }
    }
  }
};

// the centre bin N/4: every lane reads it, lane 0 alone owns it
struct CentreBin {
  float2 ci, cj;
  __device__ __forceinline__ void load(const BinPtrs& pi, const BinPtrs& pj, int m, int lane) {
    ci = (pi.lo - lane)[m];
    cj = (pj.lo - lane)[m];
  }
};

// Inside passes 1 and 3 the recursion runs on Q = R / alpha:
//   Q(t) = beta Q(t - 1) + X_i(t) X_j(t)^*,
// one multiply and two fused multiply-adds per component.  The PHAT R / |R|
// is the same for Q; scratch and the caller's state keep R itself.
__device__ __forceinline__ float2 smooth_step(float2 Q, float2 a, float2 b, float beta) {
  return make_float2(fmaf(a.x, b.x, fmaf(a.y, b.y, beta * Q.x)), fmaf(a.y, b.x, fmaf(-a.x, b.y, beta * Q.y)));
}

__device__ __forceinline__ float2 phat_pair(float2 R) {
  const float n2 = R.x * R.x + R.y * R.y;
  const float s = n2 < 1.17549435e-38f ? 0.f : rsqrtf(n2);   // a vanishing bin contributes nothing
  return make_float2(R.x * s, R.y * s);
}

// Cross-lane exchange inside a row of 16 lanes (the pair's lanes) through DPP
// row permutations: the mirrored lane 15 - l, the mirror inside each half
// row, and the lanes at xor 1 and xor 2 inside each quad.  Applied in that
// order the four steps pair every lane with a disjoint set each time, so a
// reduction leaves the full result, bit-identical, on all 16 lanes.
constexpr int kDppRowMirror = 0x140, kDppRowHalfMirror = 0x141, kDppQuadXor1 = 0xB1, kDppQuadXor2 = 0x4E;

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}

__device__ __forceinline__ float row_sum16(float v) {
  v += dpp_f<kDppRowMirror>(v);
  v += dpp_f<kDppRowHalfMirror>(v);
  v += dpp_f<kDppQuadXor1>(v);
  v += dpp_f<kDppQuadXor2>(v);
  return v;
}

// (value, index) maximum, ties to the lower index
template <int CTRL>
__device__ __forceinline__ void argmax_step(float& best, int& bi) {
  const float ov = dpp_f<CTRL>(best);
  const int oi = dpp_i<CTRL>(bi);
  if (ov > best || (ov == best && oi < bi)) {
    best = ov;
    bi = oi;
  }
}

__device__ __forceinline__ void row_argmax16(float& best, int& bi) {
  argmax_step<kDppRowMirror>(best, bi);
  argmax_step<kDppRowHalfMirror>(best, bi);
  argmax_step<kDppQuadXor1>(best, bi);
  argmax_step<kDppQuadXor2>(best, bi);
}

// Workgroups are dealt to the 8 XCDs round-robin.  Renumber them so that
// each XCD owns a contiguous run of (chunk, pair group) indices, i.e. whole
// chunks: every spectrum of a chunk is then read by up to M - 1 pairs through
// one L2 instead of being fetched into several.
__device__ __forceinline__ int64_t xcd_linear_block() {
  constexpr unsigned kXcds = 8;
  const unsigned nb = gridDim.x, xcd = blockIdx.x % kXcds, local = blockIdx.x / kXcds;
  const unsigned per = nb / kXcds, extra = nb % kXcds;
  return (int64_t)xcd * per + (xcd < extra ? xcd : extra) + local;
}

__device__ __forceinline__ float2 cscale(float2 v, float s) { return make_float2(v.x * s, v.y * s); }

// state index of bin b of pair p
__device__ __forceinline__ int64_t sidx(int p, int b, int F) { return (int64_t)p * F + b; }

// ---- pass 1: local scan of every chunk but the last ----------------------
// A workgroup owns one chunk, one tile of 64 consecutive spectrum slots and
// up to 128 consecutive pairs.  Per frame it stages the tile of every
// microphone in LDS (each spectrum value read once, 16-byte loads, double
// buffered so the next frame's loads fly during this frame's work); each
// wave is one group of up to 16 pairs and each lane advances the recursion
// of its slot for those pairs, stepping through them in their lexicographic
// (i-major) order.
constexpr int kTileSlots = 64;
constexpr int kTileGroups = 16;
constexpr int kPairsPerLane = 8;
constexpr int kTilePairs = kTileGroups * kPairsPerLane;
constexpr int kTileThreads = kTileSlots * kTileGroups;
constexpr int kTileFetch = 1;                 // float4 per thread per frame: 32 microphones at most

struct TileFetch {
  float4 v[kTileFetch];
  // frame t of the tile: [M][64 slots] as float4 (2 slots each), zero past N/2
  __device__ __forceinline__ void load(const float2* __restrict__ spec, int64_t t, int M, int NH, int slot0) {
    const int n4 = M * (kTileSlots / 2);
#pragma unroll
    for (int k = 0; k < kTileFetch; ++k) {
      const int e = threadIdx.x + kTileThreads * k, m = e / (kTileSlots / 2), sl = slot0 + 2 * (e % (kTileSlots / 2));
      v[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < n4 && sl < NH) v[k] = *reinterpret_cast<const float4*>(spec + ((t * M + m) * NH + sl));
    }
  }
  __device__ __forceinline__ void store(float4* __restrict__ dst, int M) const {
    const int n4 = M * (kTileSlots / 2);
#pragma unroll
    for (int k = 0; k < kTileFetch; ++k) {
      const int e = threadIdx.x + kTileThreads * k;
      if (e < n4) dst[e] = v[k];
    }
  }
};

// One frame for the 16 pair slots of a wave, straight-line: the scalar unit
// walks (i, j) through the pairs in lexicographic order (clamped to the last
// pair once the walk leaves the triangle; slots past the wave's pairs are
// computed and never stored) and every lane reads both operands of a pair
// from the staged rows.  DC: this lane holds slot 0, the packed (X(0), X(N/2))
// pair, whose two real bins take componentwise products; those selects are
// compiled only into the tile that contains slot 0.
template <bool DC>
__device__ __forceinline__ void tile_frame(const float2* __restrict__ row /*[M][64]*/, int s, int M, int i0, int j0,
                                           float beta, bool dc, float2 (&Q)[kPairsPerLane]) {
  int i = i0, j = j0;
#pragma unroll
  for (int q = 0; q < kPairsPerLane; ++q) {
    const float2 xi = row[i * kTileSlots + s], xj = row[j * kTileSlots + s];
    if constexpr (DC) {
      // (a.x b.x, a.y b.y) on the DC lane, a b^* elsewhere
      const float ay = dc ? 0.f : xi.y, nax = dc ? 0.f : -xi.x, bxy = dc ? xj.y : xj.x;
      Q[q] = make_float2(fmaf(xi.x, xj.x, fmaf(ay, xj.y, beta * Q[q].x)),
                         fmaf(xi.y, bxy, fmaf(nax, xj.y, beta * Q[q].y)));
    } else {
      Q[q] = smooth_step(Q[q], xi, xj, beta);
    }
    // next pair: (i, j + 1), or (i + 1, i + 2) past the end of row i
    const bool wrap = j + 1 == M;
    i = wrap ? i + 1 : i;
    j = wrap ? i + 1 : j + 1;
    const bool out = i >= M - 1;              // past (M - 2, M - 1): stay there
    i = out ? M - 2 : i;
    j = out ? M - 1 : j;
  }
}

__global__ __launch_bounds__(kTileThreads) void smooth_local_kernel(
    const float2* __restrict__ spec, int64_t T, int M, int P, int N, int64_t clen, int tiles, int pblocks,
    float alpha, float2* __restrict__ scratch) {
  extern __shared__ float4 stage[];             // [2][M][64 slots]
  const int NH = N / 2, F = NH + 1;
  int64_t v = blockIdx.x;
  const int pb = (int)(v % pblocks);
  v /= pblocks;
  const int tile = (int)(v % tiles);
  const int64_t c = v / tiles;
  // g: this wave's pair group, uniform (the pair walk below then runs on scalars)
  const int s = threadIdx.x % kTileSlots, g = __builtin_amdgcn_readfirstlane(threadIdx.x / kTileSlots);
  const int slot0 = tile * kTileSlots, slot = slot0 + s;

  // pairs [p0, p0 + np) of this wave, and the first of them as (i, j)
  const int pbase = pb * kTilePairs, pcount = P - pbase < kTilePairs ? P - pbase : kTilePairs;
  const int per = (pcount + kTileGroups - 1) / kTileGroups;
  const int p0 = pbase + g * per;
  int np = P - p0 < per ? P - p0 : per;
  if (np < 0) np = 0;
  // row i of the pair triangle holds the M - 1 - i pairs (i, i + 1 .. M - 1)
  int i0 = 0, rest = p0 < P ? p0 : 0;
  while (rest >= M - 1 - i0) {
    rest -= M - 1 - i0;
    ++i0;
  }
  const int j0 = i0 + 1 + rest;

  const float beta = 1.f - alpha;
  float2 Q[kPairsPerLane];
#pragma unroll
  for (int q = 0; q < kPairsPerLane; ++q) Q[q] = make_float2(0.f, 0.f);
  const int64_t t0 = c * clen, t1 = t0 + clen < T ? t0 + clen : T;
  const int n4 = M * (kTileSlots / 2);
  TileFetch fetch;
  fetch.load(spec, t0, M, NH, slot0);
  fetch.store(stage, M);
  __syncthreads();
  for (int64_t t = t0; t < t1; ++t) {
    const int buf = (int)((t - t0) & 1);
    if (t + 1 < t1) fetch.load(spec, t + 1, M, NH, slot0);
    const float2* row = reinterpret_cast<const float2*>(stage + buf * n4);
    if (tile == 0)
      tile_frame<true>(row, s, M, i0, j0, beta, s == 0, Q);
    else
      tile_frame<false>(row, s, M, i0, j0, beta, false, Q);
    if (t + 1 < t1) fetch.store(stage + (buf ^ 1) * n4, M);
    __syncthreads();
  }

  if (slot >= NH) return;
  float2* out = scratch + c * (int64_t)P * F;
#pragma unroll
  for (int q = 0; q < kPairsPerLane; ++q) {
    if (q < np) {
      float2* o = out + (int64_t)(p0 + q) * F;
      if (slot == 0) {
        o[0] = make_float2(alpha * Q[q].x, 0.f);
        o[NH] = make_float2(alpha * Q[q].y, 0.f);
      } else {
        o[slot] = cscale(Q[q], alpha);
      }
    }
  }
}

// ---- pass 2: carries across chunks, in place ------------------------------
// scratch[c] holds S_c (c < count - 1) on entry and R_in(c) on return.
__global__ void smooth_carry_kernel(const float2* __restrict__ state, float2* __restrict__ scratch,
                                    int64_t PF, int64_t count, float beta_len) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= PF) return;
  // The local sums do not depend on the carry: read a run of them before
  // writing the carries back in their place.
  constexpr int kRun = 8;
  float2 st = state[e];
  for (int64_t c0 = 0; c0 < count; c0 += kRun) {
    float2 local[kRun];
#pragma unroll
    for (int u = 0; u < kRun; ++u) {
      const int64_t c = c0 + u;
      local[u] = c + 1 < count ? scratch[c * PF + e] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < kRun; ++u) {
      const int64_t c = c0 + u;
      if (c < count) {
        scratch[c * PF + e] = st;
        st = make_float2(beta_len * st.x + local[u].x, beta_len * st.y + local[u].y);
      }
    }
  }
}

// ---- pass 3: rerun each chunk from its carry and evaluate FCC --------------

// Advance the recursion of slots s0 .. s0 + G - 1 by one frame and add their
// PHAT-weighted, folded bins (eq. 8) to the partial coefficients (eq. 9),
// symmetric and antisymmetric basis vectors alternating as in eq. (6).
template <int S, int G, int DB>
__device__ __forceinline__ void project_group(const SlotBins<S, G>& cur, int s0, float2 (&lo)[S], float2 (&hi)[S],
                                              float (&a)[DB], float (&b)[DB], const float* pf, int lane, int m,
                                              float beta) {
  constexpr int PW = DB + 1;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int s = s0 + g, f = lane + kGroup * s;
    lo[s] = smooth_step(lo[s], cur.il[g], cur.jl[g], beta);
    hi[s] = smooth_step(hi[s], cur.ih[g], cur.jh[g], beta);
    if (owns_bin<S>(f, m)) {
      const float2 el = phat_pair(lo[s]), eh = phat_pair(hi[s]);
      const float2 xs = cadd(el, eh), xd = csub(el, eh);
      const float* w = pf + f * PW;
#pragma unroll
      for (int k = 0; k < DB; ++k) {
        const float2 x = (k % 2 == 0) ? xs : xd;
        a[k] += w[k] * x.x;
        b[k] += w[k] * x.y;
      }
    }
  }
}

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
  constexpr int DW = 2 * PW;                      // dictionary row: 2 DB coefficients, zero past 2 D, padded
  float* pf = lds;                                // [m + 1][PW]
  float* dc = lds + (m + 1) * PW;                 // [I][DW]
  for (int e = threadIdx.x; e < (m + 1) * DB; e += kThreads) pf[(e / DB) * PW + e % DB] = pfold[e];
  for (int e = threadIdx.x; e < I * DW; e += kThreads) {
    const int row = e / DW, col = e % DW;
    dc[e] = col < 2 * D ? dict[row * 2 * D + col] : 0.f;
  }
  __syncthreads();

  const int lane = threadIdx.x % kGroup, grp = threadIdx.x / kGroup;
  const int64_t v = xcd_linear_block();
  const int pg = (int)(v % groups);
  const int64_t c = v / groups;
  const int pq = pg * kPairsPerBlock + grp;
  const bool active = pq < P;                     // idle groups mirror pair 0 so every shuffle is uniform
  const int p = active ? pq : 0;
  const int i = pairs[2 * p], j = pairs[2 * p + 1];
  const float beta = 1.f - alpha, inv_alpha = 1.f / alpha;
  const float2* in = scratch + c * (int64_t)P * F;
  float2 lo[S], hi[S], ce = make_float2(0.f, 0.f);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int f = lane + kGroup * s;
    lo[s] = hi[s] = make_float2(0.f, 0.f);
    if (f < m) {
      lo[s] = cscale(in[sidx(p, f, F)], inv_alpha);
      hi[s] = cscale(in[sidx(p, NH - f, F)], inv_alpha);
    }
  }
  if (lane == 0) ce = cscale(in[sidx(p, m, F)], inv_alpha);

  const int64_t t0 = c * clen, t1 = t0 + clen < T ? t0 + clen : T;
  const int nq = (I + kGroup - 1) / kGroup;      // lag slots in use, uniform
  const int64_t stride = (int64_t)M * NH;
  BinPtrs pi(spec + (t0 * M + i) * NH, NH, lane), pj(spec + (t0 * M + j) * NH, NH, lane);
  float a[DB], b[DB];
  CentreBin cc;
  // centre bin, sums over the pair's lanes, expansion, argmax and stores of frame t
  auto frame_tail = [&](int64_t t) {
    {
      // centre bin: every lane keeps the same R, lane 0 alone adds it; it
      // meets the symmetric basis vectors only
      ce = smooth_step(ce, cc.ci, cc.cj, beta);
      float2 ec = phat_pair(ce);
      ec = lane == 0 ? ec : make_float2(0.f, 0.f);
      const float* w = pf + m * PW;
#pragma unroll
      for (int k = 0; k < DB; k += 2) {
        a[k] += w[k] * ec.x;
        b[k] += w[k] * ec.y;
      }
    }
    // sum the coefficients over the pair's 16 lanes; every lane ends with z
#pragma unroll
    for (int k = 0; k < DB; ++k) {
      a[k] = row_sum16(a[k]);
      b[k] = row_sum16(b[k]);
    }
    // expansion to the lags of this lane and first-index argmax
    float y[kMaxLagSlots];
    float best = -3.4e38f;
    int bi = I;
#pragma unroll
    for (int q = 0; q < kMaxLagSlots; ++q) {
      y[q] = 0.f;
      if (q < nq) {
        const int ii = lane + kGroup * q;
        const float* dr = dc + (ii < I ? ii : I - 1) * DW;             // rows past I are masked below
        float v = 0.f;
#pragma unroll
        for (int k = 0; k < DB; ++k) v = fmaf(dr[2 * k + 1], b[k], fmaf(dr[2 * k], a[k], v));
        y[q] = v;
        const bool take = ii < I && v > best;
        best = take ? v : best;
        bi = take ? ii : bi;
      }
    }
    row_argmax16(best, bi);
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
  };

  // A frame is loaded and consumed group by group; the loads are not
  // pipelined across groups: at this register count three waves per SIMD
  // hide their latency better than a second buffer would.
  constexpr int G = S < kSlotGroup ? S : kSlotGroup;
  for (int64_t t = t0; t < t1; ++t, pi.advance(stride), pj.advance(stride)) {
    cc.load(pi, pj, m, lane);
#pragma unroll
    for (int k = 0; k < DB; ++k) a[k] = b[k] = 0.f;
#pragma unroll
    for (int s0 = 0; s0 < S; s0 += G) {
      SlotBins<S, G> cur;
      cur.load(pi, pj, m, lane, s0);
      project_group<S, G, DB>(cur, s0, lo, hi, a, b, pf, lane, m, beta);
      __builtin_amdgcn_sched_barrier(0);
    }
    frame_tail(t);
  }
  // the last chunk leaves R after the final frame for the next call
  if (active && t1 == T) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int f = lane + kGroup * s;
      if (f < m) {
        state[sidx(p, f, F)] = cscale(lo[s], alpha);
        state[sidx(p, NH - f, F)] = cscale(hi[s], alpha);
      }
    }
    if (lane == 0) state[sidx(p, m, F)] = cscale(ce, alpha);
  }
}

// pass 3: padded basis rows [N/4 + 1][Dfold + 1] and dictionary rows [I][2 (Dfold + 1)]
size_t smooth_lds_bytes(const SmoothArgs& a) {
  return sizeof(float) * (size_t(a.N / 4 + 1) * (a.Dfold + 1) + size_t(a.I) * 2 * (a.Dfold + 1));
}

template <int S>
hipError_t launch_s(const SmoothArgs& a, const Chunking& ch) {
  const int groups = (a.P + kPairsPerBlock - 1) / kPairsPerBlock;
  if (ch.count > 1) {
    const int tiles = (a.N / 2 + kTileSlots - 1) / kTileSlots, pblocks = (a.P + kTilePairs - 1) / kTilePairs;
    const size_t stage = 2 * sizeof(float4) * size_t(a.M) * (kTileSlots / 2);
    hipLaunchKernelGGL(smooth_local_kernel, dim3((unsigned)((ch.count - 1) * tiles * pblocks)), dim3(kTileThreads),
                       stage, a.stream, a.spec, a.T, a.M, a.P, a.N, ch.len, tiles, pblocks, a.alpha, a.scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t PF = (int64_t)a.P * (a.N / 2 + 1);
  const float beta_len = powf(1.f - a.alpha, (float)ch.len);
  hipLaunchKernelGGL(smooth_carry_kernel, dim3((unsigned)((PF + 63) / 64)), dim3(64), 0, a.stream, a.state,
                     a.scratch, PF, ch.count, beta_len);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = smooth_lds_bytes(a);
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
  const size_t lds = smooth_lds_bytes(a);
  return a.M >= 2 && a.M * (kTileSlots / 2) <= kTileFetch * kTileThreads && a.N >= 16 && a.N <= 2048 &&
         a.I <= kGroup * kMaxLagSlots && a.Dfold >= a.D &&
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
