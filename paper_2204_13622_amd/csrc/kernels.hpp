// Launch interfaces of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fcc.h"

namespace fcc {

struct StftArgs {
  const float* x;            // [M][ld] audio
  int64_t ld;
  int64_t T;                 // frames
  int M, N, hop;
  fcc_precision precision;
  const float2* twiddle;     // [N] exp(-j 2 pi f / N)
  void* out;                 // [T][M][N/2 + 1] complex, storage format
  bool raw;                  // true: X itself (FP32 only), false: X / |X|
  hipStream_t stream;
};

// direction-of-arrival search over a direction grid
struct DoaArgs {
  const float* y;            // [T][P][I] correlations
  int64_t T;
  int P, I;
  const float* table;        // [P][G] fractional lag index per pair and direction
  int G;
  int32_t* doa;              // [T] first best direction
  float* score;              // [T][G] or null
  hipStream_t stream;
};

// pair stage with recursive smoothing, alpha < 1 (eq. 1); FP32 raw spectra
struct SmoothArgs {
  const float2* spec;        // [T][M][N/2] raw spectra, packed real layout
  int64_t T;
  int M, P, N, I, D, Dfold;
  int lag0, r;
  float alpha;
  const uint8_t* pairs;      // [P][2]
  const float* pfold;        // [N/4 + 1][Dfold]
  const float* dict;         // [I][2D]
  float2* state;             // [P][N/2 + 1] R before the first frame; R after the last on return
  float2* scratch;           // smooth_scratch_bytes(T, P, N)
  int32_t* tdoa;             // [T][P] or null
  float* tau;                // [T][P] interpolated lag (samples) or null
  float* y;                  // [T][P][I] or null
  hipStream_t stream;
};

struct PairArgs {
  const void* spec;          // [T][M][F] complex, storage format
  int64_t T;
  int M, P, N, I, D;
  int lag0;                  // index of lag 0 on the grid: r tau_max
  int r;                     // lag grid spacing 1/r sample (Sec. 3)
  fcc_precision precision;
  fcc_method method;
  const uint8_t* pairs;      // [P][2]
  const float* basis32;      // [D][N/4 + 1]
  const float* dict;         // [I][2D]   (2 Dc, -2 Ds)
  const float2* lagw;        // [I][F]    exp(j 2 pi f tau_i / N)
  int Dpad;                  // D padded to the matrix-core tiles
  const void* prow16;        // half2  [Dpad][N/2] full-length rows, slot pairs
  const float2* prow32;      // float2 [Dpad][N/2]
  const float* gexp;         // [Ipad][Dpad] G = Dc - Ds
  int Dfold;                 // D padded to the FP32 fold kernel's register block
  const float* pfold;        // [N/4 + 1][Dfold] p_hat transposed, zero beyond D
  const float2* twiddle_r;   // [r N] exp(-j 2 pi n / (r N))
  int32_t* tdoa;             // [T][P] or null
  float* y;                  // [T][P][I] or null
  float* coef;               // [T][P][2D] projection coefficients (a_k, b_k), or null
  float* tau_frac;           // [T][P] argmax refined by quadratic interpolation, or null
  hipStream_t stream;
};

hipError_t launch_stft_phat(const StftArgs& a);

size_t mlp_num_params(int in_dim, int hidden);
size_t mlp_workspace_floats(int in_dim, int hidden, int64_t rows);
hipError_t mlp_forward(const float* theta, int in_dim, int hidden, const float* x, int64_t rows, float* out,
                       void* ws, hipStream_t st);
hipError_t mlp_backward(const float* theta, int in_dim, int hidden, const float* x, const float* delta,
                        int64_t rows, float* grad, float* loss_sum, float* out, void* ws, hipStream_t st);
hipError_t mlp_select(const float* out, const float* fallback, int64_t rows, float min_conf, float* tau,
                      float* conf, hipStream_t st);
hipError_t mlp_adam(float* theta, float* m, float* v, const float* grad, int64_t n, float lr, float b1, float b2,
                    float eps, int step, hipStream_t st);
hipError_t launch_pair_valu(const PairArgs& a);
bool pair_mfma_supported(const PairArgs& a);
bool pair_fold32_supported(const PairArgs& a);
hipError_t launch_pair_fold32(const PairArgs& a);
bool gcc_ifft_supported(const PairArgs& a);
size_t smooth_scratch_bytes(int64_t T, int P, int N);
bool smooth_supported(const SmoothArgs& a);
hipError_t launch_smooth(const SmoothArgs& a);
bool doa_supported(const DoaArgs& a);
hipError_t launch_doa(const DoaArgs& a);
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t stream);   // a fill kernel, safe under graph capture
hipError_t launch_gcc_ifft(const PairArgs& a);
hipError_t launch_pair_mfma(const PairArgs& a);

}  // namespace fcc
