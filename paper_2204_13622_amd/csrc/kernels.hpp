// Launch interfaces of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

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

// ---- batches of independent arrays ------------------------------------------
// One array of a batch as the device sees it (a table in the batch image).
struct BatchArray {
  int32_t M, P, N, hop, I, lag0;
  int64_t T;                 // frames
  int64_t L;                 // samples per microphone = row stride of its audio block
  int64_t audio_off;         // float offset of its [M][L] audio block
  int64_t spec_off;          // byte offset of its spectra in the workspace
  int64_t tdoa_off;          // element offset of its [T][P] output
  int64_t img_off;           // byte offset of its plan tables in the batch image
  int64_t tab_twiddle, tab_pairs, tab_prow16, tab_gexp;   // table offsets inside its plan tables
  int64_t stft_first;        // index of its first front-end item
};

// Arrays sharing one matrix-core tile shape (host side).
struct BatchClass {
  int index = 0;             // position in the batch's class list
  int kb = 0, tt = 0;        // components in blocks of 4, lags in tiles of 16
  int member_first = 0, member_count = 0;   // slice of the member list
  std::vector<int64_t> member_frames;
  int head_words_max = 0, slab_words_max = 0;
  size_t wprefix_off = 0;    // image offset of the cost prefix [member_count + 1] (int64)
  int64_t workgroups(int cus, int blocks_per_cu, int waves) const;
};

// cost of one pair-stage frame of frame size N on a class's cost scale
int64_t pair_frame_weight(int N);

// Front-end items of one frame size: items first .. first + count - 1.
struct BatchStftRange {
  int N;
  int64_t first, count;
};

struct PairTuning {
  int waves = 4;             // wavefronts per workgroup
  int blocks_per_cu = 2;
};

struct BatchRun {
  const BatchArray* arrays;  // device
  int n_arrays;
  const int32_t* members;    // device: member lists of every class, back to back
  const unsigned char* image;
  const float* audio;
  unsigned char* spec;
  int32_t* tdoa;
  const int32_t* item_array; // device: array of every front-end item
  std::vector<BatchStftRange> stft_ranges;   // one per frame size present
  fcc_precision precision;
  hipStream_t stream;
};

hipError_t launch_batch_stft(const BatchRun& r);
hipError_t launch_batch_pair(const BatchRun& r, const BatchClass& c, const PairTuning& t);
int batch_pair_waves(const BatchClass& c, const PairTuning& t);          // wavefronts per workgroup in use
int64_t batch_pair_workgroups(const BatchClass& c, const PairTuning& t); // workgroups of the class's launch
int stft_transforms_per_block(int N);
int batch_head_words(int Dpad, int NH, int TT, int P);   // LDS words before the wavefront slabs
int batch_slab_words(int N, int I);                      // LDS words of one wavefront slab

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
  fcc_operands operands;     // matrix-core operand types
  const void* prow_op;       // [Dpad][N/2] rows in the storage type's operand form (BF16 pairs, or
                             // FP16 pairs scaled by 2^e_k for e4m3), or null
  const float* gexp_op;      // [Ipad][Dpad] G with the rows' inverse scales, or null
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
bool mlp_fused_supported(int in_dim, int hidden);
hipError_t mlp_infer(const float* theta, int in_dim, int hidden, const float* x, int64_t rows, float* out,
                     hipStream_t st);
hipError_t mlp_infer_select(const float* theta, int in_dim, int hidden, const float* x, int64_t rows,
                            const float* fallback, float min_conf, float* tau, float* conf, hipStream_t st);
hipError_t mlp_select(const float* out, const float* fallback, int64_t rows, float min_conf, float* tau,
                      float* conf, hipStream_t st);
hipError_t mlp_adam(float* theta, float* m, float* v, const float* grad, int64_t n, float lr, float b1, float b2,
                    float eps, int step, hipStream_t st);
hipError_t launch_pair_valu(const PairArgs& a);
bool pair_valu_supported(const PairArgs& a);
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
// address of this device's static scratch (FCC_NOALLOC_SCRATCH_BYTES bytes), fetched once per device
hipError_t noalloc_scratch(void** out);

}  // namespace fcc
