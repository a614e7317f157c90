/*
 * fcc.h - C ABI of the MI355X (gfx950) Fast Cross-Correlation TDoA library.
 *
 * Method: F. Grondin et al., "Fast Cross-Correlation for TDoA Estimation on
 * Small Aperture Microphone Arrays", arXiv 2204.13622.  For every STFT frame
 * and every microphone pair the library forms the PHAT-weighted
 * cross-spectrum (Sec. 2, eq. 1, optionally smoothed over frames), projects
 * it on the cropped even/odd bases of the rank-D decomposition of the
 * frequency-to-lag matrix (Sec. 4, eqs. 5-9), expands the coefficients to the
 * lags -tau_max .. tau_max (step 1/r, Sec. 3) through the dictionary, and
 * returns the argmax lag (Sec. 2), optionally refined by quadratic
 * interpolation.  The GCC-PHAT comparator (Sec. 3, eq. 2) shares the front end
 * and evaluates eq. (2) at the same lags through an inverse FFT.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns fcc_status; FCC_OK is 0 and errors are negative.  No
 *   C++ exception crosses this boundary.  fcc_last_error() gives a message for
 *   the calling thread's last error.
 * - Argument errors are detected before anything is enqueued: a call that
 *   returns an error has launched no work.  FCC_ERR_HIP reports a failed
 *   launch or copy; faults that happen asynchronously show up at the caller's
 *   next synchronisation of the stream.
 * - Pointers named d_* are device pointers on the current HIP device; the
 *   caller allocates and owns every device buffer (sizes from
 *   fcc_plan_query / fcc_workspace_bytes).  Calls that compute never allocate
 *   device memory.  A plan owns only host memory.
 * - Work is enqueued on `stream` (0 = the null stream) and the call returns
 *   without waiting for it.
 * - A plan is immutable after fcc_plan_create and may be used from several
 *   threads and streams at once; workspaces must not be shared by concurrent
 *   calls.
 * - Microphone pairs p = 0 .. P-1, P = M (M - 1) / 2, enumerate (i, j), i < j,
 *   in lexicographic order: (0,1), (0,2), .., (0,M-1), (1,2), ...
 * - TDoA sign: TDoA_ij = t_i - t_j in samples.  If x_j[n] = x_i[n - d] then
 *   the result for pair (i, j) is -d (R = X_i X_j^* of eq. 1 and the
 *   exp(+j 2 pi f tau / N) kernel of eq. 2).
 * - Failure injection for tests (environment variable FCC_FAULT, read at
 *   every call): "launch" makes every call that would enqueue a kernel or a
 *   copy return FCC_ERR_HIP after its argument checks and before anything is
 *   enqueued; "alloc" makes the host allocations of fcc_plan_create and
 *   fcc_batch_create fail with FCC_ERR_INTERNAL.
 */
#ifndef FCC_H_
#define FCC_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FCC_OK = 0,
  FCC_ERR_INVALID_ARG = -1,       /* argument outside its documented range  */
  FCC_ERR_UNSUPPORTED = -2,       /* valid per the paper, not built here     */
  FCC_ERR_BASIS_AMBIGUOUS = -3,   /* the rank cuts a singular-value cluster  */
  FCC_ERR_HIP = -4,               /* a HIP launch or copy failed             */
  FCC_ERR_INTERNAL = -5
} fcc_status;

/* Storage type of the whitened spectra and of the projection operands.
 * Accumulation, PHAT normalisation, the lag expansion and the argmax are FP32
 * in every mode. */
typedef enum {
  FCC_FP32 = 0,
  FCC_BF16 = 1,
  FCC_FP16 = 2,
  FCC_FP8_E4M3 = 3                /* OCP e4m3 (finite, max 448) */
} fcc_precision;

typedef enum {
  FCC_METHOD_FCC = 0,             /* low-rank even/odd projection (Sec. 4)   */
  FCC_METHOD_GCC = 1              /* eq. (2) evaluated at the I lags (Sec. 3) */
} fcc_method;

/* Operand types of the projection's matrix-core tiles (eq. 9) for the 16-bit
 * and 8-bit storage types; FP32 accumulation either way.
 *   FCC_OPERANDS_FP16     spectra of every storage type widened to FP16
 *                         (exact for unit-modulus values), FP16 basis rows,
 *                         products p_k e_i in FP16 (the default);
 *   FCC_OPERANDS_STORAGE  operands in the storage type: BF16 spectra with BF16
 *                         basis rows and BF16 products (bf16 tiles); e4m3
 *                         spectra with e4m3 products p_k e_i, the basis rows
 *                         scaled per component by a power of two and the
 *                         dictionary by its inverse (fp8 tiles).  FP16
 *                         storage has no other type; FP32 plans ignore it.
 * Batches (fcc_batch_*) use FP16 operands. */
typedef enum {
  FCC_OPERANDS_FP16 = 0,
  FCC_OPERANDS_STORAGE = 1
} fcc_operands;

/* Problem statement of Sec. 2.  mic_xyz is copied by fcc_plan_create. */
typedef struct {
  int32_t num_mics;               /* M >= 2                                   */
  const double* mic_xyz;          /* [M][3] metres, host memory               */
  double fs;                      /* sample rate f_S, Hz, > 0                 */
  double c;                       /* speed of sound, m/s, > 0                 */
  int32_t frame_size;             /* N: power of two, 16 <= N <= 2048         */
  int32_t hop;                    /* frame advance in samples, > 0            */
  int32_t tau_max;                /* 0: ceil(d_max f_S / c) from mic_xyz      */
  int32_t rank;                   /* D in [1, I]; 0 means full rank D = I     */
  int32_t interp;                 /* r of Sec. 3: lag grid step 1/r; 1, 2, 4  */
  float alpha;                    /* eq. (1) smoothing, (0, 1]; 1 = none      */
  fcc_precision precision;
  fcc_method method;
  fcc_operands operands;          /* matrix-core operand types (above)        */
} fcc_config;

typedef struct fcc_plan_s* fcc_plan;

typedef struct {
  int32_t num_mics;               /* M                                        */
  int32_t num_pairs;              /* P = M (M - 1) / 2                        */
  int32_t frame_size;             /* N                                        */
  int32_t hop;
  int32_t num_bins;               /* F = N/2 + 1                              */
  int32_t tau_max;
  int32_t num_lags;               /* I = 2 r tau_max + 1                      */
  int32_t rank;                   /* D (FCC) or I (GCC)                       */
  int32_t rank_sym;               /* components symmetric about f = N/4       */
  int32_t rank_anti;              /* components antisymmetric about f = N/4   */
  int32_t precision;              /* fcc_precision                            */
  int32_t method;                 /* fcc_method                               */
  size_t basis_bytes;             /* size of the device plan buffer           */
  size_t spectrum_bytes_per_frame;/* M * (N/2) * (complex element size)       */
  int32_t spectrum_elem_bytes;    /* 8 (FP32), 4 (BF16/FP16), 2 (FP8)         */
  int32_t interp;                 /* r                                        */
  float alpha;
  int32_t operands;               /* fcc_operands                             */
} fcc_plan_info;

/* Validates the configuration and computes, on the host in FP64, everything a
 * geometry needs (Sec. 4, Fig. 2 "computed offline"): tau_max, the lag grid,
 * the cropped bases p_hat_k (eq. 7) and the dictionary, and the DFT
 * twiddles.  No device call is made.
 * Errors: FCC_ERR_INVALID_ARG (M < 2, non-power-of-two N, hop <= 0,
 * r tau_max >= N/4, rank outside [0, I], fs or c <= 0, interp not 1, 2 or 4,
 * alpha outside (0, 1], null pointers),
 * FCC_ERR_UNSUPPORTED (M > 32, alpha < 1 with a precision other than FP32 or
 * with method GCC, GCC with r N > 4096),
 * FCC_ERR_BASIS_AMBIGUOUS (rank cuts a cluster of singular values closer than
 * 1e-9 sigma_1, so the rank-D result is not unique). */
fcc_status fcc_plan_create(const fcc_config* config, fcc_plan* out);

void fcc_plan_destroy(fcc_plan plan);

fcc_status fcc_plan_query(fcc_plan plan, fcc_plan_info* info);

/* Copies the plan's packed tables (DFT twiddles, bases, dictionary) into
 * d_basis, a caller-owned device buffer of info.basis_bytes bytes, aligned to
 * 256 bytes.  Enqueued on `stream`; the host tables stay owned by the plan. */
fcc_status fcc_plan_upload(fcc_plan plan, void* d_basis, hipStream_t stream);

/* Number of whole frames in num_samples samples: floor((L - N) / hop) + 1,
 * or 0 when L < N (frame t covers samples [t hop, t hop + N)). */
fcc_status fcc_num_frames(fcc_plan plan, int64_t num_samples, int64_t* num_frames);

/* Bytes of workspace fcc_tdoa needs for num_frames frames: the spectra,
 * num_frames * info.spectrum_bytes_per_frame rounded up to 256, and with
 * alpha < 1 also the smoothing state and fcc_smooth_workspace_bytes. */
fcc_status fcc_workspace_bytes(fcc_plan plan, int64_t num_frames, size_t* bytes);

/* Sec. 2 front end: Hann-windowed (periodic) real DFT of every frame of every
 * microphone, each bin divided by its magnitude (per-microphone PHAT; at
 * alpha = 1, R_ij / |R_ij| = e_i e_j^* with e = X / |X|).  A bin whose squared
 * magnitude is below FLT_MIN becomes 0.  With alpha < 1 the PHAT belongs to
 * the smoothed cross-spectrum of each pair, and the raw X is written (FP32).
 *   d_x    [M][ld] FP32 audio, row m at d_x + m * ld, L samples used, ld >= L.
 *   d_spec [T][M][N/2] complex slots, interleaved (re, im), in the plan's
 *          precision ("packed real spectrum"): slot 0 holds (e(0), e(N/2)),
 *          the two real bins; slot f holds e(f) for 0 < f < N/2.
 * T = fcc_num_frames(L); T = 0 enqueues nothing. */
fcc_status fcc_spectra(fcc_plan plan, const void* d_basis, const float* d_x,
                       int64_t num_samples, int64_t ld, void* d_spec,
                       hipStream_t stream);

/* The whole path from audio: fcc_spectra into d_workspace, then
 * fcc_tdoa_from_spectra (alpha = 1) or fcc_tdoa_smoothed from R = 0
 * (alpha < 1).  d_tdoa is [T][P] int32, the lag in units of 1/r sample
 * (lag index minus r tau_max).  d_workspace holds fcc_workspace_bytes(T)
 * bytes, 256-byte aligned. */
fcc_status fcc_tdoa(fcc_plan plan, const void* d_basis, const float* d_x,
                    int64_t num_samples, int64_t ld, int32_t* d_tdoa,
                    void* d_workspace, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fcc_tdoa
 * with no workspace argument.  The spectra are staged in a static device
 * array of FCC_NOALLOC_SCRATCH_BYTES bytes that the library holds on each
 * GPU it runs on until the process ends; the frames are processed in chunks
 * of floor(FCC_NOALLOC_SCRATCH_BYTES / info.spectrum_bytes_per_frame) frames,
 * each chunk through the same kernels as fcc_tdoa, so d_tdoa equals
 * fcc_tdoa's output bit for bit.  No call allocates memory.
 *   d_x [M][ld] FP32 audio, d_tdoa [T][P] int32 (caller-owned, as fcc_tdoa).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams or threads) race and must be serialised by the caller.
 * Errors: those of fcc_tdoa; FCC_ERR_UNSUPPORTED for alpha < 1 plans (the
 * recursion's state and carries need fcc_tdoa's workspace) and for a plan
 * whose single frame of spectra exceeds FCC_NOALLOC_SCRATCH_BYTES;
 * FCC_ERR_HIP if the array's device address cannot be obtained. */
#define FCC_NOALLOC_SCRATCH_BYTES (64u << 20)
fcc_status fcc_tdoa_noalloc(fcc_plan plan, const void* d_basis, const float* d_x,
                            int64_t num_samples, int64_t ld, int32_t* d_tdoa,
                            hipStream_t stream);

/* Pairs, fold (eq. 8), projection (eq. 9), expansion 2 Re{U z} to the I lags
 * and argmax (first index on ties), from whitened spectra laid out as
 * fcc_spectra writes them; d_tdoa [T][P] int32 in units of 1/r sample.  With
 * method GCC, eq. (2) at the I lags, through an inverse FFT of r N points,
 * replaces the low-rank steps.  Plans with alpha < 1 use fcc_tdoa_smoothed
 * (FCC_ERR_UNSUPPORTED here). */
fcc_status fcc_tdoa_from_spectra(fcc_plan plan, const void* d_basis,
                                 const void* d_spec, int64_t num_frames,
                                 int32_t* d_tdoa, hipStream_t stream);

/* Same as fcc_tdoa_from_spectra, but writes the correlation itself:
 * d_y [T][P][I] FP32, lag index i <-> tau_i = i / r - tau_max.  For parity
 * checks and inspection. */
fcc_status fcc_correlation(fcc_plan plan, const void* d_basis,
                           const void* d_spec, int64_t num_frames, float* d_y,
                           hipStream_t stream);

/* The projection coefficients of eq. (9) for every pair-frame,
 * z_k = a_k + j b_k = p_hat_k . x_{s|d} (plus the centre bin for symmetric k):
 *   d_coef [T][P][2D] FP32, (a_k, b_k) interleaved, components in the order
 *   of fcc_basis_export (symmetric, antisymmetric, ...).
 * The correlation is y(tau_i) = 2 sum_k (Dc(i,k) a_k - Ds(i,k) b_k).
 * The coefficients refer to the plan's own basis (fcc_basis_export): where
 * singular values of one parity coincide, any rotation of their vectors is an
 * equally valid basis, and the planner's deterministic choice is the one used.
 * FCC method only; computed in FP32 from the spectra in any storage type. */
fcc_status fcc_coefficients(fcc_plan plan, const void* d_basis, const void* d_spec,
                            int64_t num_frames, float* d_coef, hipStream_t stream);

/* The argmax lag refined by the quadratic interpolation of Sec. 2:
 *   d_tau [T][P] FP32 samples, ((i* - r tau_max) + delta) / r with
 *   delta = (y(i*-1) - y(i*+1)) / (2 (y(i*-1) - 2 y(i*) + y(i*+1))),
 *   and delta = 0 when i* is at either end of the lag window or the
 *   denominator is 0.  FCC method only. */
fcc_status fcc_tdoa_parabolic(fcc_plan plan, const void* d_basis, const void* d_spec,
                              int64_t num_frames, float* d_tau, hipStream_t stream);

/* Host copies of the FP64 basis (Sec. 4), for inspection and tests.  Any
 * pointer may be NULL.  Order of components: symmetric, antisymmetric,
 * symmetric, ... (eq. 6).
 *   sigma [D], is_sym [D], p_hat [D][N/4+1] (eq. 7 rows, sigma included),
 *   dc, ds [I][D] real and imaginary parts of the dictionary U. */
fcc_status fcc_basis_export(fcc_plan plan, double* sigma, int32_t* is_sym,
                            double* p_hat, double* dc, double* ds);

/* ---- recursive smoothing, alpha < 1 ----------------------------------------
 * Eq. (1): R(t, f) = (1 - alpha) R(t - 1, f) + alpha X_i(t, f) X_j(t, f)^*
 * per pair and bin, then R / |R| (0 when |R|^2 < FLT_MIN), fold, projection,
 * expansion and argmax as above.  The recursion runs over the frames of the
 * call in order:
 *   d_spec     [T][M][N/2] raw spectra as fcc_spectra writes them for the plan;
 *   d_state    [P][N/2 + 1] complex FP32 (interleaved), bins in natural order:
 *              R before the first frame on entry (zeros for a new stream), R
 *              after the last frame on return, so consecutive calls continue
 *              one recursion;
 *   d_tdoa     [T][P] int32 lag in units of 1/r sample, or NULL;
 *   d_tau      [T][P] FP32 interpolated lag in samples (as fcc_tdoa_parabolic),
 *              or NULL;
 *   d_y        [T][P][I] FP32 correlation, or NULL (at least one output);
 *   d_workspace fcc_smooth_workspace_bytes(T) bytes, caller-owned.
 * Limits: rank <= 32, I <= 80 (FCC_ERR_UNSUPPORTED otherwise).  The state
 * buffer is read and written by the call: calls sharing it must be ordered. */
fcc_status fcc_smooth_workspace_bytes(fcc_plan plan, int64_t num_frames, size_t* bytes);
fcc_status fcc_tdoa_smoothed(fcc_plan plan, const void* d_basis, const void* d_spec, int64_t num_frames,
                             float* d_state, int32_t* d_tdoa, float* d_tau, float* d_y,
                             void* d_workspace, hipStream_t stream);

/* ---- direction of arrival ---------------------------------------------------
 * Sec. 6 names the next step: the TDoAs of every pair of an array feeding a
 * search over direction candidates.  For unit directions u_g the far-field
 * TDoA of pair (i, j) is tau = (r_j - r_i) . u_g f_S / c samples (the sign
 * convention of d_tdoa), at fractional lag index
 *   q[p][g] = clamp(r tau + r tau_max, 0, I - 1)
 * on the correlation's grid.  fcc_doa_table computes q on the host in FP64
 * (dirs [G][3] unit vectors and table [P][G] FP32, both host memory owned by
 * the caller).  fcc_doa scores every direction by the sum
 * over pairs of y at q[p][g], interpolated linearly between neighbouring
 * lags, from d_y [T][P][I] (fcc_correlation or fcc_tdoa_smoothed) and the
 * table copied to the device (d_table [P][G]); d_doa [T] int32 receives the
 * first direction of largest score and d_score [T][G] FP32 (may be NULL) the
 * scores.  FCC_ERR_UNSUPPORTED when one frame's correlations exceed 48 KB. */
fcc_status fcc_doa_table(fcc_plan plan, const double* dirs, int32_t num_dirs, float* table);
fcc_status fcc_doa(fcc_plan plan, const float* d_y, int64_t num_frames, const float* d_table, int32_t num_dirs,
                   int32_t* d_doa, float* d_score, hipStream_t stream);

/* ---- batches of independent arrays ------------------------------------------
 * Many arrays of uneven microphone count, aperture, sample rate, frame size and
 * rank (each with its own plan) in one pass: the front end of every array in
 * one launch per frame size present (one workgroup per block of transforms),
 * and the pair stage of every array in one persistent launch per class of
 * arrays sharing a matrix-core tile shape, each workgroup taking one
 * contiguous run of the class's frames.  With use_graph the pass is captured
 * once into a graph (per set of buffer pointers) and replayed.
 * fcc_batch_tune times candidate pair-stage launch shapes on the given buffers
 * and keeps the fastest.
 * Limits: every plan FP16 or BF16 storage (the same), method FCC, alpha = 1,
 * M <= 16, N >= 32, I <= 48, rank <= 32, and a class's tables plus two
 * wavefront slabs within 160 KB of LDS (FCC_ERR_UNSUPPORTED otherwise; e.g.
 * N = 1024 with rank 32 and I > 32 exceeds it).
 * Plans are copied; num_samples[a] fixes array a's length L_a at creation.
 * An array shorter than its frame size has no frames (T_a = 0) and no output;
 * when no array has a frame, fcc_batch_tdoa and fcc_batch_tune do nothing.
 * Buffers (caller-owned, device):
 *   d_image     info.image_bytes, 256-byte aligned, filled by fcc_batch_upload;
 *   d_audio     info.audio_floats FP32: array a's [M_a][L_a] block (row stride
 *               L_a) at offset audio_offset[a] (fcc_batch_layout);
 *   d_tdoa      info.tdoa_count int32: array a's [T_a][P_a] lags (units of 1/r
 *               sample) at offset tdoa_offset[a];
 *   d_workspace info.workspace_bytes, 256-byte aligned (the spectra of every array).
 * A batch object is not thread-safe (tuning and the graph cache mutate it);
 * calls that share a workspace must be ordered. */
typedef struct fcc_batch_s* fcc_batch;
typedef struct {
  int32_t num_arrays;
  int32_t num_classes;            /* pair-stage launches per pass             */
  size_t image_bytes;
  size_t workspace_bytes;
  int64_t audio_floats;
  int64_t tdoa_count;
} fcc_batch_info;
fcc_status fcc_batch_create(const fcc_plan* plans, int32_t num_arrays, const int64_t* num_samples, fcc_batch* out);
void fcc_batch_destroy(fcc_batch batch);
fcc_status fcc_batch_query(fcc_batch batch, fcc_batch_info* info);
/* Host arrays of num_arrays entries; any may be NULL. */
fcc_status fcc_batch_layout(fcc_batch batch, int64_t* audio_offset, int64_t* tdoa_offset, int64_t* num_frames);
fcc_status fcc_batch_upload(fcc_batch batch, void* d_image, hipStream_t stream);
fcc_status fcc_batch_tdoa(fcc_batch batch, const void* d_image, const float* d_audio, int32_t* d_tdoa,
                          void* d_workspace, int32_t use_graph, hipStream_t stream);
/* Autotuner; synchronises `stream` while timing.  Overwrites d_tdoa. */
fcc_status fcc_batch_tune(fcc_batch batch, const void* d_image, const float* d_audio, int32_t* d_tdoa,
                          void* d_workspace, hipStream_t stream);
/* The launch shapes in use: values[0] the number of front-end launches (frame
 * sizes present), values[1] 0, then per class (workgroups launched, wavefronts
 * per workgroup, workgroups per compute unit asked for); capacity >=
 * 2 + 3 num_classes. */
fcc_status fcc_batch_tuning(fcc_batch batch, int32_t* values, int32_t capacity);

/* ---- learned sub-sample TDoA ------------------------------------------------
 * Not from the paper: a multilayer perceptron refining the FCC lag of one
 * pair-frame from its projection coefficients (fcc_coefficients).  One row =
 * one pair-frame, c = (a_1, b_1, ..., a_D, b_D), in_dim = 2D.
 *   u = c / ||c||_2,  h1 = gelu(u W1 + b1),  h2 = gelu(h1 W2 + b2),
 *   (mu, s) = h2 W3 + b3,  s clipped to [-8, 8]
 * mu is the TDoA in samples, s the log-variance of a Gaussian error model
 * (confidence exp(-s/2)); gelu is the tanh form.  Matrix products run on FP16
 * matrix cores with FP32 accumulation; everything else is FP32.
 * Parameters: one FP32 vector, W1 [in_dim][hidden], b1 [hidden],
 * W2 [hidden][hidden], b2 [hidden], W3 [hidden][2], b3 [2], row-major.
 * in_dim in [1, 64], hidden a multiple of 16 in [16, 512]; rows < 2^31.
 * Workspace: fcc_mlp_workspace_bytes, caller-owned. */
size_t fcc_mlp_num_params(int32_t in_dim, int32_t hidden);
fcc_status fcc_mlp_workspace_bytes(int32_t in_dim, int32_t hidden, int64_t rows, size_t* bytes);

/* d_coef [rows][in_dim] -> d_out [rows][2] = (mu, s).  For in_dim <= 64 and
 * hidden 32, 64 or 128 one fused kernel keeps the hidden layers on chip (the
 * workspace is then unused); other shapes run layer by layer. */
fcc_status fcc_mlp_forward(const float* d_params, int32_t in_dim, int32_t hidden, const float* d_coef,
                           int64_t rows, float* d_out, void* d_workspace, hipStream_t stream);

/* Forward plus the gradient of the mean Gaussian negative log-likelihood
 * L = (1/rows) sum 0.5 (exp(-s) (mu - target)^2 + s) into d_grad (parameter
 * layout, overwritten); the summed (not averaged) loss is ADDED to
 * *d_loss_sum (one FP32 on the device); d_out receives (mu, s). */
fcc_status fcc_mlp_backward(const float* d_params, int32_t in_dim, int32_t hidden, const float* d_coef,
                            const float* d_target, int64_t rows, float* d_grad, float* d_loss_sum,
                            float* d_out, void* d_workspace, hipStream_t stream);

/* One Adam update (bias-corrected, step >= 1) of n parameters in place. */
fcc_status fcc_mlp_adam(float* d_params, float* d_m, float* d_v, const float* d_grad, int64_t n, float lr,
                        float beta1, float beta2, float eps, int32_t step, hipStream_t stream);

/* The learned estimate for every pair-frame of a plan, in one call:
 * coefficients (fcc_coefficients) -> MLP (in_dim = 2 * rank) -> (mu, s);
 * d_tau [T][P] FP32 samples is mu where the confidence exp(-s/2) is at least
 * min_confidence, and the interpolated FCC lag (fcc_tdoa_parabolic)
 * elsewhere; d_confidence [T][P] (may be NULL) receives exp(-s/2).
 * min_confidence = +inf gives plain FCC with interpolation, 0 the MLP alone.
 * Workspace: fcc_learned_workspace_bytes, caller-owned, 256-byte aligned.
 * FCC method only. */
fcc_status fcc_learned_workspace_bytes(fcc_plan plan, int32_t hidden, int64_t num_frames, size_t* bytes);
fcc_status fcc_tdoa_learned(fcc_plan plan, const void* d_basis, const void* d_spec, int64_t num_frames,
                            const float* d_params, int32_t hidden, float min_confidence, float* d_tau,
                            float* d_confidence, void* d_workspace, hipStream_t stream);

const char* fcc_status_string(fcc_status status);
const char* fcc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FCC_H_ */
