// C ABI of the FCC library: plan lifecycle, argument checks and dispatch.
// The contract of every entry point is documented in include/fcc.h.
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <tuple>
#include <map>
#include <new>
#include <string>

#include "fcc.h"
#include "kernels.hpp"
#include "plan.hpp"

struct fcc_plan_s {
  fcc::Plan p;
};

// A batch of independent arrays: copies of their plans, the layout of their
// inputs and outputs, the work classes, the tuned tile shapes and the cached
// graph of one pass.
struct fcc_batch_s {
  std::vector<fcc::Plan> plans;
  std::vector<fcc::BatchArray> arrays;
  std::vector<int32_t> members;
  std::vector<fcc::BatchClass> classes;
  std::vector<unsigned char> image;
  size_t arrays_off = 0, members_off = 0, items_off = 0;
  int64_t audio_floats = 0, tdoa_count = 0, stft_items = 0;
  size_t spec_bytes = 0, workspace_bytes = 0;
  std::vector<fcc::BatchStftRange> stft_ranges;   // front-end items, grouped by frame size
  std::vector<int32_t> item_array;                // array of every front-end item
  fcc_precision precision = FCC_FP16;
  std::vector<fcc::PairTuning> pair_tuning;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* graph_key[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace {

thread_local std::string g_last_error;

fcc_status set_error(fcc_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

fcc_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return FCC_OK;
  return set_error(FCC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Test hook (environment variable FCC_FAULT, read at every call):
//   launch  every device launch or copy fails with FCC_ERR_HIP on the host,
//           before anything is enqueued;
//   alloc   the host allocations of plans and batches fail (FCC_ERR_INTERNAL).
enum class Fault { kNone, kLaunch, kAlloc };
Fault fault_mode() {
  const char* v = std::getenv("FCC_FAULT");
  if (!v) return Fault::kNone;
  if (std::strcmp(v, "launch") == 0) return Fault::kLaunch;
  if (std::strcmp(v, "alloc") == 0) return Fault::kAlloc;
  return Fault::kNone;
}
fcc_status injected_launch_fault(const char* what) {
  if (fault_mode() != Fault::kLaunch) return FCC_OK;
  return set_error(FCC_ERR_HIP, std::string(what) + ": injected launch failure (FCC_FAULT=launch)");
}
bool injected_alloc_fault() { return fault_mode() == Fault::kAlloc; }

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int64_t frames_of(const fcc::Plan& p, int64_t L) {
  if (L < p.N) return 0;
  return (L - p.N) / p.hop + 1;
}

const unsigned char* image_ptr(const void* d_basis, size_t off) {
  return static_cast<const unsigned char*>(d_basis) + off;
}

fcc_status check_basis(const void* d_basis) {
  if (!d_basis) return set_error(FCC_ERR_INVALID_ARG, "d_basis is NULL");
  if (!aligned(d_basis, 256)) return set_error(FCC_ERR_INVALID_ARG, "d_basis must be 256-byte aligned");
  return FCC_OK;
}

fcc_status check_spec(const fcc::Plan& p, const void* d_spec) {
  if (!d_spec) return set_error(FCC_ERR_INVALID_ARG, "spectrum pointer is NULL");
  if (!aligned(d_spec, size_t(p.spec_elem))) return set_error(FCC_ERR_INVALID_ARG, "spectrum pointer misaligned");
  return FCC_OK;
}

fcc::PairArgs pair_args(const fcc::Plan& p, const void* d_basis, const void* d_spec, int64_t T,
                        hipStream_t stream) {
  fcc::PairArgs a{};
  a.spec = d_spec;
  a.T = T;
  a.M = p.M;
  a.P = p.P;
  a.N = p.N;
  a.I = p.I;
  a.D = p.D;
  a.lag0 = p.r * p.tau_max;
  a.r = p.r;
  a.precision = p.precision;
  a.method = p.method;
  a.pairs = reinterpret_cast<const uint8_t*>(image_ptr(d_basis, p.layout.pairs));
  a.basis32 = reinterpret_cast<const float*>(image_ptr(d_basis, p.layout.basis32));
  a.dict = reinterpret_cast<const float*>(image_ptr(d_basis, p.layout.dict));
  a.lagw = reinterpret_cast<const float2*>(image_ptr(d_basis, p.layout.lagw));
  a.Dpad = p.Dpad;
  a.prow16 = image_ptr(d_basis, p.layout.prow16);
  a.prow32 = reinterpret_cast<const float2*>(image_ptr(d_basis, p.layout.prow32));
  a.gexp = reinterpret_cast<const float*>(image_ptr(d_basis, p.layout.gexp));
  a.operands = p.operands;
  a.prow_op = image_ptr(d_basis, p.layout.prow_op);
  a.gexp_op = reinterpret_cast<const float*>(image_ptr(d_basis, p.layout.gexp_op));
  a.Dfold = p.Dfold;
  a.pfold = reinterpret_cast<const float*>(image_ptr(d_basis, p.layout.pfold));
  a.twiddle_r = reinterpret_cast<const float2*>(image_ptr(d_basis, p.layout.twiddle_r));
  a.stream = stream;
  return a;
}

fcc_status run_spectra(const fcc::Plan& p, const void* d_basis, const float* d_x, int64_t L,
                       int64_t ld, void* d_spec, hipStream_t stream) {
  fcc::StftArgs a{};
  a.x = d_x;
  a.ld = ld;
  a.T = frames_of(p, L);
  a.M = p.M;
  a.N = p.N;
  a.hop = p.hop;
  a.precision = p.precision;
  a.twiddle = reinterpret_cast<const float2*>(image_ptr(d_basis, p.layout.twiddle));
  a.out = d_spec;
  a.raw = p.alpha < 1.0f;                    // smoothing needs X itself; PHAT comes per pair
  a.stream = stream;
  if (fcc_status f = injected_launch_fault("stft_phat launch")) return f;
  return hip_status(fcc::launch_stft_phat(a), "stft_phat launch");
}

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

// fcc_tdoa's workspace: the spectra, and with smoothing the state and the
// chunk carries
struct TdoaWorkspace {
  size_t spec, state, scratch, total;
};
TdoaWorkspace tdoa_workspace(const fcc::Plan& p, int64_t T) {
  TdoaWorkspace w{};
  w.spec = 0;
  w.state = up256(size_t(T) * p.M * (p.N / 2) * p.spec_elem);
  w.scratch = w.state;
  w.total = w.state;
  if (p.alpha < 1.0f && T > 0) {
    w.scratch = w.state + up256(sizeof(float) * 2 * size_t(p.P) * p.F);
    w.total = w.scratch + up256(fcc::smooth_scratch_bytes(T, p.P, p.N));
  }
  return w;
}

fcc_status check_audio(const fcc::Plan& p, const float* d_x, int64_t L, int64_t ld) {
  if (L < 0) return set_error(FCC_ERR_INVALID_ARG, "num_samples must be >= 0");
  if (ld < L || ld <= 0) return set_error(FCC_ERR_INVALID_ARG, "ld must be >= num_samples and > 0");
  if (frames_of(p, L) > 0 && !d_x) return set_error(FCC_ERR_INVALID_ARG, "d_x is NULL");
  if (!aligned(d_x, 4)) return set_error(FCC_ERR_INVALID_ARG, "d_x misaligned");
  if (frames_of(p, L) * int64_t(p.M) > int64_t(INT32_MAX))
    return set_error(FCC_ERR_UNSUPPORTED, "too many frames for one call");
  return FCC_OK;
}

}  // namespace

extern "C" {

fcc_status fcc_plan_create(const fcc_config* config, fcc_plan* out) {
  if (!config || !out) return set_error(FCC_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  fcc_plan_s* h = injected_alloc_fault() ? nullptr : new (std::nothrow) fcc_plan_s;
  if (!h) return set_error(FCC_ERR_INTERNAL, "out of host memory");
  std::string err;
  fcc_status st;
  try {
    st = fcc::build_plan(*config, h->p, err);
  } catch (...) {
    st = FCC_ERR_INTERNAL;
    err = "exception while building the plan";
  }
  if (st != FCC_OK) {
    delete h;
    return set_error(st, err);
  }
  *out = h;
  return FCC_OK;
}

void fcc_plan_destroy(fcc_plan plan) { delete plan; }

fcc_status fcc_plan_query(fcc_plan plan, fcc_plan_info* info) {
  if (!plan || !info) return set_error(FCC_ERR_INVALID_ARG, "NULL argument");
  const fcc::Plan& p = plan->p;
  info->num_mics = p.M;
  info->num_pairs = p.P;
  info->frame_size = p.N;
  info->hop = p.hop;
  info->num_bins = p.F;
  info->tau_max = p.tau_max;
  info->num_lags = p.I;
  info->rank = p.D;
  info->rank_sym = p.Ds;
  info->rank_anti = p.Da;
  info->precision = p.precision;
  info->method = p.method;
  info->basis_bytes = p.layout.total;
  info->spectrum_bytes_per_frame = size_t(p.M) * (p.N / 2) * p.spec_elem;
  info->spectrum_elem_bytes = p.spec_elem;
  info->interp = p.r;
  info->alpha = p.alpha;
  info->operands = p.operands;
  return FCC_OK;
}

fcc_status fcc_plan_upload(fcc_plan plan, void* d_basis, hipStream_t stream) {
  if (!plan) return set_error(FCC_ERR_INVALID_ARG, "NULL plan");
  fcc_status st = check_basis(d_basis);
  if (st != FCC_OK) return st;
  const fcc::Plan& p = plan->p;
  if (fcc_status f = injected_launch_fault("plan upload")) return f;
  return hip_status(hipMemcpyAsync(d_basis, p.image.data(), p.image.size(), hipMemcpyHostToDevice, stream),
                    "plan upload");
}

fcc_status fcc_num_frames(fcc_plan plan, int64_t num_samples, int64_t* num_frames) {
  if (!plan || !num_frames) return set_error(FCC_ERR_INVALID_ARG, "NULL argument");
  if (num_samples < 0) return set_error(FCC_ERR_INVALID_ARG, "num_samples must be >= 0");
  *num_frames = frames_of(plan->p, num_samples);
  return FCC_OK;
}

fcc_status fcc_workspace_bytes(fcc_plan plan, int64_t num_frames, size_t* bytes) {
  if (!plan || !bytes) return set_error(FCC_ERR_INVALID_ARG, "NULL argument");
  if (num_frames < 0) return set_error(FCC_ERR_INVALID_ARG, "num_frames must be >= 0");
  const fcc::Plan& p = plan->p;
  *bytes = tdoa_workspace(p, num_frames).total;
  return FCC_OK;
}

fcc_status fcc_spectra(fcc_plan plan, const void* d_basis, const float* d_x, int64_t num_samples,
                       int64_t ld, void* d_spec, hipStream_t stream) {
  if (!plan) return set_error(FCC_ERR_INVALID_ARG, "NULL plan");
  const fcc::Plan& p = plan->p;
  fcc_status st = check_basis(d_basis);
  if (st == FCC_OK) st = check_audio(p, d_x, num_samples, ld);
  if (st != FCC_OK) return st;
  if (frames_of(p, num_samples) == 0) return FCC_OK;
  if ((st = check_spec(p, d_spec)) != FCC_OK) return st;
  return run_spectra(p, d_basis, d_x, num_samples, ld, d_spec, stream);
}

static fcc_status pair_stage(const fcc::Plan& p, const void* d_basis, const void* d_spec, int64_t T,
                             int32_t* d_tdoa, float* d_y, hipStream_t stream, float* d_coef = nullptr,
                             float* d_tau = nullptr) {
  if (T < 0) return set_error(FCC_ERR_INVALID_ARG, "num_frames must be >= 0");
  fcc_status st = check_basis(d_basis);
  if (st != FCC_OK) return st;
  if (p.alpha < 1.0f)
    return set_error(FCC_ERR_UNSUPPORTED, "with alpha < 1 the pair stage is fcc_tdoa_smoothed");
  if (T == 0) return FCC_OK;
  if ((st = check_spec(p, d_spec)) != FCC_OK) return st;
  if (!d_tdoa && !d_y && !d_coef && !d_tau) return set_error(FCC_ERR_INVALID_ARG, "output pointer is NULL");
  for (const void* o : {static_cast<const void*>(d_tdoa), static_cast<const void*>(d_y),
                        static_cast<const void*>(d_coef), static_cast<const void*>(d_tau)})
    if (o && !aligned(o, 4)) return set_error(FCC_ERR_INVALID_ARG, "output pointer misaligned");
  if (T > int64_t(INT32_MAX)) return set_error(FCC_ERR_UNSUPPORTED, "too many frames for one call");
  fcc::PairArgs a = pair_args(p, d_basis, d_spec, T, stream);
  a.tdoa = d_tdoa;
  a.y = d_y;
  a.coef = d_coef;
  a.tau_frac = d_tau;
  if (fcc_status f = injected_launch_fault("pair kernel launch")) return f;
  hipError_t e;
  if (d_coef || d_tau) {
    if (p.method != FCC_METHOD_FCC) return set_error(FCC_ERR_UNSUPPORTED, "coefficients and interpolation need the FCC method");
    if (!fcc::pair_fold32_supported(a)) return set_error(FCC_ERR_UNSUPPORTED, "shape outside the fold kernel's limits");
    e = fcc::launch_pair_fold32(a);
  } else if (fcc::gcc_ifft_supported(a)) e = fcc::launch_gcc_ifft(a);
  else if (fcc::pair_mfma_supported(a)) e = fcc::launch_pair_mfma(a);
  // FP32 spectra take the fold kernel; 16-bit and 8-bit spectra the direct
  // form, unless its lag registers cannot hold the window (I > 64)
  else if (fcc::pair_fold32_supported(a) && (p.precision == FCC_FP32 || !fcc::pair_valu_supported(a)))
    e = fcc::launch_pair_fold32(a);
  else e = fcc::launch_pair_valu(a);
  if (e == hipErrorInvalidValue)
    return set_error(FCC_ERR_UNSUPPORTED, "shape outside the pair kernel's limits");
  return hip_status(e, "pair kernel launch");
}

static fcc_status smooth_stage(const fcc::Plan& p, const void* d_basis, const void* d_spec, int64_t T,
                               float* d_state, int32_t* d_tdoa, float* d_tau, float* d_y, void* d_workspace,
                               hipStream_t stream) {
  if (T < 0) return set_error(FCC_ERR_INVALID_ARG, "num_frames must be >= 0");
  if (p.alpha >= 1.0f) return set_error(FCC_ERR_INVALID_ARG, "the plan has alpha = 1: use fcc_tdoa_from_spectra");
  fcc_status st = check_basis(d_basis);
  if (st != FCC_OK) return st;
  if (T == 0) return FCC_OK;
  if ((st = check_spec(p, d_spec)) != FCC_OK) return st;
  if (!d_state || !d_workspace) return set_error(FCC_ERR_INVALID_ARG, "d_state or d_workspace is NULL");
  if (!d_tdoa && !d_tau && !d_y) return set_error(FCC_ERR_INVALID_ARG, "output pointer is NULL");
  for (const void* o : {static_cast<const void*>(d_state), static_cast<const void*>(d_tdoa),
                        static_cast<const void*>(d_tau), static_cast<const void*>(d_y), static_cast<const void*>(d_workspace)})
    if (o && !aligned(o, 8)) return set_error(FCC_ERR_INVALID_ARG, "pointer misaligned");
  if (T > int64_t(INT32_MAX)) return set_error(FCC_ERR_UNSUPPORTED, "too many frames for one call");
  fcc::SmoothArgs a{};
  a.spec = static_cast<const float2*>(d_spec);
  a.T = T;
  a.M = p.M;
  a.P = p.P;
  a.N = p.N;
  a.I = p.I;
  a.D = p.D;
  a.Dfold = p.Dfold;
  a.lag0 = p.r * p.tau_max;
  a.r = p.r;
  a.alpha = p.alpha;
  a.pairs = reinterpret_cast<const uint8_t*>(image_ptr(d_basis, p.layout.pairs));
  a.pfold = reinterpret_cast<const float*>(image_ptr(d_basis, p.layout.pfold));
  a.dict = reinterpret_cast<const float*>(image_ptr(d_basis, p.layout.dict));
  a.state = reinterpret_cast<float2*>(d_state);
  a.scratch = static_cast<float2*>(d_workspace);
  a.tdoa = d_tdoa;
  a.tau = d_tau;
  a.y = d_y;
  a.stream = stream;
  if (!fcc::smooth_supported(a))
    return set_error(FCC_ERR_UNSUPPORTED, "shape outside the smoothing kernel's limits (rank <= 32, I <= 80)");
  if (fcc_status f = injected_launch_fault("smoothing kernels launch")) return f;
  return hip_status(fcc::launch_smooth(a), "smoothing kernels launch");
}

fcc_status fcc_tdoa_from_spectra(fcc_plan plan, const void* d_basis, const void* d_spec,
                                 int64_t num_frames, int32_t* d_tdoa, hipStream_t stream) {
  if (!plan) return set_error(FCC_ERR_INVALID_ARG, "NULL plan");
  if (num_frames > 0 && !d_tdoa) return set_error(FCC_ERR_INVALID_ARG, "d_tdoa is NULL");
  return pair_stage(plan->p, d_basis, d_spec, num_frames, d_tdoa, nullptr, stream);
}

fcc_status fcc_correlation(fcc_plan plan, const void* d_basis, const void* d_spec, int64_t num_frames,
                           float* d_y, hipStream_t stream) {
  if (!plan) return set_error(FCC_ERR_INVALID_ARG, "NULL plan");
  if (num_frames > 0 && !d_y) return set_error(FCC_ERR_INVALID_ARG, "d_y is NULL");
  return pair_stage(plan->p, d_basis, d_spec, num_frames, nullptr, d_y, stream);
}

fcc_status fcc_coefficients(fcc_plan plan, const void* d_basis, const void* d_spec, int64_t num_frames,
                            float* d_coef, hipStream_t stream) {
  if (!plan) return set_error(FCC_ERR_INVALID_ARG, "NULL plan");
  if (num_frames > 0 && !d_coef) return set_error(FCC_ERR_INVALID_ARG, "d_coef is NULL");
  return pair_stage(plan->p, d_basis, d_spec, num_frames, nullptr, nullptr, stream, d_coef, nullptr);
}

fcc_status fcc_tdoa_parabolic(fcc_plan plan, const void* d_basis, const void* d_spec, int64_t num_frames,
                              float* d_tau, hipStream_t stream) {
  if (!plan) return set_error(FCC_ERR_INVALID_ARG, "NULL plan");
  if (num_frames > 0 && !d_tau) return set_error(FCC_ERR_INVALID_ARG, "d_tau is NULL");
  return pair_stage(plan->p, d_basis, d_spec, num_frames, nullptr, nullptr, stream, nullptr, d_tau);
}

fcc_status fcc_tdoa(fcc_plan plan, const void* d_basis, const float* d_x, int64_t num_samples, int64_t ld,
                    int32_t* d_tdoa, void* d_workspace, hipStream_t stream) {
  if (!plan) return set_error(FCC_ERR_INVALID_ARG, "NULL plan");
  const fcc::Plan& p = plan->p;
  fcc_status st = check_basis(d_basis);
  if (st == FCC_OK) st = check_audio(p, d_x, num_samples, ld);
  if (st != FCC_OK) return st;
  const int64_t T = frames_of(p, num_samples);
  if (T == 0) return FCC_OK;
  if (!d_tdoa) return set_error(FCC_ERR_INVALID_ARG, "d_tdoa is NULL");
  if (!d_workspace) return set_error(FCC_ERR_INVALID_ARG, "d_workspace is NULL");
  if ((st = check_spec(p, d_workspace)) != FCC_OK) return st;
  if ((st = run_spectra(p, d_basis, d_x, num_samples, ld, d_workspace, stream)) != FCC_OK) return st;
  if (p.alpha < 1.0f) {
    // one recursion over the whole recording, from R = 0
    const TdoaWorkspace w = tdoa_workspace(p, T);
    char* ws = static_cast<char*>(d_workspace);
    float* state = reinterpret_cast<float*>(ws + w.state);
    if (fcc_status f = injected_launch_fault("fill launch")) return f;
    if ((st = hip_status(fcc::launch_fill_zero(state, 2 * int64_t(p.P) * p.F, stream), "fill launch")) != FCC_OK)
      return st;
    return smooth_stage(p, d_basis, d_workspace, T, state, d_tdoa, nullptr, nullptr, ws + w.scratch, stream);
  }
  return pair_stage(p, d_basis, d_workspace, T, d_tdoa, nullptr, stream);
}

fcc_status fcc_tdoa_noalloc(fcc_plan plan, const void* d_basis, const float* d_x, int64_t num_samples,
                            int64_t ld, int32_t* d_tdoa, hipStream_t stream) {
  if (!plan) return set_error(FCC_ERR_INVALID_ARG, "NULL plan");
  const fcc::Plan& p = plan->p;
  fcc_status st = check_basis(d_basis);
  if (st == FCC_OK) st = check_audio(p, d_x, num_samples, ld);
  if (st != FCC_OK) return st;
  if (p.alpha < 1.0f)
    return set_error(FCC_ERR_UNSUPPORTED, "alpha < 1 needs fcc_tdoa's workspace for the recursion");
  const int64_t T = frames_of(p, num_samples);
  if (T == 0) return FCC_OK;
  if (!d_tdoa) return set_error(FCC_ERR_INVALID_ARG, "d_tdoa is NULL");
  if (!aligned(d_tdoa, 4)) return set_error(FCC_ERR_INVALID_ARG, "d_tdoa misaligned");
  const size_t frame_bytes = size_t(p.M) * (p.N / 2) * p.spec_elem;
  if (frame_bytes > size_t(FCC_NOALLOC_SCRATCH_BYTES))
    return set_error(FCC_ERR_UNSUPPORTED, "one frame of spectra exceeds FCC_NOALLOC_SCRATCH_BYTES");
  if (fcc_status f = injected_launch_fault("noalloc launch")) return f;
  void* scratch = nullptr;
  if ((st = hip_status(fcc::noalloc_scratch(&scratch), "static scratch address")) != FCC_OK) return st;
  const int64_t chunk = int64_t(size_t(FCC_NOALLOC_SCRATCH_BYTES) / frame_bytes);
  for (int64_t t0 = 0; t0 < T; t0 += chunk) {
    const int64_t tc = T - t0 < chunk ? T - t0 : chunk;
    const int64_t Lc = (tc - 1) * p.hop + p.N;             // exactly tc frames
    if ((st = run_spectra(p, d_basis, d_x + t0 * p.hop, Lc, ld, scratch, stream)) != FCC_OK) return st;
    if ((st = pair_stage(p, d_basis, scratch, tc, d_tdoa + t0 * p.P, nullptr, stream)) != FCC_OK) return st;
  }
  return FCC_OK;
}

fcc_status fcc_smooth_workspace_bytes(fcc_plan plan, int64_t num_frames, size_t* bytes) {
  if (!plan || !bytes) return set_error(FCC_ERR_INVALID_ARG, "NULL argument");
  if (num_frames < 0) return set_error(FCC_ERR_INVALID_ARG, "num_frames must be >= 0");
  *bytes = up256(fcc::smooth_scratch_bytes(num_frames, plan->p.P, plan->p.N));
  return FCC_OK;
}

fcc_status fcc_tdoa_smoothed(fcc_plan plan, const void* d_basis, const void* d_spec, int64_t num_frames,
                             float* d_state, int32_t* d_tdoa, float* d_tau, float* d_y, void* d_workspace,
                             hipStream_t stream) {
  if (!plan) return set_error(FCC_ERR_INVALID_ARG, "NULL plan");
  return smooth_stage(plan->p, d_basis, d_spec, num_frames, d_state, d_tdoa, d_tau, d_y, d_workspace, stream);
}

fcc_status fcc_basis_export(fcc_plan plan, double* sigma, int32_t* is_sym, double* p_hat, double* dc,
                            double* ds) {
  if (!plan) return set_error(FCC_ERR_INVALID_ARG, "NULL plan");
  const fcc::Plan& p = plan->p;
  if (sigma) std::memcpy(sigma, p.sigma.data(), sizeof(double) * p.sigma.size());
  if (is_sym) std::memcpy(is_sym, p.is_sym.data(), sizeof(int32_t) * p.is_sym.size());
  if (p_hat) std::memcpy(p_hat, p.p_hat.data(), sizeof(double) * p.p_hat.size());
  if (dc) std::memcpy(dc, p.dc.data(), sizeof(double) * p.dc.size());
  if (ds) std::memcpy(ds, p.ds.data(), sizeof(double) * p.ds.size());
  return FCC_OK;
}

static fcc_status check_mlp_shape(int32_t in_dim, int32_t hidden, int64_t rows) {
  if (in_dim < 1 || in_dim > 64) return set_error(FCC_ERR_INVALID_ARG, "in_dim must be in [1, 64]");
  if (hidden < 16 || hidden > 512 || hidden % 16) return set_error(FCC_ERR_INVALID_ARG, "hidden must be a multiple of 16 in [16, 512]");
  if (rows < 0 || rows >= (int64_t(1) << 31)) return set_error(FCC_ERR_INVALID_ARG, "rows must be in [0, 2^31)");
  return FCC_OK;
}

size_t fcc_mlp_num_params(int32_t in_dim, int32_t hidden) {
  if (in_dim < 1 || hidden < 1) return 0;
  return fcc::mlp_num_params(in_dim, hidden);
}

fcc_status fcc_mlp_workspace_bytes(int32_t in_dim, int32_t hidden, int64_t rows, size_t* bytes) {
  if (!bytes) return set_error(FCC_ERR_INVALID_ARG, "NULL argument");
  fcc_status st = check_mlp_shape(in_dim, hidden, rows);
  if (st != FCC_OK) return st;
  *bytes = sizeof(float) * fcc::mlp_workspace_floats(in_dim, hidden, rows);
  return FCC_OK;
}

fcc_status fcc_mlp_forward(const float* d_params, int32_t in_dim, int32_t hidden, const float* d_coef,
                           int64_t rows, float* d_out, void* d_workspace, hipStream_t stream) {
  fcc_status st = check_mlp_shape(in_dim, hidden, rows);
  if (st != FCC_OK) return st;
  if (rows == 0) return FCC_OK;
  if (!d_params || !d_coef || !d_out || !d_workspace) return set_error(FCC_ERR_INVALID_ARG, "NULL pointer");
if (fcc_status f = injected_launch_fault("mlp forward launch")) return f;
  if (fcc::mlp_fused_supported(in_dim, hidden))
    return hip_status(fcc::mlp_infer(d_params, in_dim, hidden, d_coef, rows, d_out, stream), "fused mlp launch");
  return hip_status(fcc::mlp_forward(d_params, in_dim, hidden, d_coef, rows, d_out, d_workspace, stream),
                    "mlp forward launch");
}

fcc_status fcc_mlp_backward(const float* d_params, int32_t in_dim, int32_t hidden, const float* d_coef,
                            const float* d_target, int64_t rows, float* d_grad, float* d_loss_sum,
                            float* d_out, void* d_workspace, hipStream_t stream) {
  fcc_status st = check_mlp_shape(in_dim, hidden, rows);
  if (st != FCC_OK) return st;
  if (rows == 0) return FCC_OK;
  if (!d_params || !d_coef || !d_target || !d_grad || !d_loss_sum || !d_out || !d_workspace)
    return set_error(FCC_ERR_INVALID_ARG, "NULL pointer");
if (fcc_status f = injected_launch_fault("mlp backward launch")) return f;
  return hip_status(fcc::mlp_backward(d_params, in_dim, hidden, d_coef, d_target, rows, d_grad, d_loss_sum,
                                      d_out, d_workspace, stream),
                    "mlp backward launch");
}

fcc_status fcc_mlp_adam(float* d_params, float* d_m, float* d_v, const float* d_grad, int64_t n, float lr,
                        float beta1, float beta2, float eps, int32_t step, hipStream_t stream) {
  if (n < 0 || step < 1) return set_error(FCC_ERR_INVALID_ARG, "n must be >= 0 and step >= 1");
  if (n == 0) return FCC_OK;
  if (!d_params || !d_m || !d_v || !d_grad) return set_error(FCC_ERR_INVALID_ARG, "NULL pointer");
if (fcc_status f = injected_launch_fault("adam launch")) return f;
  return hip_status(fcc::mlp_adam(d_params, d_m, d_v, d_grad, n, lr, beta1, beta2, eps, step, stream),
                    "adam launch");
}

namespace {
// learned-path workspace: coefficients, fallback lags, MLP output, MLP scratch
struct LearnedCarve {
  size_t coef, fallback, out, mlp, total;
};
size_t round256(size_t b) { return (b + 255) & ~size_t(255); }
LearnedCarve learned_carve(const fcc::Plan& p, int hidden, int64_t T) {
  const int64_t R = T * p.P;
  LearnedCarve c{};
  c.coef = 0;
  c.fallback = c.coef + round256(sizeof(float) * size_t(R) * 2 * p.D);
  c.out = c.fallback + round256(sizeof(float) * size_t(R));
  c.mlp = c.out + round256(sizeof(float) * size_t(R) * 2);
  c.total = c.mlp + round256(sizeof(float) * fcc::mlp_workspace_floats(2 * p.D, hidden, R));
  if (fcc::mlp_fused_supported(2 * p.D, hidden)) c.total = c.out;   // the fused kernel keeps the layers on chip
  return c;
}
}  // namespace

fcc_status fcc_learned_workspace_bytes(fcc_plan plan, int32_t hidden, int64_t num_frames, size_t* bytes) {
  if (!plan || !bytes) return set_error(FCC_ERR_INVALID_ARG, "NULL argument");
  if (num_frames < 0) return set_error(FCC_ERR_INVALID_ARG, "num_frames must be >= 0");
  fcc_status st = check_mlp_shape(2 * plan->p.D, hidden, num_frames * plan->p.P);
  if (st != FCC_OK) return st;
  *bytes = learned_carve(plan->p, hidden, num_frames).total;
  return FCC_OK;
}

fcc_status fcc_tdoa_learned(fcc_plan plan, const void* d_basis, const void* d_spec, int64_t num_frames,
                            const float* d_params, int32_t hidden, float min_confidence, float* d_tau,
                            float* d_confidence, void* d_workspace, hipStream_t stream) {
  if (!plan) return set_error(FCC_ERR_INVALID_ARG, "NULL plan");
  const fcc::Plan& p = plan->p;
  if (num_frames < 0) return set_error(FCC_ERR_INVALID_ARG, "num_frames must be >= 0");
  if (p.method != FCC_METHOD_FCC) return set_error(FCC_ERR_UNSUPPORTED, "the learned stage needs the FCC method");
  const int64_t R = num_frames * p.P;
  fcc_status st = check_mlp_shape(2 * p.D, hidden, R);
  if (st != FCC_OK) return st;
  if (num_frames == 0) return FCC_OK;
  if (!d_params || !d_tau || !d_workspace) return set_error(FCC_ERR_INVALID_ARG, "NULL pointer");
  if (!aligned(d_workspace, 256)) return set_error(FCC_ERR_INVALID_ARG, "d_workspace must be 256-byte aligned");
  if (!aligned(d_tau, 4) || !aligned(d_params, 4) || (d_confidence && !aligned(d_confidence, 4)))
    return set_error(FCC_ERR_INVALID_ARG, "pointer misaligned");
  const LearnedCarve c = learned_carve(p, hidden, num_frames);
  char* ws = static_cast<char*>(d_workspace);
  float* coef = reinterpret_cast<float*>(ws + c.coef);
  float* fallback = reinterpret_cast<float*>(ws + c.fallback);
  float* out = reinterpret_cast<float*>(ws + c.out);
  // one pass over the spectra gives both the coefficients and the interpolated lag
  if ((st = pair_stage(p, d_basis, d_spec, num_frames, nullptr, nullptr, stream, coef, fallback)) != FCC_OK)
    return st;
  if (fcc::mlp_fused_supported(2 * p.D, hidden))
    return hip_status(fcc::mlp_infer_select(d_params, 2 * p.D, hidden, coef, R, fallback, min_confidence, d_tau,
                                            d_confidence, stream),
                      "fused mlp launch");
  if ((st = hip_status(fcc::mlp_forward(d_params, 2 * p.D, hidden, coef, R, out, ws + c.mlp, stream),
                       "mlp forward launch")) != FCC_OK)
    return st;
  return hip_status(fcc::mlp_select(out, fallback, R, min_confidence, d_tau, d_confidence, stream),
                    "select launch");
}

fcc_status fcc_doa_table(fcc_plan plan, const double* dirs, int32_t num_dirs, float* table) {
  if (!plan || !dirs || !table) return set_error(FCC_ERR_INVALID_ARG, "NULL argument");
  if (num_dirs < 1) return set_error(FCC_ERR_INVALID_ARG, "num_dirs must be >= 1");
  const fcc::Plan& p = plan->p;
  for (int64_t e = 0; e < 3 * int64_t(num_dirs); ++e)
    if (!std::isfinite(dirs[e])) return set_error(FCC_ERR_INVALID_ARG, "a direction has a non-finite entry");
  const double scale = p.r * p.fs / p.c, lag0 = double(p.r) * p.tau_max, top = double(p.I - 1);
  int pp = 0;
  for (int i = 0; i < p.M; ++i)
    for (int j = i + 1; j < p.M; ++j, ++pp) {
      const double bx = p.xyz[3 * j] - p.xyz[3 * i], by = p.xyz[3 * j + 1] - p.xyz[3 * i + 1],
                   bz = p.xyz[3 * j + 2] - p.xyz[3 * i + 2];
      for (int g = 0; g < num_dirs; ++g) {
        const double* u = dirs + 3 * size_t(g);
        double qv = scale * (bx * u[0] + by * u[1] + bz * u[2]) + lag0;
        qv = qv < 0.0 ? 0.0 : (qv > top ? top : qv);
        table[size_t(pp) * num_dirs + g] = float(qv);
      }
    }
  return FCC_OK;
}

fcc_status fcc_doa(fcc_plan plan, const float* d_y, int64_t num_frames, const float* d_table, int32_t num_dirs,
                   int32_t* d_doa, float* d_score, hipStream_t stream) {
  if (!plan) return set_error(FCC_ERR_INVALID_ARG, "NULL plan");
  if (num_frames < 0 || num_dirs < 1) return set_error(FCC_ERR_INVALID_ARG, "num_frames >= 0 and num_dirs >= 1");
  if (num_frames == 0) return FCC_OK;
  if (!d_y || !d_table || !d_doa) return set_error(FCC_ERR_INVALID_ARG, "NULL pointer");
  for (const void* o : {static_cast<const void*>(d_y), static_cast<const void*>(d_table),
                        static_cast<const void*>(d_doa), static_cast<const void*>(d_score)})
    if (o && !aligned(o, 4)) return set_error(FCC_ERR_INVALID_ARG, "pointer misaligned");
  fcc::DoaArgs a{};
  a.y = d_y;
  a.T = num_frames;
  a.P = plan->p.P;
  a.I = plan->p.I;
  a.table = d_table;
  a.G = num_dirs;
  a.doa = d_doa;
  a.score = d_score;
  a.stream = stream;
  if (!fcc::doa_supported(a)) return set_error(FCC_ERR_UNSUPPORTED, "one frame's correlations exceed 48 KB");
  if (fcc_status f = injected_launch_fault("doa launch")) return f;
  return hip_status(fcc::launch_doa(a), "doa launch");
}

// ---- batches ---------------------------------------------------------------

}  // extern "C": the helpers below are C++

namespace {

size_t batch_align(size_t b) { return (b + 255) & ~size_t(255); }

void batch_drop_graph(fcc_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  for (auto& k : b->graph_key) k = nullptr;
}

fcc::BatchRun batch_run(fcc_batch b, const void* d_image, const float* d_audio, int32_t* d_tdoa, void* d_ws,
                        hipStream_t stream) {
  fcc::BatchRun r{};
  const unsigned char* img = static_cast<const unsigned char*>(d_image);
  r.arrays = reinterpret_cast<const fcc::BatchArray*>(img + b->arrays_off);
  r.n_arrays = int(b->arrays.size());
  r.members = reinterpret_cast<const int32_t*>(img + b->members_off);
  r.image = img;
  r.audio = d_audio;
  r.spec = static_cast<unsigned char*>(d_ws);
  r.tdoa = d_tdoa;
  r.item_array = reinterpret_cast<const int32_t*>(img + b->items_off);
  r.stft_ranges = b->stft_ranges;
  r.precision = b->precision;
  r.stream = stream;
  return r;
}

hipError_t batch_enqueue(fcc_batch b, const fcc::BatchRun& r) {
  hipError_t e = fcc::launch_batch_stft(r);
  if (e != hipSuccess) return e;
  for (size_t c = 0; c < b->classes.size(); ++c)
    if ((e = fcc::launch_batch_pair(r, b->classes[c], b->pair_tuning[c])) != hipSuccess) return e;
  return hipSuccess;
}

fcc_status batch_check(fcc_batch b, const void* d_image, const float* d_audio, int32_t* d_tdoa, void* d_ws) {
  if (!b) return set_error(FCC_ERR_INVALID_ARG, "NULL batch");
  if (!d_image || !d_ws || (b->audio_floats > 0 && !d_audio) || (b->tdoa_count > 0 && !d_tdoa))
    return set_error(FCC_ERR_INVALID_ARG, "NULL pointer");
  if (!aligned(d_image, 256) || !aligned(d_ws, 256) || !aligned(d_audio, 4) || !aligned(d_tdoa, 4))
    return set_error(FCC_ERR_INVALID_ARG, "d_image and d_workspace must be 256-byte aligned");
  return FCC_OK;
}

}  // namespace

extern "C" {

fcc_status fcc_batch_create(const fcc_plan* plans, int32_t num_arrays, const int64_t* num_samples, fcc_batch* out) {
  if (!plans || !num_samples || !out || num_arrays < 1)
    return set_error(FCC_ERR_INVALID_ARG, "plans, num_samples and out must be non-NULL, num_arrays >= 1");
  *out = nullptr;
  fcc_batch b = injected_alloc_fault() ? nullptr : new (std::nothrow) fcc_batch_s;
  if (!b) return set_error(FCC_ERR_INTERNAL, "out of host memory");
  auto fail = [&](fcc_status st, const char* msg) {
    delete b;
    return set_error(st, msg);
  };
  b->precision = plans[0] ? plans[0]->p.precision : FCC_FP16;
  // classes: arrays sharing the tile shape (components in blocks of four, lag
  // tiles) and the frame size, so a class's LDS is sized for its own frames
  std::map<std::tuple<int, int, int>, std::vector<int>> by_shape;
  size_t img = 0, spec = 0;
  for (int a = 0; a < num_arrays; ++a) {
    if (!plans[a]) return fail(FCC_ERR_INVALID_ARG, "NULL plan");
    const fcc::Plan& p = plans[a]->p;
    if (num_samples[a] < 0) return fail(FCC_ERR_INVALID_ARG, "num_samples must be >= 0");
    if (p.precision != b->precision) return fail(FCC_ERR_INVALID_ARG, "every plan of a batch has the same precision");
    if (p.precision != FCC_FP16 && p.precision != FCC_BF16)
      return fail(FCC_ERR_UNSUPPORTED, "batches are built for FP16 or BF16 spectra");
    if (p.method != FCC_METHOD_FCC || p.alpha < 1.0f)
      return fail(FCC_ERR_UNSUPPORTED, "batches run the FCC method without smoothing");
    const int kb = p.Dpad / 4, tt = p.I <= 16 ? 1 : (p.I <= 32 ? 2 : 3);
    if (p.M > 16 || p.N < 32 || p.I > 48 || !(kb == 1 || kb == 2 || kb == 3 || kb == 4 || kb == 6 || kb == 8))
      return fail(FCC_ERR_UNSUPPORTED, "an array is outside the matrix-core pair stage (M <= 16, N >= 32, I <= 48, rank <= 32)");
    b->plans.push_back(p);
    fcc::BatchArray d{};
    d.M = p.M;
    d.P = p.P;
    d.N = p.N;
    d.hop = p.hop;
    d.I = p.I;
    d.lag0 = p.r * p.tau_max;
    d.L = num_samples[a];
    d.T = frames_of(p, num_samples[a]);
    if (d.T * int64_t(p.M) > int64_t(INT32_MAX)) return fail(FCC_ERR_UNSUPPORTED, "too many frames in one array");
    d.audio_off = b->audio_floats;
    d.spec_off = int64_t(spec);
    d.tdoa_off = b->tdoa_count;
    d.img_off = int64_t(img);
    d.tab_twiddle = int64_t(p.layout.twiddle);
    d.tab_pairs = int64_t(p.layout.pairs);
    d.tab_prow16 = int64_t(p.layout.prow16);
    d.tab_gexp = int64_t(p.layout.gexp);
    b->audio_floats += int64_t(p.M) * num_samples[a];
    b->tdoa_count += d.T * p.P;
    spec += batch_align(size_t(d.T) * p.M * (p.N / 2) * p.spec_elem);
    img += batch_align(p.layout.total);
    b->arrays.push_back(d);
    by_shape[{kb, tt, p.N}].push_back(a);
  }
  // front-end items: blocks of transforms, numbered frame size by frame size
  // (one launch per size), array by array within a size
  std::vector<int> sizes;
  for (const fcc::BatchArray& d : b->arrays)
    if (std::find(sizes.begin(), sizes.end(), d.N) == sizes.end()) sizes.push_back(d.N);
  std::sort(sizes.begin(), sizes.end());
  for (int N : sizes) {
    fcc::BatchStftRange g{N, b->stft_items, 0};
    const int fpb = fcc::stft_transforms_per_block(N);
    for (int a = 0; a < num_arrays; ++a) {
      fcc::BatchArray& d = b->arrays[a];
      if (d.N != N) continue;
      d.stft_first = b->stft_items;
      const int64_t items = (d.T * d.M + fpb - 1) / fpb;
      b->item_array.insert(b->item_array.end(), size_t(items), int32_t(a));
      b->stft_items += items;
    }
    g.count = b->stft_items - g.first;
    b->stft_ranges.push_back(g);
  }
  std::vector<std::vector<int64_t>> prefixes;     // per class: cost prefix over its members
  for (auto& kv : by_shape) {
    std::vector<int64_t> c_prefix(1, 0);
    fcc::BatchClass c;
    c.index = int(b->classes.size());
    c.kb = std::get<0>(kv.first);
    c.tt = std::get<1>(kv.first);
    c.member_first = int(b->members.size());
    c.member_count = int(kv.second.size());
    for (int a : kv.second) {
      const fcc::BatchArray& d = b->arrays[a];
      b->members.push_back(a);
      c.member_frames.push_back(d.T);
      c_prefix.push_back(c_prefix.back() + d.T * fcc::pair_frame_weight(d.N));
      c.head_words_max = std::max(c.head_words_max, fcc::batch_head_words(4 * c.kb, d.N / 2, c.tt, d.P));
      c.slab_words_max = std::max(c.slab_words_max, fcc::batch_slab_words(d.N, d.I));
    }
    // the launcher's own condition: two wavefronts' slabs beside the tables
    if (sizeof(uint32_t) * (size_t(c.head_words_max) + 2 * size_t(c.slab_words_max)) > 160 * 1024)
      return fail(FCC_ERR_UNSUPPORTED, "a class's tables and two wavefront slabs exceed 160 KB of LDS");
    b->classes.push_back(c);
    prefixes.push_back(std::move(c_prefix));
  }
  b->pair_tuning.assign(b->classes.size(), fcc::PairTuning{});
  b->arrays_off = img;
  b->members_off = batch_align(b->arrays_off + sizeof(fcc::BatchArray) * b->arrays.size());
  b->items_off = batch_align(b->members_off + sizeof(int32_t) * b->members.size());
  size_t end = batch_align(b->items_off + sizeof(int32_t) * b->item_array.size());
  for (size_t c = 0; c < b->classes.size(); ++c) {
    b->classes[c].wprefix_off = end;
    end = batch_align(end + sizeof(int64_t) * prefixes[c].size());
  }
  b->image.assign(end, 0);
  for (int a = 0; a < num_arrays; ++a)
    std::memcpy(b->image.data() + b->arrays[a].img_off, b->plans[a].image.data(), b->plans[a].image.size());
  std::memcpy(b->image.data() + b->arrays_off, b->arrays.data(), sizeof(fcc::BatchArray) * b->arrays.size());
  std::memcpy(b->image.data() + b->members_off, b->members.data(), sizeof(int32_t) * b->members.size());
  if (!b->item_array.empty())
    std::memcpy(b->image.data() + b->items_off, b->item_array.data(), sizeof(int32_t) * b->item_array.size());
  for (size_t c = 0; c < b->classes.size(); ++c)
    std::memcpy(b->image.data() + b->classes[c].wprefix_off, prefixes[c].data(), sizeof(int64_t) * prefixes[c].size());
  b->spec_bytes = spec;
  b->workspace_bytes = batch_align(spec) + 256;
  *out = b;
  return FCC_OK;
}

void fcc_batch_destroy(fcc_batch b) {
  if (!b) return;
  batch_drop_graph(b);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  delete b;
}

fcc_status fcc_batch_query(fcc_batch b, fcc_batch_info* info) {
  if (!b || !info) return set_error(FCC_ERR_INVALID_ARG, "NULL argument");
  info->num_arrays = int32_t(b->arrays.size());
  info->num_classes = int32_t(b->classes.size());
  info->image_bytes = b->image.size();
  info->workspace_bytes = b->workspace_bytes;
  info->audio_floats = b->audio_floats;
  info->tdoa_count = b->tdoa_count;
  return FCC_OK;
}

fcc_status fcc_batch_layout(fcc_batch b, int64_t* audio_offset, int64_t* tdoa_offset, int64_t* num_frames) {
  if (!b) return set_error(FCC_ERR_INVALID_ARG, "NULL batch");
  for (size_t a = 0; a < b->arrays.size(); ++a) {
    if (audio_offset) audio_offset[a] = b->arrays[a].audio_off;
    if (tdoa_offset) tdoa_offset[a] = b->arrays[a].tdoa_off;
    if (num_frames) num_frames[a] = b->arrays[a].T;
  }
  return FCC_OK;
}

fcc_status fcc_batch_upload(fcc_batch b, void* d_image, hipStream_t stream) {
  if (!b || !d_image) return set_error(FCC_ERR_INVALID_ARG, "NULL argument");
  if (!aligned(d_image, 256)) return set_error(FCC_ERR_INVALID_ARG, "d_image must be 256-byte aligned");
  if (fcc_status f = injected_launch_fault("batch upload")) return f;
  return hip_status(hipMemcpyAsync(d_image, b->image.data(), b->image.size(), hipMemcpyHostToDevice, stream),
                    "batch image copy");
}

fcc_status fcc_batch_tdoa(fcc_batch b, const void* d_image, const float* d_audio, int32_t* d_tdoa, void* d_workspace,
                          int32_t use_graph, hipStream_t stream) {
  fcc_status st = batch_check(b, d_image, d_audio, d_tdoa, d_workspace);
  if (st != FCC_OK) return st;
  if (b->tdoa_count == 0) return FCC_OK;          // no array holds a whole frame: nothing to launch
  if (fcc_status f = injected_launch_fault("batch launch")) return f;
  if (!use_graph)
    return hip_status(batch_enqueue(b, batch_run(b, d_image, d_audio, d_tdoa, d_workspace, stream)), "batch launch");
  const void* key[4] = {d_image, d_audio, d_tdoa, d_workspace};
  if (!b->exec || !std::equal(key, key + 4, b->graph_key)) {
    batch_drop_graph(b);
    if (!b->capture_stream &&
        hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess)
      return set_error(FCC_ERR_HIP, "capture stream creation failed");
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_status(e, "graph capture begin");
    const hipError_t le = batch_enqueue(b, batch_run(b, d_image, d_audio, d_tdoa, d_workspace, b->capture_stream));
    e = hipStreamEndCapture(b->capture_stream, &graph);
    if (le != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_status(le, "batch launch during capture");
    }
    if (e != hipSuccess) return hip_status(e, "graph capture end");
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      b->exec = nullptr;
      return hip_status(e, "graph instantiation");
    }
    std::copy(key, key + 4, b->graph_key);
  }
  return hip_status(hipGraphLaunch(b->exec, stream), "graph launch");
}

fcc_status fcc_batch_tune(fcc_batch b, const void* d_image, const float* d_audio, int32_t* d_tdoa, void* d_workspace,
                          hipStream_t stream) {
  fcc_status st = batch_check(b, d_image, d_audio, d_tdoa, d_workspace);
  if (st != FCC_OK) return st;
  if (b->tdoa_count == 0) return FCC_OK;          // nothing to time: the default shapes stay
  if (fcc_status f = injected_launch_fault("batch tuning launch")) return f;
  batch_drop_graph(b);
  const fcc::BatchRun r = batch_run(b, d_image, d_audio, d_tdoa, d_workspace, stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return set_error(FCC_ERR_HIP, "event creation failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set_error(FCC_ERR_HIP, "event creation failed");
  }
  const int reps = 3;
  // time `launch` reps times after one untimed run; +inf when it cannot run
  auto time_of = [&](auto&& launch) -> float {
    hipError_t e = hipSuccess;
    for (int w = 0; w < 1 + reps && e == hipSuccess; ++w) {
      if (w == 1) e = hipEventRecord(e0, stream);
      if (e == hipSuccess) e = launch();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 3.4e38f;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 3.4e38f;
    return ms;
  };
  fcc_status result = FCC_OK;
  float best = 3.4e38f;
  // the front end has no shape to choose (one workgroup per block of
  // transforms); the pair stage reads the spectra it writes
  if (time_of([&] { return fcc::launch_batch_stft(r); }) >= 3.4e38f)
    result = set_error(FCC_ERR_HIP, "front end failed");
  for (size_t c = 0; c < b->classes.size() && result == FCC_OK; ++c) {
    best = 3.4e38f;
    fcc::PairTuning best_p = b->pair_tuning[c];
    for (int waves : {2, 3, 4})
      for (int bpc : {1, 2, 3, 4}) {
        const fcc::PairTuning t{waves, bpc};
        const float ms = time_of([&] { return fcc::launch_batch_pair(r, b->classes[c], t); });
        if (ms < best) {
          best = ms;
          best_p = t;
        }
      }
    if (best >= 3.4e38f) result = set_error(FCC_ERR_HIP, "no pair tiling ran");
    b->pair_tuning[c] = best_p;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return result;
}

fcc_status fcc_batch_tuning(fcc_batch b, int32_t* values, int32_t capacity) {
  if (!b || !values) return set_error(FCC_ERR_INVALID_ARG, "NULL argument");
  const int32_t need = 2 + 3 * int32_t(b->classes.size());
  if (capacity < need) return set_error(FCC_ERR_INVALID_ARG, "capacity below 2 + 3 * num_classes");
  values[0] = int32_t(b->stft_ranges.size());
  values[1] = 0;
  for (size_t c = 0; c < b->classes.size(); ++c) {
    values[2 + 3 * c] = int32_t(fcc::batch_pair_workgroups(b->classes[c], b->pair_tuning[c]));
    values[3 + 3 * c] = fcc::batch_pair_waves(b->classes[c], b->pair_tuning[c]);
    values[4 + 3 * c] = b->pair_tuning[c].blocks_per_cu;
  }
  return FCC_OK;
}

const char* fcc_status_string(fcc_status status) {
  int32_t v;                          // the int a C caller passed, whatever its value
  std::memcpy(&v, &status, sizeof v);
  switch (v) {
    case FCC_OK: return "FCC_OK";
    case FCC_ERR_INVALID_ARG: return "FCC_ERR_INVALID_ARG";
    case FCC_ERR_UNSUPPORTED: return "FCC_ERR_UNSUPPORTED";
    case FCC_ERR_BASIS_AMBIGUOUS: return "FCC_ERR_BASIS_AMBIGUOUS";
    case FCC_ERR_HIP: return "FCC_ERR_HIP";
    case FCC_ERR_INTERNAL: return "FCC_ERR_INTERNAL";
  }
  return "unknown fcc_status";
}

const char* fcc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
