// Host-side exercise of the planner and of the C ABI's argument checks, built
// with AddressSanitizer and UndefinedBehaviorSanitizer on the host code (the
// library's device objects are linked as built).  It never enqueues device
// work: every call below either returns before any HIP call (argument errors,
// refusals, host queries, the basis export) or meets the FCC_FAULT=launch
// hook, which fails launches on the host.  Exit status 0 when every status
// matches; any sanitizer report aborts with a non-zero status.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "fcc.h"

static int g_fail = 0;

static void expect(fcc_status got, fcc_status want, const char* what) {
  if (got != want) {
    std::printf("FAIL %s: got %d (%s) want %d: %s\n", what, int(got), fcc_status_string(got), int(want),
                fcc_last_error());
    ++g_fail;
  }
}

static fcc_config circle(int M, double radius) {
  static std::vector<double> xyz;
  xyz.assign(3 * size_t(M), 0.0);
  for (int m = 0; m < M; ++m) {
    xyz[3 * m] = radius * std::cos(2.0 * M_PI * m / M);
    xyz[3 * m + 1] = radius * std::sin(2.0 * M_PI * m / M);
  }
  fcc_config c{};
  c.num_mics = M;
  c.mic_xyz = xyz.data();
  c.fs = 16000.0;
  c.c = 343.0;
  c.frame_size = 512;
  c.hop = 128;
  c.tau_max = 0;
  c.rank = 0;
  c.interp = 1;
  c.alpha = 1.0f;
  c.precision = FCC_FP16;
  c.method = FCC_METHOD_FCC;
  c.operands = FCC_OPERANDS_FP16;
  return c;
}

static void refused(fcc_config c, fcc_status want, const char* what) {
  fcc_plan p = nullptr;
  expect(fcc_plan_create(&c, &p), want, what);
  if (p) fcc_plan_destroy(p);
}

int main() {
  // ---- planner refusals ------------------------------------------------------
  fcc_config c = circle(16, 0.05);
  { fcc_config b = c; b.num_mics = 1; refused(b, FCC_ERR_INVALID_ARG, "M = 1"); }
  { fcc_config b = c; b.num_mics = 40; refused(b, FCC_ERR_UNSUPPORTED, "M = 40"); }
  { fcc_config b = c; b.mic_xyz = nullptr; refused(b, FCC_ERR_INVALID_ARG, "mic_xyz NULL"); }
  { fcc_config b = c; b.frame_size = 500; refused(b, FCC_ERR_INVALID_ARG, "N not a power of two"); }
  { fcc_config b = c; b.frame_size = 4096; refused(b, FCC_ERR_INVALID_ARG, "N above 2048"); }
  { fcc_config b = c; b.hop = 0; refused(b, FCC_ERR_INVALID_ARG, "hop 0"); }
  { fcc_config b = c; b.fs = 0.0; refused(b, FCC_ERR_INVALID_ARG, "fs 0"); }
  { fcc_config b = c; b.c = -1.0; refused(b, FCC_ERR_INVALID_ARG, "c < 0"); }
  { fcc_config b = c; b.fs = NAN; refused(b, FCC_ERR_INVALID_ARG, "fs NaN"); }
  { fcc_config b = c; b.interp = 3; refused(b, FCC_ERR_INVALID_ARG, "interp 3"); }
  { fcc_config b = c; b.alpha = 0.0f; refused(b, FCC_ERR_INVALID_ARG, "alpha 0"); }
  { fcc_config b = c; b.alpha = 1.5f; refused(b, FCC_ERR_INVALID_ARG, "alpha 1.5"); }
  { fcc_config b = c; b.alpha = 0.5f; refused(b, FCC_ERR_UNSUPPORTED, "alpha < 1 at fp16"); }
  { fcc_config b = c; b.precision = fcc_precision(7); refused(b, FCC_ERR_INVALID_ARG, "precision 7"); }
  { fcc_config b = c; b.method = fcc_method(5); refused(b, FCC_ERR_INVALID_ARG, "method 5"); }
  { fcc_config b = c; b.operands = fcc_operands(9); refused(b, FCC_ERR_INVALID_ARG, "operands 9"); }
  { fcc_config b = c; b.tau_max = -1; refused(b, FCC_ERR_INVALID_ARG, "tau_max < 0"); }
  { fcc_config b = c; b.tau_max = 200; refused(b, FCC_ERR_INVALID_ARG, "r tau_max >= N/4"); }
  { fcc_config b = c; b.rank = -2; refused(b, FCC_ERR_INVALID_ARG, "rank < 0"); }
  { fcc_config b = c; b.rank = 12; refused(b, FCC_ERR_INVALID_ARG, "rank > I"); }
  { fcc_config b = c; b.method = FCC_METHOD_GCC; b.interp = 4; b.frame_size = 2048; b.hop = 512;
    refused(b, FCC_ERR_UNSUPPORTED, "GCC r N > 4096"); }
  { fcc_config b = c; b.frame_size = 512; b.tau_max = 40; b.rank = 16;
    refused(b, FCC_ERR_BASIS_AMBIGUOUS, "rank inside a singular-value cluster"); }
  { fcc_config b = c; std::vector<double> xyz(3 * 16, 0.0); xyz[5] = INFINITY; b.mic_xyz = xyz.data();
    refused(b, FCC_ERR_INVALID_ARG, "non-finite position"); }
  expect(fcc_plan_create(nullptr, nullptr), FCC_ERR_INVALID_ARG, "NULL config");
  {
    // out-of-range values a C caller can store in the enum fields
    fcc_config b = c;
    const int32_t bad = -3;
    std::memcpy(&b.precision, &bad, sizeof bad);
    refused(b, FCC_ERR_INVALID_ARG, "precision -3");
    const int32_t big = 1 << 20;
    b = c;
    std::memcpy(&b.operands, &big, sizeof big);
    refused(b, FCC_ERR_INVALID_ARG, "operands 2^20");
  }

  // ---- valid plans: query, sizes, basis export (every precision, method, r, alpha)
  const fcc_precision precs[] = {FCC_FP32, FCC_BF16, FCC_FP16, FCC_FP8_E4M3};
  for (fcc_precision pr : precs)
    for (int r : {1, 2})
      for (int D : {0, 6}) {
        fcc_config b = c;
        b.precision = pr;
        b.interp = r;
        b.rank = D;
        b.operands = pr == FCC_BF16 || pr == FCC_FP8_E4M3 ? FCC_OPERANDS_STORAGE : FCC_OPERANDS_FP16;
        fcc_plan p = nullptr;
        expect(fcc_plan_create(&b, &p), FCC_OK, "valid plan");
        if (!p) continue;
        fcc_plan_info info{};
        expect(fcc_plan_query(p, &info), FCC_OK, "query");
        const int Dr = info.rank, I = info.num_lags, Bs = info.frame_size / 4 + 1;
        std::vector<double> sigma(Dr), ph(size_t(Dr) * Bs), dc(size_t(I) * Dr), ds(size_t(I) * Dr);
        std::vector<int32_t> sym(Dr);
        expect(fcc_basis_export(p, sigma.data(), sym.data(), ph.data(), dc.data(), ds.data()), FCC_OK, "export");
        for (int k = 1; k < Dr; ++k)
          if (!(sigma[k] <= sigma[k - 1] * (1 + 1e-12))) { std::printf("FAIL sigma order\n"); ++g_fail; }
        int64_t T = -1;
        expect(fcc_num_frames(p, 960000, &T), FCC_OK, "num_frames");
        if (T != 7497) { std::printf("FAIL T = %lld\n", (long long)T); ++g_fail; }
        expect(fcc_num_frames(p, 100, &T), FCC_OK, "num_frames short");
        if (T != 0) { std::printf("FAIL short T\n"); ++g_fail; }
        expect(fcc_num_frames(p, -1, &T), FCC_ERR_INVALID_ARG, "num_frames < 0");
        size_t ws = 0;
        expect(fcc_workspace_bytes(p, 7497, &ws), FCC_OK, "workspace bytes");
        if (ws < size_t(7497) * info.spectrum_bytes_per_frame) { std::printf("FAIL workspace\n"); ++g_fail; }
        expect(fcc_workspace_bytes(p, -5, &ws), FCC_ERR_INVALID_ARG, "workspace < 0");
        expect(fcc_basis_export(p, nullptr, nullptr, nullptr, nullptr, nullptr), FCC_OK, "export, no outputs");
        expect(fcc_basis_export(nullptr, sigma.data(), nullptr, nullptr, nullptr, nullptr), FCC_ERR_INVALID_ARG,
               "export NULL plan");
        // DoA table on the host
        const double dirs[6] = {1, 0, 0, 0, 1, 0};
        std::vector<float> tab(size_t(info.num_pairs) * 2);
        expect(fcc_doa_table(p, dirs, 2, tab.data()), FCC_OK, "doa table");
        expect(fcc_doa_table(p, dirs, 0, tab.data()), FCC_ERR_INVALID_ARG, "doa table no dirs");
        fcc_plan_destroy(p);
      }

  // ---- argument errors of the device calls (nothing is enqueued) ------------
  fcc_plan p = nullptr;
  expect(fcc_plan_create(&c, &p), FCC_OK, "plan");
  void* fake = reinterpret_cast<void*>(uintptr_t(1) << 20);   // aligned, never dereferenced
  void* odd = reinterpret_cast<void*>((uintptr_t(1) << 20) + 2);
  float* fx = static_cast<float*>(fake);
  int32_t* ft = static_cast<int32_t*>(fake);
  expect(fcc_tdoa(nullptr, fake, fx, 960000, 960000, ft, fake, nullptr), FCC_ERR_INVALID_ARG, "tdoa NULL plan");
  expect(fcc_tdoa(p, nullptr, fx, 960000, 960000, ft, fake, nullptr), FCC_ERR_INVALID_ARG, "tdoa NULL basis");
  expect(fcc_tdoa(p, odd, fx, 960000, 960000, ft, fake, nullptr), FCC_ERR_INVALID_ARG, "tdoa basis misaligned");
  expect(fcc_tdoa(p, fake, fx, 960000, 100, ft, fake, nullptr), FCC_ERR_INVALID_ARG, "tdoa ld < L");
  expect(fcc_tdoa(p, fake, fx, -1, 100, ft, fake, nullptr), FCC_ERR_INVALID_ARG, "tdoa L < 0");
  expect(fcc_tdoa(p, fake, nullptr, 960000, 960000, ft, fake, nullptr), FCC_ERR_INVALID_ARG, "tdoa NULL x");
  expect(fcc_tdoa(p, fake, fx, 960000, 960000, nullptr, fake, nullptr), FCC_ERR_INVALID_ARG, "tdoa NULL out");
  expect(fcc_tdoa(p, fake, fx, 960000, 960000, ft, nullptr, nullptr), FCC_ERR_INVALID_ARG, "tdoa NULL ws");
  expect(fcc_tdoa(p, fake, fx, 100, 100, nullptr, nullptr, nullptr), FCC_OK, "tdoa no frame");
  expect(fcc_tdoa_noalloc(p, fake, fx, 960000, 960000, nullptr, nullptr), FCC_ERR_INVALID_ARG, "noalloc NULL out");
  expect(fcc_tdoa_from_spectra(p, fake, fake, -1, ft, nullptr), FCC_ERR_INVALID_ARG, "from_spectra T < 0");
  expect(fcc_tdoa_from_spectra(p, fake, nullptr, 10, ft, nullptr), FCC_ERR_INVALID_ARG, "from_spectra NULL spec");
  expect(fcc_correlation(p, fake, fake, 10, nullptr, nullptr), FCC_ERR_INVALID_ARG, "correlation NULL y");
  expect(fcc_spectra(p, fake, fx, 960000, 960000, nullptr, nullptr), FCC_ERR_INVALID_ARG, "spectra NULL out");
  expect(fcc_plan_upload(p, odd, nullptr), FCC_ERR_INVALID_ARG, "upload misaligned");
  expect(fcc_tdoa_smoothed(p, fake, fake, 10, static_cast<float*>(fake), ft, nullptr, nullptr, fake, nullptr),
         FCC_ERR_INVALID_ARG, "smoothed on an alpha = 1 plan");
  expect(fcc_mlp_forward(static_cast<float*>(fake), 0, 128, fx, 10, fx, fake, nullptr), FCC_ERR_INVALID_ARG,
         "mlp in_dim 0");
  expect(fcc_mlp_adam(fx, fx, fx, fx, -1, 1e-3f, 0.9f, 0.999f, 1e-8f, 1, nullptr), FCC_ERR_INVALID_ARG, "adam n < 0");
  size_t mws = 0;
  expect(fcc_mlp_workspace_bytes(22, 128, 1000, &mws), FCC_OK, "mlp workspace");
  {
    fcc_config s = c;
    s.precision = FCC_FP32;
    s.alpha = 0.5f;
    fcc_plan q = nullptr;
    expect(fcc_plan_create(&s, &q), FCC_OK, "smoothed plan");
    expect(fcc_tdoa_noalloc(q, fake, fx, 960000, 960000, ft, nullptr), FCC_ERR_UNSUPPORTED, "noalloc alpha < 1");
    expect(fcc_tdoa_from_spectra(q, fake, fake, 10, ft, nullptr), FCC_ERR_UNSUPPORTED, "pair stage alpha < 1");
    fcc_plan_destroy(q);
  }

  // ---- batches: refusals and host layout -------------------------------------
  {
    fcc_plan plans[3] = {p, nullptr, nullptr};
    int64_t L[3] = {16000, 32000, 8000};
    fcc_batch bt = nullptr;
    expect(fcc_batch_create(plans, 0, L, &bt), FCC_ERR_INVALID_ARG, "batch of none");
    expect(fcc_batch_create(plans, 2, L, &bt), FCC_ERR_INVALID_ARG, "batch NULL plan");
    fcc_config b8 = c;
    b8.num_mics = 8;
    fcc_config c8 = circle(8, 0.03);
    c8.precision = FCC_FP16;
    fcc_plan q = nullptr, r = nullptr;
    expect(fcc_plan_create(&c8, &q), FCC_OK, "batch plan 2");
    fcc_config c32 = c8;
    c32.precision = FCC_FP32;
    expect(fcc_plan_create(&c32, &r), FCC_OK, "batch plan fp32");
    plans[1] = r;
    expect(fcc_batch_create(plans, 2, L, &bt), FCC_ERR_INVALID_ARG, "batch mixed precision");
    plans[1] = q;
    int64_t Lbad[2] = {16000, -3};
    expect(fcc_batch_create(plans, 2, Lbad, &bt), FCC_ERR_INVALID_ARG, "batch L < 0");
    expect(fcc_batch_create(plans, 2, L, &bt), FCC_OK, "batch");
    if (bt) {
      fcc_batch_info bi{};
      expect(fcc_batch_query(bt, &bi), FCC_OK, "batch query");
      std::vector<int64_t> ao(2), to(2), nf(2);
      expect(fcc_batch_layout(bt, ao.data(), to.data(), nf.data()), FCC_OK, "batch layout");
      if (nf[0] != 122 || nf[1] != (32000 - 512) / 128 + 1) { std::printf("FAIL batch frames\n"); ++g_fail; }
      expect(fcc_batch_tdoa(bt, nullptr, fx, ft, fake, 1, nullptr), FCC_ERR_INVALID_ARG, "batch NULL image");
      fcc_batch_destroy(bt);
    }
    fcc_plan_destroy(q);
    fcc_plan_destroy(r);
  }

  // ---- failure injection -------------------------------------------------------
  setenv("FCC_FAULT", "launch", 1);
  expect(fcc_tdoa(p, fake, fx, 960000, 960000, ft, fake, nullptr), FCC_ERR_HIP, "injected launch: tdoa");
  if (!std::strstr(fcc_last_error(), "injected")) { std::printf("FAIL injected message\n"); ++g_fail; }
  expect(fcc_tdoa_noalloc(p, fake, fx, 960000, 960000, ft, nullptr), FCC_ERR_HIP, "injected launch: noalloc");
  expect(fcc_tdoa_from_spectra(p, fake, fake, 10, ft, nullptr), FCC_ERR_HIP, "injected launch: pair stage");
  expect(fcc_spectra(p, fake, fx, 960000, 960000, fake, nullptr), FCC_ERR_HIP, "injected launch: spectra");
  expect(fcc_plan_upload(p, fake, nullptr), FCC_ERR_HIP, "injected launch: upload");
  expect(fcc_mlp_adam(fx, fx, fx, fx, 100, 1e-3f, 0.9f, 0.999f, 1e-8f, 1, nullptr), FCC_ERR_HIP,
         "injected launch: adam");
  // argument errors still come first
  expect(fcc_tdoa(p, nullptr, fx, 960000, 960000, ft, fake, nullptr), FCC_ERR_INVALID_ARG,
         "injected launch: argument error first");
  setenv("FCC_FAULT", "alloc", 1);
  {
    fcc_plan q = nullptr;
    expect(fcc_plan_create(&c, &q), FCC_ERR_INTERNAL, "injected alloc: plan");
    if (q) { std::printf("FAIL plan returned\n"); ++g_fail; fcc_plan_destroy(q); }
    fcc_plan plans[1] = {p};
    int64_t L[1] = {16000};
    fcc_batch bt = nullptr;
    expect(fcc_batch_create(plans, 1, L, &bt), FCC_ERR_INTERNAL, "injected alloc: batch");
  }
  unsetenv("FCC_FAULT");
  fcc_plan_destroy(p);
  std::printf("%s: %d failed checks\n", g_fail ? "FAIL" : "OK", g_fail);
  return g_fail ? 1 : 0;
}
