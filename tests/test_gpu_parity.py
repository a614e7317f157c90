"""GPU path (through the C ABI) against the FP64 oracle.

FP32 bar: relative correlation error <= 1e-4 per pair-frame, and integer TDoA
bit-exact wherever the oracle's top two correlation values are more than
2e-4 max|y| apart (see tests/parity.py).
"""
import sys

import numpy as np
import pytest

import oracle.fcc_oracle as O
from gen import make_recording, white_pair, random_signals, circular_array, square_array
from tests.parity import corr_errors, tdoa_report

pytestmark = pytest.mark.gpu

EPS32 = 1e-4


def _say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def fcc():
    import paper_2204_13622_amd as fcc
    fcc._lib.load()
    return fcc


def _dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _oracle_spec_tensor(torch, X, dtype):
    """Oracle-whitened spectra e = X / |X| as a packed [T, M, N/2, 2] device tensor."""
    from paper_2204_13622_amd import Plan
    arr = Plan.pack_spectrum(O.phat(X)).astype(np.float32)
    return torch.from_numpy(arr).cuda().to(dtype).contiguous()


def _plan(fcc, rec, D, **kw):
    return fcc.Plan(rec.mic_xyz, rec.fs, rec.c, frame_size=rec.N, hop=rec.hop, rank=D, **kw)


def _check_fp32(t_gpu, y_gpu, y_ref, tau_max):
    if y_gpu is not None:
        e = corr_errors(y_gpu, y_ref)
        assert e.size == 0 or e.max() <= EPS32, f"max rel corr err {e.max():.3e}"
    rep = tdoa_report(t_gpu, y_ref, tau_max, EPS32)
    assert rep["mismatch_qualified"] == 0, rep
    assert rep["invalid_elsewhere"] == 0, rep
    return rep


# ---------------------------------------------------------------- front end --

@pytest.mark.parametrize("config,seconds", [(1, 1.0), (2, 2.0), (3, 1.0)])
def test_spectra_fp32(torch, fcc, config, seconds):
    _say(f"fcc_spectra fp32 config {config} {seconds}s")
    rec = make_recording(config, seconds=seconds)
    p = _plan(fcc, rec, 0)
    spec = p.spectra(_dev(torch, rec.x))
    torch.cuda.synchronize()
    X = O.stft(rec.x, rec.N, rec.hop)
    e_ref = O.phat(X)
    e_gpu = fcc.Plan.unpack_spectrum(spec.cpu().numpy())
    assert e_gpu.shape == e_ref.shape
    mag = np.abs(X)
    rms = np.sqrt((mag ** 2).mean(-1, keepdims=True))
    # an FP32 FFT errs by ~1e-7 of the frame's RMS bin magnitude in every bin, so
    # the phase of a bin of magnitude |X| errs by about that divided by |X|
    d = np.abs(e_gpu - e_ref)
    scaled = np.where(mag > 0, d * mag / np.where(rms > 0, rms, 1), d)
    print(f"max |de| |X| / rms = {scaled.max():.2e}, max |de| = {d.max():.2e}", flush=True)
    assert scaled.max() < 1e-5
    assert np.abs(np.abs(e_gpu[mag > 0]) - 1).max() < 1e-5


@pytest.mark.parametrize("precision", ["fp16", "bf16", "fp8"])
@pytest.mark.parametrize("config,seconds", [(1, 1.0), (2, 1.0), (3, 0.3)])
def test_storage_encoding(torch, fcc, precision, config, seconds):
    """The front end's storage encoders: the whitened spectra in a 16- or
    8-bit type are the FP32 spectra of the same kernel rounded to nearest
    even, bit for bit (host rounding by torch)."""
    _say(f"storage encoding {precision} config {config}")
    rec = make_recording(config, seconds=seconds)
    x = _dev(torch, rec.x)
    ref = _plan(fcc, rec, 0).spectra(x)
    p = _plan(fcc, rec, 0, precision=precision)
    got = p.spectra(x)
    torch.cuda.synchronize()
    want = ref.cpu().to(p.spectrum_dtype())
    g = got.cpu().view(torch.uint8 if precision == "fp8" else torch.int16)
    w = want.view(torch.uint8 if precision == "fp8" else torch.int16)
    bad = int((g != w).sum())
    print(f"{precision}: {bad} of {g.numel()} values differ", flush=True)
    assert bad == 0


# ----------------------------------------------------- pair stage (isolated) --

@pytest.mark.parametrize("config,seconds,D", [(1, 1.0, 9), (1, 1.0, 5), (2, 1.0, 6), (2, 1.0, 11),
                                              (3, 0.5, 15), (3, 0.5, 29)])
def test_pair_stage_from_oracle_spectra(torch, fcc, config, seconds, D):
    _say(f"fcc_correlation / fcc_tdoa_from_spectra fp32 config {config} D={D}")
    rec = make_recording(config, seconds=seconds)
    p = _plan(fcc, rec, D)
    X = O.stft(rec.x, rec.N, rec.hop)
    spec = _oracle_spec_tensor(torch, X, torch.float32)
    y = p.correlation(spec)
    t = p.tdoa_from_spectra(spec)
    torch.cuda.synchronize()
    B = O.fcc_basis(rec.N, p.tau_max, D)
    y_ref = O.fcc_corr(O.phat(O.cross_spectrum(X)), B)
    _check_fp32(t.cpu().numpy(), y.cpu().numpy(), y_ref, p.tau_max)


@pytest.mark.parametrize("config,seconds", [(1, 1.0), (2, 1.0), (3, 0.5)])
def test_gcc_method(torch, fcc, config, seconds):
    _say(f"GCC method fp32 config {config}")
    rec = make_recording(config, seconds=seconds)
    p = _plan(fcc, rec, 0, method="gcc")
    X = O.stft(rec.x, rec.N, rec.hop)
    spec = _oracle_spec_tensor(torch, X, torch.float32)
    y = p.correlation(spec)
    t = p.tdoa_from_spectra(spec)
    torch.cuda.synchronize()
    y_ref = O.gcc_corr(O.phat(O.cross_spectrum(X)), rec.N, p.tau_max)
    _check_fp32(t.cpu().numpy(), y.cpu().numpy(), y_ref, p.tau_max)


@pytest.mark.parametrize("M,N,tau_max", [(3, 16, 3), (5, 32, 7), (2, 64, 1), (7, 256, 20), (32, 256, 9),
                                         (16, 2048, 30)])
def test_gcc_shapes(torch, fcc, M, N, tau_max):
    """Odd pair counts, the smallest transforms, many mics, and a shape whose
    spectra do not fit the IFFT kernel's LDS (direct eq. (2) kernel)."""
    _say(f"GCC shapes M={M} N={N} tau_max={tau_max}")
    x = random_signals(300 + M, M, 6 * N, kind="gated")
    p = fcc.Plan(circular_array(M, 0.05), 16000.0, frame_size=N, hop=N // 2, tau_max=tau_max, method="gcc")
    assert p.I == 2 * tau_max + 1
    X = O.stft(x, N, N // 2)
    spec = _oracle_spec_tensor(torch, X, torch.float32)
    y = p.correlation(spec)
    t = p.tdoa_from_spectra(spec)
    torch.cuda.synchronize()
    y_ref = O.gcc_corr(O.phat(O.cross_spectrum(X)), N, tau_max)
    _check_fp32(t.cpu().numpy(), y.cpu().numpy(), y_ref, tau_max)


@pytest.mark.parametrize("M,N,tau_max,seconds", [(16, 512, 5, 1.0), (16, 2048, 30, 0.5)])
def test_gcc_fp16_spectra(torch, fcc, M, N, tau_max, seconds):
    """GCC on FP16-stored spectra (inverse FFT, and the direct eq. (2) kernel
    where the spectra exceed the FFT kernel's LDS) against the oracle on the
    same quantised spectra: the arithmetic after decoding is FP32."""
    _say(f"GCC fp16 spectra M={M} N={N}")
    from paper_2204_13622_amd import Plan
    x = random_signals(500 + N, M, int(16000 * seconds))
    p = fcc.Plan(circular_array(M, 0.05), 16000.0, frame_size=N, hop=N // 4, tau_max=tau_max, method="gcc",
                 precision="fp16")
    X = O.stft(x, N, N // 4)
    packed = Plan.pack_spectrum(O.phat(X)).astype(np.float16)
    e = Plan.unpack_spectrum(packed.astype(np.float64))
    R = np.stack([e[:, i] * np.conj(e[:, j]) for i, j in O.mic_pairs(M)], axis=1)
    y_ref = O.gcc_corr(R, N, tau_max)
    spec = torch.from_numpy(packed).cuda().contiguous()
    y = p.correlation(spec).cpu().numpy()
    t = p.tdoa_from_spectra(spec).cpu().numpy()
    _check_fp32(t, y, y_ref, tau_max)


@pytest.mark.parametrize("config,seconds", [(1, 1.0), (2, 2.0)])
def test_gcc_end_to_end(torch, fcc, config, seconds):
    _say(f"GCC end to end config {config}")
    rec = make_recording(config, seconds=seconds)
    p = _plan(fcc, rec, 0, method="gcc")
    t = p.tdoa(_dev(torch, rec.x))
    torch.cuda.synchronize()
    t_ref, y_ref = O.gcc_tdoa(rec.x, rec.N, rec.hop, p.tau_max, return_corr=True)
    rep = tdoa_report(t.cpu().numpy(), y_ref, p.tau_max, EPS32)
    assert rep["mismatch_qualified"] == 0, rep
    assert rep["agreement"] > 0.99, rep


# ------------------------------------------------------------- end to end --

@pytest.mark.parametrize("config,seconds,D", [(1, 1.0, 9), (2, 3.0, 6), (2, 3.0, 11), (3, 1.0, 15)])
def test_end_to_end_fp32(torch, fcc, config, seconds, D):
    _say(f"fcc_tdoa fp32 config {config} {seconds}s D={D}")
    rec = make_recording(config, seconds=seconds)
    p = _plan(fcc, rec, D)
    x = _dev(torch, rec.x)
    t = p.tdoa(x)
    y = p.correlation(p.spectra(x))
    torch.cuda.synchronize()
    t_ref, y_ref = O.fcc_tdoa(rec.x, rec.N, rec.hop, p.tau_max, D, return_corr=True)
    rep = _check_fp32(t.cpu().numpy(), y.cpu().numpy(), y_ref, p.tau_max)
    assert rep["agreement"] > 0.99


def test_config1_planted_delays(torch, fcc):
    _say("fcc_tdoa config 1 planted delays")
    rec = make_recording(1)
    p = _plan(fcc, rec, 9)
    t = p.tdoa(_dev(torch, rec.x)).cpu().numpy()
    expect = np.array([rec.delays[i] - rec.delays[j] for i, j in p.pairs()])
    assert (t == expect[None, :]).mean() > 0.97


def test_full_size_config2_sampled(torch, fcc):
    """The benchmark's workload (60 s, M = 16) in its launch configuration;
    the oracle checks a sample of frames one by one."""
    _say("fcc_tdoa fp32 config 2 full size, sampled frames")
    rec = make_recording(2)
    rng = np.random.default_rng(2024)
    for D in (6, 11):
        p = _plan(fcc, rec, D)
        x = _dev(torch, rec.x)
        t = p.tdoa(x)
        y = p.correlation(p.spectra(x))
        torch.cuda.synchronize()
        T = p.num_frames(rec.L)
        assert tuple(t.shape) == (T, 120)
        frames = np.unique(np.concatenate([[0, T - 1], rng.choice(T, 48, replace=False)]))
        t_ref, y_ref = O.fcc_tdoa(rec.x, rec.N, rec.hop, p.tau_max, D, frames=frames,
                                  return_corr=True)
        _check_fp32(t.cpu().numpy()[frames], y.cpu().numpy()[frames], y_ref, p.tau_max)


def _quantize(packed, precision):
    """Packed FP64 spectra rounded to a storage type on the host (round to
    nearest even), returned as (device tensor in that type, FP64 values)."""
    import torch as _t
    dt = {"fp16": _t.float16, "bf16": _t.bfloat16, "fp8": _t.float8_e4m3fn}[precision]
    q = _t.from_numpy(np.ascontiguousarray(packed, dtype=np.float32)).to(dt)
    return q.cuda().contiguous(), q.to(_t.float64).numpy()


@pytest.fixture(scope="module")
def rec2_full():
    """The benchmark workload (60 s, 16 microphones on a 5 cm circle, 16 kHz,
    N = 512, hop 128: T = 7497 frames, 120 pairs) and its FP64 whitened
    spectra in the packed layout."""
    from paper_2204_13622_amd import Plan
    rec = make_recording(2)
    X = O.stft(rec.x, rec.N, rec.hop)
    packed = Plan.pack_spectrum(O.phat(X))
    del X
    return rec, packed


# bar on the same operands: an operand type of unit roundoff u rounds each
# product p_k e_i and each rotated spectrum value by at most u, so a term of
# the sums errs by at most 2u relative; the FP16 bar (5e-3) is about 5 x 2u,
# and the BF16 and e4m3 bars keep that multiple
SAME_OPERANDS_BAR = {"fp16": 5e-3, "bf16": 2e-2, "fp8": 0.64}


@pytest.mark.parametrize("precision,D,min_agree,max_err,operands", [
    ("fp16", 11, 0.995, 5e-3, "fp16"), ("fp16", 6, 0.995, 5e-3, "fp16"),
    ("bf16", 11, 0.98, 3e-2, "fp16"), ("bf16", 6, 0.98, 3e-2, "fp16"),
    ("fp8", 11, 0.90, 0.3, "fp16"), ("fp8", 6, 0.90, 0.3, "fp16"),
    ("bf16", 11, 0.98, 3e-2, "storage"), ("bf16", 6, 0.98, 3e-2, "storage"),
    ("fp8", 11, 0.85, 0.4, "storage"), ("fp8", 6, 0.85, 0.4, "storage")])
def test_full_size_headline_16bit(torch, fcc, rec2_full, precision, D, min_agree, max_err, operands):
    """The benchmarked call at full size: fcc_tdoa on 60 s of the benchmark
    workload, T = 7497 frames.  The pair stage's persistent grid holds
    2 x CUs workgroups of 4 wavefronts, so every wavefront walks 3-4 frames
    and the next-frame prefetch runs.

    (1) Same operands: the oracle's whitened spectra, rounded to the storage
        type on the host, go through fcc_correlation / fcc_tdoa_from_spectra
        (the launch shape fcc_tdoa uses at this T); sampled frames are compared
        with the FP64 correlation of those rounded spectra at 5e-3, the
        integer lags bit-exact where the top two values are 1e-2 max|y| apart.
    (2) fcc_tdoa on the audio equals fcc_tdoa_from_spectra(fcc_spectra(x))
        on every pair-frame (the same kernels).
    (3) Against the FP64 oracle on the unquantised audio: agreement rate and
        maximum relative correlation error, bounded per storage type."""
    rec, packed = rec2_full
    _say(f"headline full size: config 2, T=7497, {precision}, D={D}, {operands} operands")
    p = _plan(fcc, rec, D, precision=precision, operands=operands)
    bar = SAME_OPERANDS_BAR[precision] if operands == "storage" else 5e-3
    T = p.num_frames(rec.L)
    assert T == 7497 and p.P == 120 and p.I == 11
    rng = np.random.default_rng(2200 + D)
    frames = np.unique(np.concatenate([[0, 1, T - 2, T - 1], rng.choice(T, 60, replace=False)]))
    B = O.fcc_basis(rec.N, p.tau_max, D)

    # (1) same operands
    spec_q, e_q = _quantize(packed, precision)
    y = p.correlation(spec_q)
    t = p.tdoa_from_spectra(spec_q)
    torch.cuda.synchronize()
    assert tuple(y.shape) == (T, 120, 11) and tuple(t.shape) == (T, 120)
    e = fcc.Plan.unpack_spectrum(e_q[frames])
    R = np.stack([e[:, i] * np.conj(e[:, j]) for i, j in O.mic_pairs(16)], axis=1)
    y_ref = O.fcc_corr(R, B)
    y_s, t_s = y.cpu().numpy()[frames], t.cpu().numpy()[frames]
    del y, spec_q
    err = corr_errors(y_s, y_ref)
    rep = tdoa_report(t_s, y_ref, p.tau_max, bar)
    print(f"[same operands {precision} D={D} {operands}] max rel corr err {err.max():.3e}, "
          f"mean {err.mean():.3e}, agreement {rep['agreement']:.5f} ({rep['qualified']} qualified)", flush=True)
    assert err.max() < bar
    assert rep["mismatch_qualified"] == 0, rep
    assert rep["invalid_elsewhere"] == 0, rep

    # (2) the benchmarked entry point runs the same kernels
    x = _dev(torch, rec.x)
    t_full = p.tdoa(x)
    spec = p.spectra(x)
    t_two = p.tdoa_from_spectra(spec)
    y = p.correlation(spec)
    torch.cuda.synchronize()
    assert torch.equal(t_full, t_two)

    # (3) against the FP64 oracle on the unquantised audio
    t_ref, y_ref = O.fcc_tdoa(rec.x, rec.N, rec.hop, p.tau_max, D, frames=frames, return_corr=True)
    y_s, t_s = y.cpu().numpy()[frames], t_full.cpu().numpy()[frames]
    del y, spec
    e = corr_errors(y_s, y_ref)
    rep = tdoa_report(t_s, y_ref, p.tau_max, float(e.max()))
    print(f"[fp64 oracle {precision} D={D} {operands}] agreement {rep['agreement']:.5f} max rel err "
          f"{e.max():.3e} mean {e.mean():.3e}", flush=True)
    assert rep["agreement"] >= min_agree
    assert e.max() <= max_err
    assert rep["mismatch_qualified"] == 0


@pytest.fixture(scope="module")
def rec3():
    return make_recording(3)                   # 120 s, 16 mics, 48 kHz: T = 22497 frames


@pytest.mark.parametrize("precision,D,min_agree,max_err", [
    ("fp32", 15, 1.0, EPS32), ("fp16", 15, 0.995, 5e-3), ("bf16", 15, 0.98, 3e-2),
    ("fp8", 15, 0.90, 0.3), ("fp16", 29, 0.995, 5e-3)])
def test_full_size_config3_sampled(torch, fcc, rec3, precision, D, min_agree, max_err):
    """The mixed-precision workload at full size (120 s at 48 kHz, N = 1024)
    in the launch configuration the library uses for it; the FP64 oracle
    on the unquantised audio checks a sample of frames."""
    _say(f"fcc_tdoa config 3 full size, {precision}, D={D}, sampled frames")
    rec = rec3
    p = _plan(fcc, rec, D, precision=precision)
    x = _dev(torch, rec.x)
    t = p.tdoa(x)
    y = p.correlation(p.spectra(x))
    torch.cuda.synchronize()
    T = p.num_frames(rec.L)
    assert tuple(t.shape) == (T, 120) and T == 22497
    rng = np.random.default_rng(3000 + D)
    frames = np.unique(np.concatenate([[0, T - 1], rng.choice(T, 32, replace=False)]))
    t_ref, y_ref = O.fcc_tdoa(rec.x, rec.N, rec.hop, p.tau_max, D, frames=frames, return_corr=True)
    t_s, y_s = t.cpu().numpy()[frames], y.cpu().numpy()[frames]
    del y
    if precision == "fp32":
        rep = _check_fp32(t_s, y_s, y_ref, p.tau_max)
        print(f"[{precision} D={D}] agreement {rep['agreement']:.5f}", flush=True)
        return
    e = corr_errors(y_s, y_ref)
    rep = tdoa_report(t_s, y_ref, p.tau_max, float(e.max()))
    print(f"[{precision} D={D}] agreement {rep['agreement']:.5f} max rel err {e.max():.3e} "
          f"mean {e.mean():.3e}", flush=True)
    assert rep["agreement"] >= min_agree
    assert e.max() <= max_err
    assert rep["mismatch_qualified"] == 0


# ------------------------------------------------------------- edge cases --

def test_short_and_empty(torch, fcc):
    _say("edge: L < N and L == N")
    p = fcc.Plan(square_array(0.05), 16000.0)
    x = _dev(torch, random_signals(1, 4, 511))
    t = p.tdoa(x)
    assert tuple(t.shape) == (0, 6)
    x = _dev(torch, random_signals(2, 4, 512))
    t = p.tdoa(x).cpu().numpy()
    t_ref, y_ref = O.fcc_tdoa(random_signals(2, 4, 512), 512, 128, p.tau_max, p.rank,
                              return_corr=True)
    _check_fp32(t, None, y_ref, p.tau_max)


def test_zero_and_gated_input(torch, fcc):
    _say("edge: all-zero and gated input")
    p = fcc.Plan(square_array(0.05), 16000.0)
    t = p.tdoa(torch.zeros((4, 4096), device="cuda")).cpu().numpy()
    assert np.all(t == -p.tau_max)              # y == 0: first lag wins
    xg = random_signals(3, 4, 8192, kind="gated")
    t = p.tdoa(_dev(torch, xg)).cpu().numpy()
    t_ref, y_ref = O.fcc_tdoa(xg, 512, 128, p.tau_max, p.rank, return_corr=True)
    _check_fp32(t, None, y_ref, p.tau_max)


def test_row_stride_and_odd_shapes(torch, fcc):
    _say("edge: ld > L, M = 2, 3, 32, N = 256, 2048")
    rng = np.random.default_rng(9)
    for M, N, hop, radius in ((2, 256, 100, 0.03), (3, 512, 128, 0.05), (32, 512, 256, 0.05),
                              (5, 2048, 512, 0.1)):
        xyz = circular_array(M, radius)
        p = fcc.Plan(xyz, 16000.0, frame_size=N, hop=hop)
        L = 3 * N + 37
        big = rng.standard_normal((M, L + 19)).astype(np.float32)
        xt = _dev(torch, big)[:, :L]
        t = p.tdoa(xt).cpu().numpy()
        t_ref, y_ref = O.fcc_tdoa(big[:, :L], N, hop, p.tau_max, p.rank, return_corr=True)
        _check_fp32(t, None, y_ref, p.tau_max)


def test_swap_negates(torch, fcc):
    _say("swap: reversed microphone order negates TDoA")
    rec = make_recording(2, seconds=2.0, M=6)
    p = fcc.Plan(rec.mic_xyz, rec.fs, frame_size=512, hop=128, rank=6)
    q = fcc.Plan(rec.mic_xyz[::-1].copy(), rec.fs, frame_size=512, hop=128, rank=6)
    t1 = p.tdoa(_dev(torch, rec.x)).cpu().numpy()
    t2 = q.tdoa(_dev(torch, rec.x[::-1])).cpu().numpy()
    pr1 = p.pairs()
    idx2 = {pq: k for k, pq in enumerate(q.pairs())}
    M = rec.M
    y_ref = O.fcc_tdoa(rec.x, 512, 128, p.tau_max, 6, return_corr=True)[1]
    rep = tdoa_report(t1, y_ref, p.tau_max, EPS32)
    qual = np.ones_like(t1, dtype=bool)
    s = np.sort(y_ref, -1)
    qual = (s[..., -1] - s[..., -2]) > 2 * EPS32 * np.abs(y_ref).max(-1)
    for k, (i, j) in enumerate(pr1):
        k2 = idx2[(M - 1 - j, M - 1 - i)]
        assert np.all(t1[qual[:, k], k] == -t2[qual[:, k], k2])
    assert rep["mismatch_qualified"] == 0


@pytest.mark.parametrize("delta", [-3, -1, 0, 2, 4])
def test_integer_delay(torch, fcc, delta):
    _say(f"integer delay {delta}")
    x = white_pair(100 + delta, 8192, delta)
    p = fcc.Plan(np.array([[0, 0, 0], [0.1, 0, 0]]), 16000.0)
    t = p.tdoa(_dev(torch, x)).cpu().numpy()
    assert np.all(t[:, 0] == -delta)


def test_deterministic(torch, fcc):
    _say("determinism: repeated runs are bitwise equal")
    rec = make_recording(2, seconds=2.0)
    p = _plan(fcc, rec, 6)
    x = _dev(torch, rec.x)
    spec0 = p.spectra(x)
    y0 = p.correlation(spec0)
    t0 = p.tdoa(x)
    for _ in range(3):
        assert torch.equal(p.spectra(x), spec0)
        assert torch.equal(p.correlation(spec0), y0)
        assert torch.equal(p.tdoa(x), t0)


# ------------------------------------------------------- mixed precision --

@pytest.mark.parametrize("precision,min_agree,max_err", [("bf16", 0.98, 3e-2), ("fp16", 0.995, 5e-3),
                                                         ("fp8", 0.90, 0.3)])
def test_precision_modes(torch, fcc, precision, min_agree, max_err):
    _say(f"precision {precision} config 2, 3 s, D=6")
    rec = make_recording(2, seconds=3.0)
    p = _plan(fcc, rec, 6, precision=precision)
    x = _dev(torch, rec.x)
    t = p.tdoa(x).cpu().numpy()
    y = p.correlation(p.spectra(x)).cpu().numpy()
    t_ref, y_ref = O.fcc_tdoa(rec.x, rec.N, rec.hop, p.tau_max, 6, return_corr=True)
    e = corr_errors(y, y_ref)
    rep = tdoa_report(t, y_ref, p.tau_max, float(e.max()))
    print(f"[{precision}] agreement {rep['agreement']:.5f} max rel err {e.max():.3e} "
          f"mean {e.mean():.3e}", flush=True)
    assert rep["agreement"] >= min_agree
    assert e.max() <= max_err
    assert rep["mismatch_qualified"] == 0


# ------------------------------------------- matrix-core pair stage (16-bit) --

def _quantized_reference(X, dtype_np, B):
    """Oracle correlation of the spectra exactly as the GPU receives them:
    e = X / |X| rounded to the storage type, products formed in FP64."""
    from paper_2204_13622_amd import Plan
    packed = Plan.pack_spectrum(O.phat(X)).astype(dtype_np).astype(np.float64)
    e = Plan.unpack_spectrum(packed)
    pr = O.mic_pairs(e.shape[1])
    R = np.stack([e[:, i] * np.conj(e[:, j]) for i, j in pr], axis=1)
    return packed, O.fcc_corr(R, B)


@pytest.mark.parametrize("config,seconds,D,M", [(2, 1.0, 6, None), (2, 1.0, 11, None),
                                                (3, 0.3, 15, None), (3, 0.3, 29, None),
                                                (5, 1.0, 5, None), (2, 1.0, 9, 5), (1, 1.0, 9, None),
                                                # one, two and three blocks of four microphones
                                                (2, 1.0, 6, 2), (2, 1.0, 6, 3), (2, 0.5, 9, 8), (2, 0.5, 9, 12)])
def test_mfma_pair_stage_fp16(torch, fcc, config, seconds, D, M):
    _say(f"matrix-core pair stage fp16 config {config} D={D} M={M}")
    rec = make_recording(config, seconds=seconds, M=M) if M else make_recording(config, seconds=seconds)
    p = _plan(fcc, rec, D, precision="fp16")
    X = O.stft(rec.x, rec.N, rec.hop)
    B = O.fcc_basis(rec.N, p.tau_max, D)
    packed, y_ref = _quantized_reference(X, np.float16, B)
    spec = torch.from_numpy(packed.astype(np.float16)).cuda().contiguous()
    y = p.correlation(spec).cpu().numpy()
    t = p.tdoa_from_spectra(spec).cpu().numpy()
    e = corr_errors(y, y_ref)
    print(f"fp16 operands: max rel corr err {e.max():.3e}, mean {e.mean():.3e}", flush=True)
    # FP16 operands carry 2^-11 relative rounding; sums over N terms of unit
    # size against a peak of order N keep the relative error near 1e-3
    assert e.max() < 5e-3
    rep = tdoa_report(t, y_ref, p.tau_max, 5e-3)
    assert rep["mismatch_qualified"] == 0, rep
    assert rep["invalid_elsewhere"] == 0, rep


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
@pytest.mark.parametrize("config,seconds,D,M", [(2, 1.0, 6, None), (2, 1.0, 11, 9), (2, 1.0, 6, 2),
                                                (3, 0.3, 15, None), (3, 0.3, 29, 7), (1, 1.0, 9, None)])
def test_native_operand_pair_stage(torch, fcc, precision, config, seconds, D, M):
    """Matrix-core tiles in the storage type (BF16, or e4m3 with per-component
    power-of-two scales) against the FP64 oracle on the same rounded spectra;
    full and partial blocks of four microphones, one to two lag tiles."""
    _say(f"native operands {precision} config {config} D={D} M={M}")
    rec = make_recording(config, seconds=seconds, M=M) if M else make_recording(config, seconds=seconds)
    p = _plan(fcc, rec, D, precision=precision, operands="storage")
    assert p.info.operands == 1
    X = O.stft(rec.x, rec.N, rec.hop)
    B = O.fcc_basis(rec.N, p.tau_max, D)
    from paper_2204_13622_amd import Plan
    spec_q, e_q = _quantize(Plan.pack_spectrum(O.phat(X)), precision)
    e = Plan.unpack_spectrum(e_q)
    R = np.stack([e[:, i] * np.conj(e[:, j]) for i, j in O.mic_pairs(e.shape[1])], axis=1)
    y_ref = O.fcc_corr(R, B)
    y = p.correlation(spec_q).cpu().numpy()
    t = p.tdoa_from_spectra(spec_q).cpu().numpy()
    bar = SAME_OPERANDS_BAR[precision]
    err = corr_errors(y, y_ref)
    print(f"{precision} operands: max rel corr err {err.max():.3e}, mean {err.mean():.3e}", flush=True)
    assert err.max() < bar
    rep = tdoa_report(t, y_ref, p.tau_max, bar)
    assert rep["mismatch_qualified"] == 0, rep
    assert rep["invalid_elsewhere"] == 0, rep


# ------------------------------------------------------- rank and size limits --

# bar: FP32 where the kernel decodes the spectra to FP32 (fold kernel, direct
# form), 5e-3 on the matrix cores
@pytest.mark.parametrize("M,N,tau_max,D,precision,tol", [
    (3, 512, 48, 64, "fp32", EPS32),    # largest rank: the fold kernel with 64 components, I = 97
    (4, 512, 20, 32, "fp16", 5e-3),     # largest matrix-core rank: eight blocks of four, three lag tiles
    (4, 1024, 20, 32, "fp16", EPS32),   # the same at N = 1024 exceeds the matrix-core LDS: the direct form
    (20, 512, 20, 16, "fp16", EPS32),   # more than 16 microphones: the direct form
    (4, 512, 24, 40, "fp16", EPS32),    # rank above 32 and I = 49: the direct form
    (32, 512, 20, 24, "fp16", EPS32),   # 32 microphones: 496 pairs over 256 threads, 78 KB of LDS
    (4, 512, 40, 32, "fp16", EPS32),    # I = 81 > 64 at 16-bit storage: the fold kernel
])
def test_rank_and_size_limits(torch, fcc, M, N, tau_max, D, precision, tol):
    _say(f"limits M={M} N={N} tau_max={tau_max} D={D} {precision}")
    hop = N // 4
    x = random_signals(1400 + M + D, M, N + 40 * hop)
    p = fcc.Plan(circular_array(M, 0.05), 16000.0, frame_size=N, hop=hop, tau_max=tau_max, rank=D,
                 precision=precision)
    X = O.stft(x, N, hop)
    B = O.fcc_basis(N, tau_max, D)
    if precision == "fp32":
        spec = _oracle_spec_tensor(torch, X, torch.float32)
        y_ref = O.fcc_corr(O.phat(O.cross_spectrum(X)), B)
    else:
        packed, y_ref = _quantized_reference(X, np.float16, B)
        spec = torch.from_numpy(packed.astype(np.float16)).cuda().contiguous()
    y = p.correlation(spec).cpu().numpy()
    t = p.tdoa_from_spectra(spec).cpu().numpy()
    assert y.shape == y_ref.shape == (41, p.P, 2 * tau_max + 1)
    e = corr_errors(y, y_ref)
    print(f"max rel corr err {e.max():.3e}", flush=True)
    assert e.max() <= tol
    rep = tdoa_report(t, y_ref, tau_max, tol)
    assert rep["mismatch_qualified"] == 0 and rep["invalid_elsewhere"] == 0, rep


@pytest.mark.parametrize("M,N,tau_max,D", [
    (16, 256, 5, 11),      # the whole frame in one chunk (16.5 KB of bins)
    (16, 512, 5, 11),      # two chunks of folded bins (the benchmark shape)
    (9, 1024, 14, 15),     # two chunks, odd microphone count
    (16, 1024, 14, 15),    # four chunks (the 48 kHz shape)
    (16, 2048, 14, 15),    # four chunks of 128 folded bins each (33 KB)
    (2, 64, 1, 3),         # one pair, one chunk
])
def test_fold_kernel_chunks(torch, fcc, M, N, tau_max, D):
    """FP32 pair stage (the fold kernel) against the oracle on shapes that
    stage the frame's folded bins in one, two and four chunks."""
    _say(f"fold chunks M={M} N={N} tau_max={tau_max} D={D}")
    hop = N // 4
    x = random_signals(1700 + M + N, M, N + 24 * hop)
    p = fcc.Plan(circular_array(M, 0.05), 16000.0, frame_size=N, hop=hop, tau_max=tau_max, rank=D,
                 precision="fp32")
    X = O.stft(x, N, hop)
    spec = _oracle_spec_tensor(torch, X, torch.float32)
    y_ref = O.fcc_corr(O.phat(O.cross_spectrum(X)), O.fcc_basis(N, tau_max, D))
    y = p.correlation(spec).cpu().numpy()
    t = p.tdoa_from_spectra(spec).cpu().numpy()
    assert y.shape == y_ref.shape == (25, p.P, 2 * tau_max + 1)
    rep = _check_fp32(t, y, y_ref, tau_max)
    print(rep, flush=True)


# ------------------------------------------------------ coefficients (eq. 9) --

def _sigma_clusters(sigma, is_sym, rel=1e-6):
    """Components of one parity whose singular values lie within rel sigma_0 of
    their neighbour: inside such a cluster the basis vectors, and with them the
    coefficients, are fixed only up to an orthogonal rotation."""
    groups = []
    for parity in (True, False):
        cur = []
        for k in [k for k in range(len(sigma)) if bool(is_sym[k]) == parity]:
            if cur and sigma[cur[-1]] - sigma[k] > rel * sigma[0]:
                groups.append(cur)
                cur = []
            cur.append(k)
        if cur:
            groups.append(cur)
    return groups


@pytest.mark.parametrize("config,seconds,D,r,precision", [(2, 1.0, 11, 1, "fp32"), (2, 1.0, 6, 1, "fp16"),
                                                          (3, 0.3, 15, 1, "fp32"), (1, 1.0, 9, 2, "fp32")])
def test_coefficients_match_oracle(torch, fcc, config, seconds, D, r, precision):
    """fcc_coefficients against the oracle's z_k (eq. 9) on the same spectra,
    (a_k, b_k) = (Re z_k, Im z_k).  An isolated component must match with its
    sign; a cluster of equal singular values must match after the orthogonal
    rotation that best aligns it (Procrustes).  Bar: per pair-frame within 1e-4
    of max_k |z_k|."""
    _say(f"coefficients config {config} D={D} r={r} {precision}")
    rec = make_recording(config, seconds=seconds)
    p = _plan(fcc, rec, D, interp=r, precision=precision)
    X = O.stft(rec.x, rec.N, rec.hop)
    B = O.fcc_basis(rec.N, p.tau_max, D, r)
    from paper_2204_13622_amd import Plan
    packed = Plan.pack_spectrum(O.phat(X)).astype(np.float16 if precision == "fp16" else np.float32)
    e = Plan.unpack_spectrum(packed.astype(np.float64))
    R = np.stack([e[:, i] * np.conj(e[:, j]) for i, j in O.mic_pairs(p.M)], axis=1)
    z_ref = O.fcc_coefficients(R, B).reshape(-1, D)
    spec = torch.from_numpy(packed).cuda().contiguous()
    c = p.coefficients(spec).cpu().numpy().astype(np.float64)
    assert c.shape == (len(X), p.P, 2 * D)
    z = (c[..., 0::2] + 1j * c[..., 1::2]).reshape(-1, D)
    aligned = np.empty_like(z)
    groups = _sigma_clusters(B.sigma, B.is_sym)
    for g in groups:
        U, _, Vt = np.linalg.svd(np.real(z_ref[:, g].conj().T @ z[:, g]))
        Q = U @ Vt                                         # z[:, g] ~ z_ref[:, g] Q
        if len(g) == 1:
            assert Q[0, 0] == 1.0, g                       # an isolated component keeps its sign
        aligned[:, g] = z[:, g] @ Q.T
    scale = np.abs(z_ref).max(-1)
    err = np.abs(aligned - z_ref).max(-1) / np.where(scale > 0, scale, 1.0)
    print(f"clusters {[len(g) for g in groups]}, max rel coefficient err {err.max():.3e}", flush=True)
    assert err.max() <= EPS32


def test_wrong_outputs_refused(torch, fcc):
    """Caller-supplied outputs and workspaces of the wrong shape, type or size
    are refused on the host, before any launch; correct ones are used."""
    _say("binding: wrong out / workspace refused")
    rec = make_recording(1)
    p = _plan(fcc, rec, 9, precision="fp16")
    x = _dev(torch, rec.x)
    T = p.num_frames(rec.L)
    spec = p.spectra(x)
    bad_outs = [torch.empty((T - 1, p.P), dtype=torch.int32, device="cuda"),
                torch.empty((T, p.P), dtype=torch.int64, device="cuda"),
                torch.empty((p.P, T), dtype=torch.int32, device="cuda").t(),
                torch.empty((T, p.P), dtype=torch.int32)]
    for bad in bad_outs:
        with pytest.raises(ValueError):
            p.tdoa(x, out=bad)
        with pytest.raises(ValueError):
            p.tdoa_from_spectra(spec, out=bad)
    with pytest.raises(ValueError):
        p.tdoa(x, workspace=torch.empty(p.workspace_bytes(T) - 1, dtype=torch.uint8, device="cuda"))
    with pytest.raises(ValueError):
        p.correlation(spec, out=torch.empty((T, p.P, p.I - 1), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        p.spectra(x, out=torch.empty((T, p.M, p.N // 2, 2), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        p.coefficients(spec, out=torch.empty((T, p.P, 2 * p.rank + 2), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        p.tdoa_parabolic(spec, out=torch.empty((T, p.P), dtype=torch.int32, device="cuda"))
    out = torch.full((T, p.P), 99, dtype=torch.int32, device="cuda")
    ws = torch.empty(p.workspace_bytes(T), dtype=torch.uint8, device="cuda")
    assert p.tdoa(x, out=out, workspace=ws) is out
    assert torch.equal(out, p.tdoa_from_spectra(spec))
