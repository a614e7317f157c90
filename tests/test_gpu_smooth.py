"""GPU against the FP64 oracle at the paper's own operating point: the lag grid
of step 1/r (Sec. 3) and recursive cross-spectrum smoothing with alpha < 1
(eq. 1), for FCC, the interpolated lag and the GCC-PHAT comparator."""
import sys

import numpy as np
import pytest

import oracle.fcc_oracle as O
from gen import make_recording, random_signals, circular_array
from tests.parity import corr_errors, tdoa_report

pytestmark = pytest.mark.gpu

EPS32 = 1e-4
PAIR_15CM = np.array([[0.0, 0.0, 0.0], [0.15, 0.0, 0.0]])


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


def _spec(torch, X, dtype):
    from paper_2204_13622_amd import Plan
    return torch.from_numpy(Plan.pack_spectrum(O.phat(X)).astype(np.float32)).cuda().to(dtype).contiguous()


def _two_mic(seed, seconds=1.0, delay=3.5, snr_db=10.0):
    """White source with a fractional delay between two mics, as in the
    paper's pair experiments (x_1[n] = s[n - delay])."""
    from gen import fractional_delay
    rng = np.random.default_rng(seed)
    L = int(16000 * seconds)
    pad = 64
    s = rng.standard_normal(L + 2 * pad)
    x = np.stack([fractional_delay(s, 0.0, pad, L), fractional_delay(s, delay, pad, L)])
    x += rng.standard_normal(x.shape) * np.sqrt(10.0 ** (-snr_db / 10.0))
    return x.astype(np.float32)


# ------------------------------------------------------------------ r > 1 --

@pytest.mark.parametrize("r,D", [(2, 8), (2, 33), (4, 8)])
def test_fcc_interp_fp32(torch, fcc, r, D):
    _say(f"FCC fp32 r={r} D={D}")
    x = _two_mic(700 + r, seconds=1.0)
    p = fcc.Plan(PAIR_15CM, 16000.0, c=335.0, frame_size=512, hop=256, tau_max=8, rank=D, interp=r)
    X = O.stft(x, 512, 256)
    spec = _spec(torch, X, torch.float32)
    y = p.correlation(spec).cpu().numpy()
    t = p.tdoa_from_spectra(spec).cpu().numpy()
    tau = p.tdoa_parabolic(spec).cpu().numpy()
    Rh = O.phat(O.cross_spectrum(X))
    y_ref = O.fcc_corr(Rh, O.fcc_basis(512, 8, D, r))
    e = corr_errors(y, y_ref)
    assert e.max() <= EPS32, e.max()
    rep = tdoa_report(t, y_ref, r * 8, EPS32)
    assert rep["mismatch_qualified"] == 0 and rep["invalid_elsewhere"] == 0, rep
    tau_ref = O.tdoa_parabolic_from_corr(y_ref, 8, r)
    same = t == O.tdoa_from_corr(y_ref, 8, r)
    assert np.abs(tau - tau_ref)[same].max() < 1e-3
    # the delay is 3.5 samples late on mic 1: TDoA_01 = -3.5
    assert abs(np.median(tau) + 3.5) < 0.1


@pytest.mark.parametrize("r", [2, 4])
def test_gcc_interp(torch, fcc, r):
    _say(f"GCC r={r}")
    x = _two_mic(800 + r)
    p = fcc.Plan(PAIR_15CM, 16000.0, c=335.0, frame_size=512, hop=256, tau_max=8, interp=r, method="gcc")
    X = O.stft(x, 512, 256)
    spec = _spec(torch, X, torch.float32)
    y = p.correlation(spec).cpu().numpy()
    t = p.tdoa_from_spectra(spec).cpu().numpy()
    y_ref = O.gcc_corr(O.phat(O.cross_spectrum(X)), 512, 8, r)
    e = corr_errors(y, y_ref)
    assert e.max() <= EPS32, e.max()
    rep = tdoa_report(t, y_ref, r * 8, EPS32)
    assert rep["mismatch_qualified"] == 0 and rep["invalid_elsewhere"] == 0, rep


@pytest.mark.parametrize("M,N,r,tau_max", [(16, 512, 2, 5), (5, 128, 4, 7), (3, 64, 2, 3)])
def test_gcc_interp_shapes(torch, fcc, M, N, r, tau_max):
    _say(f"GCC shapes M={M} N={N} r={r}")
    x = random_signals(900 + M, M, 5 * N)
    p = fcc.Plan(circular_array(M, 0.05), 16000.0, frame_size=N, hop=N // 2, tau_max=tau_max, interp=r,
                 method="gcc")
    X = O.stft(x, N, N // 2)
    spec = _spec(torch, X, torch.float32)
    y = p.correlation(spec).cpu().numpy()
    y_ref = O.gcc_corr(O.phat(O.cross_spectrum(X)), N, tau_max, r)
    assert corr_errors(y, y_ref).max() <= EPS32


def test_fcc_interp_fp16_matrix_cores(torch, fcc):
    """I = 33 needs the third 16-lag tile of the matrix-core pair kernel."""
    _say("FCC fp16 r=2 I=33")
    from paper_2204_13622_amd import Plan
    rec = make_recording(2, seconds=1.0)
    p = fcc.Plan(rec.mic_xyz, rec.fs, frame_size=512, hop=128, tau_max=8, rank=8, interp=2, precision="fp16")
    assert p.I == 33
    X = O.stft(rec.x, 512, 128)
    packed = Plan.pack_spectrum(O.phat(X)).astype(np.float16)
    e = Plan.unpack_spectrum(packed.astype(np.float64))
    R = np.stack([e[:, i] * np.conj(e[:, j]) for i, j in O.mic_pairs(16)], axis=1)
    y_ref = O.fcc_corr(R, O.fcc_basis(512, 8, 8, 2))
    spec = torch.from_numpy(packed).cuda().contiguous()
    y = p.correlation(spec).cpu().numpy()
    t = p.tdoa_from_spectra(spec).cpu().numpy()
    assert corr_errors(y, y_ref).max() < 5e-3
    rep = tdoa_report(t, y_ref, 16, 5e-3)
    assert rep["mismatch_qualified"] == 0 and rep["invalid_elsewhere"] == 0, rep


# -------------------------------------------------------------- alpha < 1 --

def _smoothed_ref(x, N, hop, tau_max, D, r, alpha):
    X = O.stft(x, N, hop)
    Rh = O.phat(O.cross_spectrum(X, alpha))
    return O.fcc_corr(Rh, O.fcc_basis(N, tau_max, D, r))


@pytest.mark.parametrize("case", [
    dict(kind="pair", seconds=2.0, N=512, hop=256, tau_max=8, D=8, r=2, alpha=0.1),     # Table 1 setting
    dict(kind="pair", seconds=1.0, N=512, hop=256, tau_max=8, D=5, r=1, alpha=0.5),
    dict(kind="cfg2", seconds=2.0, N=512, hop=128, tau_max=0, D=11, r=1, alpha=0.1),
    dict(kind="cfg5", seconds=1.0, N=512, hop=128, tau_max=0, D=5, r=2, alpha=0.3),
    dict(kind="small", seconds=0.2, N=32, hop=16, tau_max=3, D=4, r=2, alpha=0.2),
    # every slot count per lane (N/64) and the wide bases, which load a frame in groups
    dict(kind="rand", M=4, seconds=0.3, N=128, hop=64, tau_max=6, D=6, r=2, alpha=0.1),
    dict(kind="rand", M=3, seconds=0.3, N=256, hop=128, tau_max=14, D=30, r=2, alpha=0.4),
    dict(kind="rand", M=3, seconds=1.0, N=1024, hop=512, tau_max=12, D=20, r=1, alpha=0.2),
    dict(kind="rand", M=2, seconds=1.5, N=2048, hop=1024, tau_max=20, D=13, r=1, alpha=0.3),
    dict(kind="rand", M=3, seconds=0.5, N=512, hop=256, tau_max=10, D=17, r=1, alpha=0.25),
    dict(kind="rand", M=3, seconds=0.5, N=512, hop=256, tau_max=9, D=13, r=4, alpha=0.3),   # I = 73: five lag slots
])
def test_smoothed_matches_oracle(torch, fcc, case):
    _say(f"smoothed {case}")
    if case["kind"] == "pair":
        x, xyz, fs = _two_mic(1000 + case["D"], seconds=case["seconds"]), PAIR_15CM, 16000.0
    elif case["kind"] == "small":
        x, xyz, fs = random_signals(1100, 4, int(16000 * case["seconds"])), circular_array(4, 0.02), 16000.0
    elif case["kind"] == "rand":
        M = case["M"]
        x, xyz, fs = random_signals(1200 + case["N"], M, int(16000 * case["seconds"])), circular_array(M, 0.05), 16000.0
    else:
        rec = make_recording(2 if case["kind"] == "cfg2" else 5, seconds=case["seconds"])
        x, xyz, fs = rec.x, rec.mic_xyz, rec.fs
    N, hop, D, r, alpha = case["N"], case["hop"], case["D"], case["r"], case["alpha"]
    p = fcc.Plan(xyz, fs, c=335.0 if case["kind"] == "pair" else 343.0, frame_size=N, hop=hop,
                 tau_max=case["tau_max"], rank=D, interp=r, alpha=alpha)
    xd = _dev(torch, x)
    spec = p.spectra(xd)
    out = p.tdoa_smoothed(spec, tdoa=True, tau=True, y=True)
    t_full = p.tdoa(xd).cpu().numpy()
    torch.cuda.synchronize()
    y_ref = _smoothed_ref(x, N, hop, p.tau_max, D, r, alpha)
    y = out["y"].cpu().numpy()
    e = corr_errors(y, y_ref)
    print(f"smoothed: frames {y.shape[0]}, max rel corr err {e.max():.3e}", flush=True)
    assert e.max() <= EPS32
    t = out["tdoa"].cpu().numpy()
    rep = tdoa_report(t, y_ref, r * p.tau_max, EPS32)
    assert rep["mismatch_qualified"] == 0 and rep["invalid_elsewhere"] == 0, rep
    assert np.array_equal(t_full, t)                       # whole path from audio: same recursion from 0
    same = t == O.tdoa_from_corr(y_ref, p.tau_max, r)
    tau_ref = O.tdoa_parabolic_from_corr(y_ref, p.tau_max, r)
    assert np.abs(out["tau"].cpu().numpy() - tau_ref)[same].max() < 1e-3
    # the returned state is R after the last frame
    X = O.stft(x, N, hop)
    R_last = O.cross_spectrum(X, alpha)[-1]
    st = out["state"].cpu().numpy()
    st = st[..., 0] + 1j * st[..., 1]
    assert np.abs(st - R_last).max() <= 1e-4 * np.abs(R_last).max()


def test_smoothed_streaming_continues_the_recursion(torch, fcc):
    """Two calls sharing the state equal one call over all frames."""
    _say("smoothed streaming")
    rec = make_recording(5, seconds=2.0)
    p = fcc.Plan(rec.mic_xyz, rec.fs, frame_size=512, hop=128, rank=5, interp=2, alpha=0.1)
    spec = p.spectra(_dev(torch, rec.x))
    T = spec.shape[0]
    whole = p.tdoa_smoothed(spec, y=True)
    cut = 97
    first = p.tdoa_smoothed(spec[:cut].contiguous(), y=True)
    second = p.tdoa_smoothed(spec[cut:].contiguous(), state=first["state"], y=True)
    y = np.concatenate([first["y"].cpu().numpy(), second["y"].cpu().numpy()])
    yw = whole["y"].cpu().numpy()
    assert y.shape[0] == T
    assert corr_errors(y, yw).max() < 1e-5
    assert np.abs(second["state"].cpu().numpy() - whole["state"].cpu().numpy()).max() <= \
        1e-5 * np.abs(whole["state"].cpu().numpy()).max()


def test_smoothed_short_calls(torch, fcc):
    """Calls of 1, 2, 9 and 17 frames (one chunk, two chunks with a shorter
    tail, three chunks) carrying the state between them reproduce the oracle's
    single recursion over all frames."""
    _say("smoothed short calls")
    M, N, hop = 4, 512, 128
    x = random_signals(1300, M, N + 59 * hop)
    p = fcc.Plan(circular_array(M, 0.05), 16000.0, frame_size=N, hop=hop, rank=8, interp=2, alpha=0.2)
    spec = p.spectra(_dev(torch, x))
    T = spec.shape[0]
    assert T == 60
    state, ys, ts, t0 = None, [], [], 0
    for n in (1, 1, 2, 9, 17, 5, T - 35):
        out = p.tdoa_smoothed(spec[t0:t0 + n].contiguous(), state=state, y=True)
        state = out["state"]
        ys.append(out["y"].cpu().numpy())
        ts.append(out["tdoa"].cpu().numpy())
        t0 += n
    y, t = np.concatenate(ys), np.concatenate(ts)
    y_ref = _smoothed_ref(x, N, hop, p.tau_max, 8, 2, 0.2)
    assert y.shape == y_ref.shape
    assert corr_errors(y, y_ref).max() <= EPS32
    rep = tdoa_report(t, y_ref, 2 * p.tau_max, EPS32)
    assert rep["mismatch_qualified"] == 0 and rep["invalid_elsewhere"] == 0, rep
    R_last = O.cross_spectrum(O.stft(x, N, hop), 0.2)[-1]
    st = state.cpu().numpy()
    assert np.abs(st[..., 0] + 1j * st[..., 1] - R_last).max() <= 1e-4 * np.abs(R_last).max()


def test_smoothed_errors(torch, fcc):
    p = fcc.Plan(PAIR_15CM, 16000.0, frame_size=512, hop=256, tau_max=8, rank=8, interp=2, alpha=0.1)
    spec = p.spectra(_dev(torch, _two_mic(1)))
    with pytest.raises(fcc.FccError) as ei:
        p.tdoa_from_spectra(spec)                          # alpha < 1 runs through the smoothed entry
    assert ei.value.name == "FCC_ERR_UNSUPPORTED"
    q = fcc.Plan(PAIR_15CM, 16000.0, frame_size=512, hop=256, tau_max=8, rank=8)
    with pytest.raises(fcc.FccError):
        q.tdoa_smoothed(q.spectra(_dev(torch, _two_mic(1))))
    out = p.tdoa_smoothed(spec[:0])                        # no frames: nothing to do, state untouched
    assert out["tdoa"].shape == (0, 1) and float(out["state"].abs().max()) == 0.0
    # rank above 32: outside the smoothing kernels, refused before any launch
    w = fcc.Plan(PAIR_15CM, 16000.0, frame_size=512, hop=256, tau_max=24, rank=40, alpha=0.1)
    with pytest.raises(fcc.FccError) as ei:
        w.tdoa_smoothed(w.spectra(_dev(torch, _two_mic(2))))
    assert ei.value.name == "FCC_ERR_UNSUPPORTED"
