"""Batches of heterogeneous arrays on the GPU: every array's output equals the
single-array path bit for bit (same kernels, same arithmetic), with and
without the graph, after autotuning, and on repeated graph replays."""
import sys

import numpy as np
import pytest

import oracle.fcc_oracle as O
from gen import batch_arrays
from tests.parity import tdoa_report, corr_errors

pytestmark = pytest.mark.gpu


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


def _plans(fcc, arrays, precision):
    out = []
    for a in arrays:
        p0 = fcc.Plan(a["xyz"], a["fs"], frame_size=a["N"], hop=a["hop"], precision=precision)
        out.append(fcc.Plan(a["xyz"], a["fs"], frame_size=a["N"], hop=a["hop"], rank=p0.tau_max + 1,
                            precision=precision))
    return out


@pytest.mark.parametrize("precision,count,seconds", [("fp16", 24, 0.3), ("bf16", 9, 0.2)])
def test_batch_equals_single_arrays(torch, fcc, precision, count, seconds):
    _say(f"batch {precision} {count} arrays")
    arrays = batch_arrays(4100 + count, count, seconds)
    plans = _plans(fcc, arrays, precision)
    b = fcc.Batch(plans, [a["x"].shape[1] for a in arrays])
    audio = b.pack([torch.from_numpy(a["x"]) for a in arrays])
    expect = [p.tdoa(torch.from_numpy(a["x"]).cuda()).cpu().numpy() for p, a in zip(plans, arrays)]
    for graph in (False, True):
        got = [t.cpu().numpy().copy() for t in b.split(b.tdoa(audio, graph=graph))]
        for a, (g, e) in enumerate(zip(got, expect)):
            assert np.array_equal(g, e), (graph, a)
    tuned = b.tune(audio)
    print("tuning:", tuned, flush=True)
    assert len(tuned["pair_classes"]) == b.info.num_classes
    # graph replays with eager work of the same library in between
    for rep in range(3):
        out = b.tdoa(audio, graph=True)
        plans[rep].tdoa(torch.from_numpy(arrays[rep]["x"]).cuda())
        torch.cuda.synchronize()
        for a, (g, e) in enumerate(zip(b.split(out), expect)):
            assert np.array_equal(g.cpu().numpy(), e), (rep, a)


def test_batch_against_oracle(torch, fcc):
    """Two arrays of the batch through the FP64 oracle on the same quantised spectra."""
    _say("batch vs oracle")
    from paper_2204_13622_amd import Plan
    arrays = batch_arrays(4200, 6, 0.25)
    plans = _plans(fcc, arrays, "fp16")
    b = fcc.Batch(plans, [a["x"].shape[1] for a in arrays])
    out = b.split(b.tdoa(b.pack([torch.from_numpy(a["x"]) for a in arrays])))
    for a in (0, 3):
        p, x = plans[a], arrays[a]["x"]
        spec = p.spectra(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
        e = Plan.unpack_spectrum(spec)
        R = np.stack([e[:, i] * np.conj(e[:, j]) for i, j in O.mic_pairs(p.M)], axis=1)
        y_ref = O.fcc_corr(R, O.fcc_basis(p.N, p.tau_max, p.rank))
        rep = tdoa_report(out[a].cpu().numpy(), y_ref, p.tau_max, 5e-3)
        assert rep["mismatch_qualified"] == 0 and rep["invalid_elsewhere"] == 0, rep


def test_batch_short_and_empty_arrays(torch, fcc):
    """Arrays with no frame (shorter than the frame size, or no samples), one
    frame and two frames beside whole ones: the whole arrays equal the
    single-array path and the empty ones have no output.  A batch in which no
    array has a frame runs and tunes as a no-op."""
    _say("batch with short and empty arrays")
    arrays = batch_arrays(4300, 6, 0.25)
    plans = _plans(fcc, arrays, "fp16")
    N = [a["N"] for a in arrays]
    hop = [a["hop"] for a in arrays]
    lengths = [N[0] - 1, N[1], N[2] + hop[2], 0, arrays[4]["x"].shape[1], arrays[5]["x"].shape[1]]
    xs = [np.ascontiguousarray(a["x"][:, :L]) for a, L in zip(arrays, lengths)]
    b = fcc.Batch(plans, lengths)
    assert b.frames[:4] == [0, 1, 2, 0]
    audio = b.pack([torch.from_numpy(x) for x in xs])
    for graph in (False, True, True):
        out = [t.cpu().numpy().copy() for t in b.split(b.tdoa(audio, graph=graph))]
        for a, (p, x) in enumerate(zip(plans, xs)):
            if b.frames[a] == 0:
                assert out[a].shape == (0, p.P), a
            else:
                assert np.array_equal(out[a], p.tdoa(torch.from_numpy(x).cuda()).cpu().numpy()), (graph, a)
    empty = fcc.Batch(plans[:2], [N[0] - 1, 5])
    assert empty.info.tdoa_count == 0
    audio = empty.pack([torch.from_numpy(np.ascontiguousarray(arrays[0]["x"][:, :N[0] - 1])),
                        torch.from_numpy(np.ascontiguousarray(arrays[1]["x"][:, :5]))])
    for graph in (False, True):
        parts = empty.split(empty.tdoa(audio, graph=graph))
        assert [tuple(t.shape) for t in parts] == [(0, plans[0].P), (0, plans[1].P)]
    assert len(empty.tune(audio)["pair_classes"]) == empty.info.num_classes
    torch.cuda.synchronize()


def test_batch_wide_tiles(torch, fcc):
    """Classes of three lag tiles (I = 41, 47) and six or eight blocks of four
    components (ranks 20-32), two arrays sharing one class, beside narrow
    ones: every array equals the single-array path bit for bit.  A class
    whose tables and two wavefront slabs exceed the LDS is refused at
    creation."""
    _say("batch with wide tiles")
    from gen import circular_array, random_signals
    too_big = fcc.Plan(circular_array(4, 0.05), 16000.0, frame_size=1024, hop=256, tau_max=20, rank=32,
                       precision="fp16")
    with pytest.raises(fcc.FccError) as ei:
        fcc.Batch([too_big], [4800])
    assert ei.value.name == "FCC_ERR_UNSUPPORTED"
    shapes = [(4, 512, 20, 32), (5, 512, 20, 30), (6, 512, 20, 24), (3, 1024, 23, 20), (8, 512, 10, 12),
              (16, 256, 5, 6)]
    plans, xs = [], []
    for k, (M, N, tau_max, D) in enumerate(shapes):
        plans.append(fcc.Plan(circular_array(M, 0.05), 16000.0, frame_size=N, hop=N // 4, tau_max=tau_max,
                              rank=D, precision="fp16"))
        xs.append(random_signals(4400 + k, M, 4800 + 37 * k))
    b = fcc.Batch(plans, [x.shape[1] for x in xs])
    assert b.info.num_classes == 5
    audio = b.pack([torch.from_numpy(x) for x in xs])
    expect = [p.tdoa(torch.from_numpy(x).cuda()).cpu().numpy() for p, x in zip(plans, xs)]
    for graph in (False, True):
        for a, (g, e) in enumerate(zip(b.split(b.tdoa(audio, graph=graph)), expect)):
            assert np.array_equal(g.cpu().numpy(), e), (graph, a)
    b.tune(audio)
    for a, (g, e) in enumerate(zip(b.split(b.tdoa(audio, graph=True)), expect)):
        assert np.array_equal(g.cpu().numpy(), e), ("tuned", a)


def test_batch_full_scale(torch, fcc):
    """The batched workload at its stated scale: 256 arrays x 10 s (M 2-16,
    2-10 cm, 16 / 48 kHz, N 256 / 512 / 1024, rank tau_max + 1), autotuned,
    graph-captured.  Every array's lags equal the single-array path bit for
    bit; four arrays spanning the frame sizes and both rates are checked
    against the FP64 oracle on sampled frames: the single-array path's
    correlation y on the same FP16 spectra within 5e-3, and the batch's lags
    bit-exact where the top two values are 1e-2 max|y| apart; and the batch's
    own lags against the FP64 oracle on the raw audio."""
    _say("batch full scale: 256 arrays x 10 s")
    from paper_2204_13622_amd import Plan
    arrays = batch_arrays(4000, 256, 10.0)
    plans = _plans(fcc, arrays, "fp16")
    b = fcc.Batch(plans, [a["x"].shape[1] for a in arrays])
    audio = b.pack([torch.from_numpy(a["x"]) for a in arrays])
    units = sum(T * p.P for T, p in zip(b.frames, plans))
    b.tune(audio)
    out = [t.cpu().numpy().copy() for t in b.split(b.tdoa(audio, graph=True))]
    del audio
    print(f"{units} pair-frames in {b.info.num_classes} classes", flush=True)
    picks = {}
    for a, (arr, p) in enumerate(zip(arrays, plans)):
        x = torch.from_numpy(arr["x"]).cuda()
        assert np.array_equal(out[a], p.tdoa(x).cpu().numpy()), a
        picks.setdefault((arr["N"], arr["fs"]), a)
    chosen = sorted(picks.values())
    assert len({arrays[a]["N"] for a in chosen}) == 3 and len({arrays[a]["fs"] for a in chosen}) == 2
    rng = np.random.default_rng(4001)
    for a in chosen[:6]:
        p, x = plans[a], arrays[a]["x"]
        T = b.frames[a]
        frames = np.unique(np.concatenate([[0, T - 1], rng.choice(T, 16, replace=False)]))
        X = O.stft(x, p.N, p.hop, frames=frames)
        packed = Plan.pack_spectrum(O.phat(X)).astype(np.float16)
        e = Plan.unpack_spectrum(packed.astype(np.float64))
        R = np.stack([e[:, i] * np.conj(e[:, j]) for i, j in O.mic_pairs(p.M)], axis=1)
        y_ref = O.fcc_corr(R, O.fcc_basis(p.N, p.tau_max, p.rank))
        y = p.correlation(torch.from_numpy(packed).cuda().contiguous()).cpu().numpy()
        err = corr_errors(y, y_ref)
        rep = tdoa_report(p.tdoa_from_spectra(torch.from_numpy(packed).cuda().contiguous()).cpu().numpy(),
                          y_ref, p.tau_max, 5e-3)
        print(f"array {a}: M={p.M} N={p.N} fs={arrays[a]['fs']:.0f} D={p.rank} "
              f"max rel corr err {err.max():.2e}, qualified {rep['qualified']}", flush=True)
        assert err.max() < 5e-3
        assert rep["mismatch_qualified"] == 0 and rep["invalid_elsewhere"] == 0, rep
        # the batch's own lags (its own front end) against the FP64 oracle on
        # the raw audio, at the error the single-array correlation shows there
        y64 = O.fcc_corr(O.phat(O.cross_spectrum(X)), O.fcc_basis(p.N, p.tau_max, p.rank))
        y_gpu = p.correlation(p.spectra(torch.from_numpy(x).cuda())).cpu().numpy()[frames]
        e64 = corr_errors(y_gpu, y64)
        rep_b = tdoa_report(out[a][frames], y64, p.tau_max, float(e64.max()))
        assert e64.max() < 5e-3
        assert rep_b["mismatch_qualified"] == 0, rep_b
