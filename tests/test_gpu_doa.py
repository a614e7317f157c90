"""DoA search on the GPU against the FP64 oracle (oracle/doa_oracle.py), on the
same correlations, and end to end from audio."""
import sys

import numpy as np
import pytest

import oracle.doa_oracle as DO
from gen import circular_array, fractional_delay, sphere_grid, random_signals

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


def _xyz3d(M=6):
    return np.vstack([circular_array(M, 0.05), [[0.0, 0.0, 0.05]]])


def _plane_wave(xyz, u, fs=16000.0, c=343.0, seconds=0.5, seed=3, snr_db=20.0):
    rng = np.random.default_rng(seed)
    L = int(fs * seconds)
    pad = 64
    s = rng.standard_normal(L + 2 * pad)
    d = -(np.asarray(xyz) @ u) * fs / c
    x = np.stack([fractional_delay(s, dm, pad, L) for dm in d])
    x += rng.standard_normal(x.shape) * np.sqrt(10.0 ** (-snr_db / 10.0))
    return x.astype(np.float32)


def _check_scores(doa, score, y, q):
    idx_ref, s_ref = DO.doa_search(y, q)
    tol = 1e-5 * np.abs(y).max(-1).sum(-1, keepdims=True) + 1e-6       # per frame: sum over pairs of max|y|
    assert np.all(np.abs(score - s_ref) <= tol)
    srt = np.sort(s_ref, axis=-1)
    gap = srt[:, -1] - srt[:, -2] if s_ref.shape[1] > 1 else np.full(len(s_ref), np.inf)
    qualified = gap > 2 * tol[:, 0]
    assert np.array_equal(doa[qualified], idx_ref[qualified])
    # elsewhere the chosen direction is within the tolerance of the best
    chosen = np.take_along_axis(s_ref, doa[:, None].astype(np.int64), 1)[:, 0]
    assert np.all(chosen >= srt[:, -1] - 2 * tol[:, 0])


@pytest.mark.parametrize("G,M,r,seconds", [(512, 6, 2, 0.5), (1000, 6, 1, 0.37), (200, 16, 1, 0.3),
                                           (77, 31, 2, 0.2),
                                           (1, 6, 1, 0.2),         # one direction: always index 0
                                           (2600, 6, 2, 0.21)])    # eleven lane rounds, the last partial
def test_doa_scores_match_oracle(torch, fcc, G, M, r, seconds):
    _say(f"DoA parity G={G} M={M} r={r}")
    xyz = _xyz3d(M)
    dirs = sphere_grid(G)
    x = _plane_wave(xyz, dirs[G // 3], seconds=seconds)
    p = fcc.Plan(xyz, 16000.0, frame_size=512, hop=128, rank=0, interp=r)
    y = p.correlation(p.spectra(torch.from_numpy(x).cuda()))
    table = p.doa_table(dirs)
    doa, score = p.doa(y, table, score=True)
    doa_only, _ = p.doa(y, table)
    q = DO.lag_positions(xyz, dirs, 16000.0, 343.0, p.tau_max, r)
    _check_scores(doa.cpu().numpy(), score.cpu().numpy(), y.cpu().numpy().astype(np.float64), q)
    assert np.array_equal(doa.cpu().numpy(), doa_only.cpu().numpy())


def test_doa_end_to_end_direction(torch, fcc):
    _say("DoA end to end")
    xyz = _xyz3d()
    dirs = sphere_grid(512)
    p = fcc.Plan(xyz, 16000.0, frame_size=512, hop=128, rank=8, interp=2)
    table = p.doa_table(dirs)
    for k in (37, 150, 401):
        x = _plane_wave(xyz, dirs[k], seed=k)
        doa, _ = p.doa(p.correlation(p.spectra(torch.from_numpy(x).cuda())), table)
        ang = np.degrees(np.arccos(np.clip(dirs[doa.cpu().numpy()] @ dirs[k], -1, 1)))
        assert np.median(ang) < 12.0, (k, np.median(ang))


def test_doa_planar_mirror_ties_take_the_first_index(torch, fcc):
    """A planar array cannot tell z from -z: mirrored directions score exactly
    alike and the first index wins."""
    _say("DoA mirror ties")
    xyz = circular_array(8, 0.05)
    up = sphere_grid(64, upper=True)
    dirs = np.concatenate([up, up * np.array([1.0, 1.0, -1.0])])
    p = fcc.Plan(xyz, 16000.0, frame_size=512, hop=128, rank=0)
    x = random_signals(5, 8, 16000 // 4)
    y = p.correlation(p.spectra(torch.from_numpy(x).cuda()))
    doa, score = p.doa(y, p.doa_table(dirs), score=True)
    s = score.cpu().numpy()
    assert np.array_equal(s[:, :64], s[:, 64:])
    assert np.all(doa.cpu().numpy() < 64)


def test_doa_on_smoothed_correlations(torch, fcc):
    _say("DoA smoothed")
    xyz = _xyz3d()
    dirs = sphere_grid(256)
    p = fcc.Plan(xyz, 16000.0, frame_size=512, hop=256, rank=8, interp=2, alpha=0.2)
    x = _plane_wave(xyz, dirs[77], seconds=1.0)
    y = p.tdoa_smoothed(p.spectra(torch.from_numpy(x).cuda()), tdoa=False, y=True)["y"]
    doa, _ = p.doa(y, p.doa_table(dirs))
    ang = np.degrees(np.arccos(np.clip(dirs[doa.cpu().numpy()[5:]] @ dirs[77], -1, 1)))
    assert np.median(ang) < 12.0


def test_doa_errors(torch, fcc):
    p = fcc.Plan(_xyz3d(), 16000.0, frame_size=512, hop=128)
    table = p.doa_table(sphere_grid(10))
    y = torch.zeros((0, p.P, p.I), dtype=torch.float32, device="cuda")
    doa, _ = p.doa(y, table)
    assert doa.shape == (0,)
    with pytest.raises(ValueError):
        p.doa(torch.zeros((3, p.P, p.I + 1), device="cuda"), table)
