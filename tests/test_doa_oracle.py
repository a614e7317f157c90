"""Pins of the FP64 DoA search (oracle/doa_oracle.py) to geometry and to
closed forms, with planted mistakes that the pins must catch."""
import numpy as np
import pytest

import oracle.doa_oracle as DO
import oracle.fcc_oracle as O
from gen import circular_array, fractional_delay, sphere_grid


def _plane_wave(xyz, u, fs, c, seconds=0.5, seed=3):
    """White source from direction u: mic m hears s(t + (r_m . u) / c)."""
    rng = np.random.default_rng(seed)
    L = int(fs * seconds)
    pad = 64
    s = rng.standard_normal(L + 2 * pad)
    d = -(np.asarray(xyz) @ u) * fs / c                     # arrival delays in samples
    return np.stack([fractional_delay(s, dm, pad, L) for dm in d])


def _angle_deg(a, b):
    return np.degrees(np.arccos(np.clip(np.dot(a, b) / np.linalg.norm(a) / np.linalg.norm(b), -1, 1)))


def _search(xyz, dirs, x, fs, c, N=512, hop=256, r=2, lag_positions=DO.lag_positions):
    tm = O.tau_max_from_geometry(xyz, fs, c)
    y = O.gcc_corr(O.pipeline_spectra(x, N, hop), N, tm, r)
    q = lag_positions(xyz, dirs, fs, c, tm, r)
    return DO.doa_search(y, q)


def _xyz3d():
    # a non-planar array: the circle plus one raised mic, so up and down differ
    return np.vstack([circular_array(6, 0.05), [[0.0, 0.0, 0.05]]])


@pytest.mark.parametrize("k", [37, 150, 401])
def test_plane_wave_direction_found(k):
    xyz, fs, c = _xyz3d(), 16000.0, 343.0
    dirs = sphere_grid(512)
    idx, s = _search(xyz, dirs, _plane_wave(xyz, dirs[k], fs, c), fs, c)
    assert np.median([_angle_deg(dirs[i], dirs[k]) for i in idx]) < 12.0


def test_linear_correlation_is_interpolated_exactly():
    xyz, fs, c, tm, r = circular_array(4, 0.05), 16000.0, 343.0, 3, 2
    dirs = sphere_grid(64)
    q = DO.lag_positions(xyz, dirs, fs, c, tm, r)
    I = 2 * r * tm + 1
    a, b = np.array([0.3, -1.0, 2.0, 0.5, -0.2, 1.5]), np.array([1.0, 2.0, -3.0, 0.0, 4.0, 0.5])
    y = (a[:, None] * np.arange(I)[None, :] + b[:, None])[None]       # [1, P, I]
    assert np.allclose(DO.srp_scores(y, q)[0], (a[:, None] * q + b[:, None]).sum(0), atol=1e-12)


def test_delta_at_exact_lags_scores_P():
    # lags that land on grid points: a pair along x and a direction along x
    xyz = np.array([[0.0, 0, 0], [0.0686, 0, 0], [0, 0.0686, 0]])    # 0.0686 m = 3.2 samples at 16 kHz / 343 m/s
    fs, c, r = 16000.0, 343.0, 5
    tm = 4
    u = np.array([[1.0, 0, 0], [0, 1.0, 0], [-1.0, 0, 0]])
    q = DO.lag_positions(xyz, u, fs, c, tm, r)
    assert np.allclose(q, np.rint(q), atol=1e-9)
    I = 2 * r * tm + 1
    y = np.zeros((1, 3, I))
    for p in range(3):
        y[0, p, int(round(q[p, 0]))] = 1.0
    idx, s = DO.doa_search(y, q)
    assert idx[0] == 0 and abs(s[0, 0] - 3.0) < 1e-9 and s[0, 1] < 2.0 and s[0, 2] < 2.0


def test_relabelled_mics_give_the_same_scores():
    xyz, fs, c, r = _xyz3d(), 16000.0, 343.0, 2
    dirs = sphere_grid(128)
    x = _plane_wave(xyz, dirs[5], fs, c)
    tm = O.tau_max_from_geometry(xyz, fs, c)
    y = O.gcc_corr(O.pipeline_spectra(x, 512, 256), 512, tm, r)
    s = DO.srp_scores(y, DO.lag_positions(xyz, dirs, fs, c, tm, r))
    perm = np.arange(xyz.shape[0])[::-1]                   # reversed labels: every pair swaps its ends
    y2 = O.gcc_corr(O.pipeline_spectra(x[perm], 512, 256), 512, tm, r)
    s2 = DO.srp_scores(y2, DO.lag_positions(xyz[perm], dirs, fs, c, tm, r))
    assert np.allclose(s, s2, rtol=1e-9, atol=1e-9 * np.abs(s).max())


# ---------------------------------------------------------- planted mistakes --

def _positions_wrong_sign(xyz, dirs, fs, c, tm, r=1):
    return DO.lag_positions(-np.asarray(xyz), dirs, fs, c, tm, r)


def _positions_no_offset(xyz, dirs, fs, c, tm, r=1):
    return np.clip(DO.lag_positions(xyz, dirs, fs, c, tm, r) - r * tm, 0, 2 * r * tm)


def test_planted_wrong_sign_is_caught():
    xyz, fs, c = _xyz3d(), 16000.0, 343.0
    dirs = sphere_grid(512)
    idx, _ = _search(xyz, dirs, _plane_wave(xyz, dirs[37], fs, c), fs, c, lag_positions=_positions_wrong_sign)
    assert np.median([_angle_deg(dirs[i], dirs[37]) for i in idx]) > 12.0


def test_planted_missing_offset_is_caught():
    xyz, fs, c = _xyz3d(), 16000.0, 343.0
    dirs = sphere_grid(512)
    idx, _ = _search(xyz, dirs, _plane_wave(xyz, dirs[150], fs, c), fs, c, lag_positions=_positions_no_offset)
    assert np.median([_angle_deg(dirs[i], dirs[150]) for i in idx]) > 12.0


def test_planted_nearest_neighbour_is_caught():
    q = np.array([0.25, 1.5, 2.75])
    y = np.arange(4.0)[None] * 2.0
    nearest = y[..., np.rint(q).astype(int)]
    assert not np.allclose(nearest, 2.0 * q)
    assert np.allclose(DO.interp_lag(y, q), 2.0 * q)
