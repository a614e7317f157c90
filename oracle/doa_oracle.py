"""FP64 reference of the direction-of-arrival search over all pairs (test
infrastructure: only the test-suite imports this module).

The paper's conclusion names the next step: TDoAs of every pair of an array
feeding a search over DoA candidates.  The search here is the steered
response of the pairwise correlations:

    for a unit direction u, the far-field arrival time at mic m is -(r_m . u) / c,
    so pair (i, j) sees tau_ij(u) = (r_j - r_i) . u  f_S / c  samples
    (TDoA_ij = t_i - t_j, the sign convention of the correlation);
    its position on the lag grid tau_k = k / r - tau_max is
    q_ij(u) = r tau_ij(u) + r tau_max, clipped to [0, I - 1];
    score(u) = sum over pairs of y_ij at q_ij(u), linearly interpolated
    between the two neighbouring grid lags;
    DoA = the first direction of largest score.
"""
from __future__ import annotations

import numpy as np

from .fcc_oracle import mic_pairs


def lag_positions(mic_xyz, dirs, fs: float, c: float, tau_max: int, r: int = 1) -> np.ndarray:
    """q [P, G]: fractional lag-grid index of every pair for every direction."""
    xyz = np.asarray(mic_xyz, dtype=np.float64)
    u = np.asarray(dirs, dtype=np.float64)
    I = 2 * r * tau_max + 1
    q = np.empty((len(mic_pairs(xyz.shape[0])), u.shape[0]))
    for p, (i, j) in enumerate(mic_pairs(xyz.shape[0])):
        tau = (u @ (xyz[j] - xyz[i])) * fs / c
        q[p] = np.clip(r * tau + r * tau_max, 0.0, I - 1)
    return q


def interp_lag(y, q) -> np.ndarray:
    """y [..., I] read at fractional indices q [G] by linear interpolation: [..., G]."""
    y = np.asarray(y, dtype=np.float64)
    I = y.shape[-1]
    i0 = np.minimum(np.floor(q).astype(np.int64), max(I - 2, 0))
    w = q - i0
    if I == 1:
        return np.repeat(y[..., :1], q.size, axis=-1)
    return (1.0 - w) * y[..., i0] + w * y[..., i0 + 1]


def srp_scores(y, q) -> np.ndarray:
    """score [T, G] = sum over pairs of the interpolated correlation; y [T, P, I], q [P, G]."""
    y = np.asarray(y, dtype=np.float64)
    s = np.zeros((y.shape[0], q.shape[1]))
    for p in range(y.shape[1]):
        s += interp_lag(y[:, p, :], q[p])
    return s


def doa_search(y, q):
    """(index [T] of the first best direction, scores [T, G])."""
    s = srp_scores(y, q)
    return np.argmax(s, axis=-1).astype(np.int32), s
