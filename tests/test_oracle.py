"""The FP64 oracle against its pins (CPU only), plus planted-mistake checks
showing that each pin family catches a plausible error in the oracle."""
import numpy as np
import pytest

import oracle.fcc_oracle as O
from tests import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(O)


def test_basis_svd_other_shapes():
    P.pin_basis_svd(O, N=1024, tm=14, r=1)
    P.pin_basis_svd(O, N=512, tm=8, r=2)
    P.pin_basis_symmetry(O, N=1024, tm=14, D=15)
    P.pin_basis_symmetry(O, N=512, tm=8, D=8, r=2)
    P.pin_dictionary_parity(O, N=512, tm=4, D=9)


@pytest.mark.parametrize("D", [None, "half"])
def test_integer_delay_fcc(D):
    def fn(x):
        tm = 5
        rank = 2 * tm + 1 if D is None else tm + 1
        return O.fcc_tdoa(x, 512, 128, tm, rank)
    P.pin_integer_delay(O, fn)


def test_integer_delay_gcc():
    P.pin_integer_delay(O, lambda x: O.gcc_tdoa(x, 512, 128, 5))


def test_ambiguous_cut_refused():
    # N = 1024, tau_max = 14: the two largest symmetric values differ by ~1e-14
    with pytest.raises(O.BasisAmbiguous):
        O.fcc_basis(1024, 14, 1)
    with pytest.raises(O.BasisAmbiguous):
        O.fcc_basis(1024, 14, 3)
    O.fcc_basis(1024, 14, 15)
    O.fcc_basis(1024, 14, 29)


def test_geometry_tau_max():
    from gen import make_recording, circular_array, square_array
    assert O.tau_max_from_geometry(square_array(0.05), 16000, 343.0) == 4
    assert O.tau_max_from_geometry(circular_array(16, 0.05), 16000, 343.0) == 5
    assert O.tau_max_from_geometry(circular_array(16, 0.05), 48000, 343.0) == 14
    assert O.tau_max_from_geometry(circular_array(8, 0.04), 16000, 343.0) == 4
    r = make_recording(1)
    assert O.tau_max_from_geometry(r.mic_xyz, r.fs, r.c) == 4


def test_config1_recovers_planted_delays():
    from gen import make_recording
    r = make_recording(1)
    t = O.fcc_tdoa(r.x, r.N, r.hop, 4, 9)
    expect = np.array([r.delays[i] - r.delays[j] for i, j in O.mic_pairs(4)])
    assert t.shape == (122, 6)
    assert (t == expect[None, :]).mean() > 0.97


# ------------------------------------------------------- planted mistakes ---

def _fold_wrong_sign(Rhat, N):
    s, d, c = ORIG["fold"](Rhat, N)
    return s, s, c


def _fold_no_centre(Rhat, N):
    s, d, c = ORIG["fold"](Rhat, N)
    return s, d, 0 * c


def _expand_wrong_sign(z, B):
    return 2.0 * (z.real @ B.Dc.T + z.imag @ B.Ds.T)


def _cross_conj_swapped(X, alpha=1.0):
    return np.conj(ORIG["cross_spectrum"](X, alpha))


def _phat_unnormalised(R):
    return np.asarray(R, dtype=np.complex128)


def _window_symmetric(N):
    n = np.arange(N)
    return 0.5 - 0.5 * np.cos(2 * np.pi * n / (N - 1))


def _gcc_irfft(Rhat, N, tau_max, r=1):
    # textbook inverse real FFT: DC and Nyquist weighted once, unlike eq. (2)
    s = np.fft.irfft(Rhat, n=r * N, axis=-1) * (r * N)
    n = np.rint(O.lag_grid(tau_max, r) * r).astype(np.int64) % (r * N)
    return s[..., n]


def _basis_cut_off_by_one(N, tau_max, D, r=1, gap_tol=1e-9):
    # keeps components 1 .. D-1 and D+1 instead of 1 .. D
    I = 2 * r * tau_max + 1
    if D == I:
        return ORIG["fcc_basis"](N, tau_max, D, r, gap_tol)
    B = ORIG["fcc_basis"](N, tau_max, D + 1, r, gap_tol)
    keep = [k for k in range(D + 1) if k != D - 1]
    for name in ("sigma", "is_sym", "v_full", "p_hat"):
        setattr(B, name, getattr(B, name)[keep])
    B.Dc, B.Ds, B.D = B.Dc[:, keep], B.Ds[:, keep], D
    return B


def _lag_grid_reversed(tau_max, r=1):
    return ORIG["lag_grid"](tau_max, r)[::-1].copy()


ORIG = {k: getattr(O, k) for k in ("fold", "cross_spectrum", "fcc_basis", "lag_grid")}

MUTATIONS = [
    ("fold", _fold_wrong_sign, [P.pin_fold_identity]),
    ("fold", _fold_no_centre, [P.pin_fold_identity, P.pin_full_rank_is_gcc]),
    ("fcc_expand", _expand_wrong_sign, [P.pin_fold_identity, P.pin_full_rank_is_gcc]),
    ("cross_spectrum", _cross_conj_swapped, [P.pin_cross_and_phat]),
    ("phat", _phat_unnormalised, [P.pin_cross_and_phat]),
    ("hann_periodic", _window_symmetric, [P.pin_window, P.pin_stft_bruteforce, P.pin_stft_tone]),
    ("gcc_corr", _gcc_irfft, [P.pin_gcc_closed_form, P.pin_gcc_circular_xcorr]),
    ("fcc_basis", _basis_cut_off_by_one, [P.pin_eckart_young]),
    ("lag_grid", _lag_grid_reversed, [P.pin_gcc_closed_form, P.pin_basis_svd]),
]


@pytest.mark.parametrize("name,bad,pins", MUTATIONS,
                         ids=[f"{m[0]}:{m[1].__name__}" for m in MUTATIONS])
def test_planted_mistake_is_caught(monkeypatch, name, bad, pins):
    monkeypatch.setattr(O, name, bad)
    for pin in pins:
        with pytest.raises(AssertionError):
            pin(O)


def test_planted_delay_sign_is_caught(monkeypatch):
    monkeypatch.setattr(O, "cross_spectrum", _cross_conj_swapped)
    with pytest.raises(AssertionError):
        P.pin_integer_delay(O, lambda x: O.gcc_tdoa(x, 512, 128, 5))
