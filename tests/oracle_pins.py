"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each `pin_*` function raises AssertionError when the oracle is wrong.  They
take the oracle module as an argument so that the mutation tests can run the
same pins on an oracle with a planted mistake and see them fail.

None of these re-type the oracle's own formula: each compares against a
brute-force evaluation, a closed form, an invariant, or a number the paper
prints.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ------------------------------------------------------------------ STFT ---

def brute_dft_real(frame: np.ndarray) -> np.ndarray:
    """O(N^2) forward DFT, bins 0..N/2, written as explicit sums."""
    N = frame.size
    out = np.zeros(N // 2 + 1, dtype=np.complex128)
    for f in range(N // 2 + 1):
        acc = 0.0 + 0.0j
        for n in range(N):
            ang = 2.0 * math.pi * f * n / N
            acc += frame[n] * complex(math.cos(ang), -math.sin(ang))
        out[f] = acc
    return out


def pin_window(o):
    for N in (8, 16, 64, 512):
        w = o.hann_periodic(N)
        assert abs(w[0]) < 1e-15 and abs(w[N // 2] - 1.0) < 1e-15
        assert np.allclose(w[1:], w[1:][::-1], atol=1e-15)       # w[n] = w[N-n]
        assert abs(w.sum() - N / 2) < 1e-9                       # periodic form
        assert abs(w[N // 4] - 0.5) < 1e-15


def pin_stft_bruteforce(o):
    rng = np.random.default_rng(7)
    for N, hop in ((8, 2), (16, 4), (32, 8)):
        x = rng.standard_normal((2, 5 * N))
        X = o.stft(x, N, hop)
        T = (x.shape[1] - N) // hop + 1
        assert X.shape == (T, 2, N // 2 + 1)
        # window from its defining property: raised cosine with zero at n = 0
        w = np.array([math.sin(math.pi * n / N) ** 2 for n in range(N)])
        for t in range(T):
            for m in range(2):
                ref = brute_dft_real(w * x[m, t * hop: t * hop + N])
                assert np.abs(X[t, m] - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())


def pin_stft_tone(o):
    """Hann-windowed cosine on an integer bin f0: X(f0) = N/4, X(f0 +- 1) = -N/8."""
    N = 64
    for f0 in (2, 5, 17, 30):
        n = np.arange(3 * N)
        x = np.cos(2 * np.pi * f0 * n / N)[None, :]
        X = o.stft(x, N, N)
        expect = np.zeros(N // 2 + 1)
        expect[f0] = N / 4
        expect[f0 - 1] = expect[f0 + 1] = -N / 8
        assert np.abs(X[:, 0, :] - expect).max() < 1e-11


def pin_frames(o):
    assert o.num_frames(16000, 512, 128) == 122
    assert o.num_frames(960000, 512, 128) == 7497
    assert o.num_frames(5760000, 1024, 256) == 22497
    assert o.num_frames(511, 512, 128) == 0
    assert o.num_frames(512, 512, 128) == 1
    x = np.arange(40, dtype=float)[None, :]
    fr = o.frame_signal(x, 8, 3)
    assert fr.shape == (11, 1, 8) and fr[2, 0, 0] == 6 and fr[10, 0, 7] == 37


# ------------------------------------------------------ pairs, eq.1, PHAT ---

def pin_pairs(o):
    p = o.mic_pairs(5)
    assert len(p) == 10 and p[0] == (0, 1) and p[3] == (0, 4) and p[4] == (1, 2)
    assert p[-1] == (3, 4)


def pin_cross_and_phat(o):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((4, 3, 9)) + 1j * rng.standard_normal((4, 3, 9))
    X[1, 2, 4] = 0.0
    C = o.cross_spectrum(X, 1.0)
    pr = o.mic_pairs(3)
    for p, (i, j) in enumerate(pr):          # R = X_i X_j^* elementwise
        for t in range(4):
            for f in range(9):
                a, b = X[t, i, f], X[t, j, f]
                ref = complex(a.real * b.real + a.imag * b.imag,
                              a.imag * b.real - a.real * b.imag)
                assert abs(C[t, p, f] - ref) < 1e-14
    Rh = o.phat(C)
    mag = np.abs(Rh)
    assert np.all((np.abs(mag - 1) < 1e-14) | (mag == 0))
    assert np.all((mag == 0) == (C == 0))
    # factorisation at alpha = 1: phase of X_i times conjugate phase of X_j
    e = np.where(np.abs(X) > 0, X / np.where(np.abs(X) > 0, np.abs(X), 1), 0)
    for p, (i, j) in enumerate(pr):
        assert np.abs(Rh[:, p] - e[:, i] * np.conj(e[:, j])).max() < 1e-14
    # scale invariance: positive per-(frame, mic) gains leave PHAT unchanged
    g = rng.uniform(0.1, 10.0, size=(4, 3, 1))
    assert np.abs(o.phat(o.cross_spectrum(X * g, 1.0)) - Rh).max() < 1e-13


def pin_recursion(o):
    """Constant input: R(t) = (1 - (1 - alpha)^(t+1)) C, a geometric series."""
    X = np.ones((6, 2, 3), dtype=complex) * (0.5 + 2.0j)
    C = X[:, 0] * np.conj(X[:, 1])
    for alpha in (1.0, 0.5, 0.1):
        R = o.cross_spectrum(X, alpha)[:, 0]
        for t in range(6):
            assert np.abs(R[t] - (1 - (1 - alpha) ** (t + 1)) * C[t]).max() < 1e-14


# ------------------------------------------------------------- GCC, eq.2 ---

def brute_inverse_dft_real(E: np.ndarray, N: int) -> np.ndarray:
    """u[n] = (1/N) sum over the full Hermitian spectrum of E (bins 0..N/2)."""
    u = np.zeros(N)
    for n in range(N):
        acc = 0.0
        for k in range(N):
            ek = E[k] if k <= N // 2 else np.conj(E[N - k])
            acc += (ek * complex(math.cos(2 * math.pi * k * n / N),
                                 math.sin(2 * math.pi * k * n / N))).real
        u[n] = acc / N
    return u


def pin_gcc_circular_xcorr(o):
    """Eq. (2) = N * circular cross-correlation of the PHAT-whitened frames plus
    the DC and Nyquist terms that eq. (2) counts twice."""
    rng = np.random.default_rng(11)
    for N, tm in ((16, 3), (32, 5)):
        x = rng.standard_normal((2, N))
        X = o.stft(x, N, N)[0]
        e = X / np.abs(X)
        u0, u1 = brute_inverse_dft_real(e[0], N), brute_inverse_dft_real(e[1], N)
        Rh = o.phat(o.cross_spectrum(X[None], 1.0))[0, 0]
        y = o.gcc_corr(Rh, N, tm, 1)
        for i, tau in enumerate(range(-tm, tm + 1)):
            cc = sum(u0[(n + tau) % N] * u1[n] for n in range(N))
            ref = N * cc + Rh[0].real + Rh[N // 2].real * (-1) ** (tau % 2)
            assert abs(y[i] - ref) < 1e-10, (N, tau, y[i], ref)


def pin_gcc_closed_form(o):
    """R_hat(f) = exp(j 2 pi f delta / N): y(-delta) = N + 2, else 1 + (-1)^(tau+delta)."""
    N, tm = 64, 6
    for delta in (-4, -1, 0, 3):
        Rh = np.exp(2j * np.pi * np.arange(N // 2 + 1) * delta / N)
        y = o.gcc_corr(Rh, N, tm, 1)
        for i, tau in enumerate(range(-tm, tm + 1)):
            ref = N + 2 if tau == -delta else 1 + (-1) ** ((tau + delta) % 2)
            assert abs(y[i] - ref) < 1e-11
    # half-sample delay on the r = 2 grid peaks at -delta with N + 2
    for delta in (-2.5, 0.5, 1.5):
        Rh = np.exp(2j * np.pi * np.arange(N // 2 + 1) * delta / N)
        y = o.gcc_corr(Rh, N, tm, 2)
        i = int(np.argmax(y))
        assert abs(o.lag_grid(tm, 2)[i] + delta) < 1e-12 and abs(y[i] - (N + 2)) < 1e-10


def pin_gcc_r2_integer_lags(o):
    rng = np.random.default_rng(5)
    X = o.stft(rng.standard_normal((3, 600)), 64, 16)
    Rh = o.phat(o.cross_spectrum(X, 1.0))
    y1 = o.gcc_corr(Rh, 64, 5, 1)
    y2 = o.gcc_corr(Rh, 64, 5, 2)
    assert np.abs(y2[..., ::2] - y1).max() < 1e-11


def pin_integer_delay(o, tdoa_fn):
    """x_1[n] = x_0[n - delta] (white noise): TDoA_01 = -delta in every frame."""
    from gen import white_pair
    for delta in (-3, -1, 0, 2, 4):
        x = white_pair(100 + delta, 4096, delta)
        t = tdoa_fn(x)
        assert np.all(t[:, 0] == -delta), (delta, t[:, 0])


# ---------------------------------------------------------- basis, Sec. 4 ---

def build_W(N, tau):
    """Eq. (3): w(tau, f) = exp(j 2 pi f tau / N), f = 0 .. N/2."""
    f = np.arange(N // 2 + 1)
    return np.exp(2j * np.pi * np.outer(tau, f) / N)


def pin_basis_svd(o, N=512, tm=5, r=1):
    I = 2 * r * tm + 1
    B = o.fcc_basis(N, tm, I, r)
    tau = np.arange(I) / r - tm
    W = build_W(N, tau)
    U = B.Dc + 1j * B.Ds
    V = B.v_full
    # components below 1e-4 sigma_1 are determined only up to rounding noise
    nz = B.sigma > 1e-4 * B.sigma[0]
    # W v_k = sigma_k u_k and W^H u_k = sigma_k v_k
    assert np.abs(W @ V.T - U * B.sigma).max() < 1e-11
    assert np.abs((W.conj().T @ U)[:, nz] - (V.T * B.sigma)[:, nz]).max() < 1e-10
    assert np.abs(V @ V.T - np.eye(I)).max() < 1e-12
    assert np.abs(U[:, nz].conj().T @ U[:, nz] - np.eye(nz.sum())).max() < 1e-11
    # Parseval over every singular value: ||W||_F^2 = I (N/2 + 1)
    ss, sa = o.all_singular_values(N, tm, r)
    assert abs((ss ** 2).sum() + (sa ** 2).sum() - I * (N // 2 + 1)) < 1e-8
    # kept values are the largest of all
    allv = np.sort(np.concatenate([ss, sa]))[::-1]
    assert np.abs(np.sort(B.sigma)[::-1] - allv[:I]).max() < 1e-10


def pin_basis_symmetry(o, N=512, tm=5, D=11, r=1):
    B = o.fcc_basis(N, tm, D, r)
    m = N // 4
    f = np.arange(N // 2 + 1)
    for k in range(D):
        v = B.v_full[k]
        sgn = 1.0 if B.is_sym[k] else -1.0
        assert np.array_equal(v, sgn * v[N // 2 - f])      # eq. (6), exact
        if not B.is_sym[k]:
            assert v[m] == 0.0
        assert np.abs(B.p_hat[k] - B.sigma[k] * v[:m + 1]).max() < 1e-12
    # order of eq. (6): k = 1, 3, ... symmetric; k = 2, 4, ... antisymmetric
    assert list(B.is_sym) == [k % 2 == 0 for k in range(D)]
    # the alternation agrees with the singular values (interlacing)
    tol = 1e-12 * B.sigma[0]
    assert np.all(B.sigma[:-1] >= B.sigma[1:] - tol)


def pin_dictionary_parity(o, N=512, tm=5, D=11):
    """Dc even, Ds odd in tau; at integer lags a symmetric k feeds Dc only at
    even tau and Ds only at odd tau, an antisymmetric k the reverse."""
    B = o.fcc_basis(N, tm, D, 1)
    rev = slice(None, None, -1)
    # left singular vectors of a weak component carry error ~ eps sigma_1 / sigma_k
    tol = 1e-14 * B.sigma[0] / B.sigma + 1e-15
    assert np.all(np.abs(B.Dc - B.Dc[rev]).max(axis=0) < tol)
    assert np.all(np.abs(B.Ds + B.Ds[rev]).max(axis=0) < tol)
    tau = np.arange(-tm, tm + 1)
    even = (tau % 2 == 0)
    for k in range(D):
        if B.is_sym[k]:
            assert np.all(B.Dc[~even, k] == 0) and np.all(B.Ds[even, k] == 0)
        else:
            assert np.all(B.Dc[even, k] == 0) and np.all(B.Ds[~even, k] == 0)


def pin_eckart_young(o, N=256, tm=4):
    I = 2 * tm + 1
    tau = np.arange(I) - tm
    W = build_W(N, tau)
    ss, sa = o.all_singular_values(N, tm, 1)
    allv = np.sort(np.concatenate([ss, sa]))[::-1]
    for D in range(1, I + 1):
        B = o.fcc_basis(N, tm, D, 1)
        WD = (B.Dc + 1j * B.Ds) @ (B.sigma[:, None] * B.v_full)
        err = np.linalg.norm(W - WD) ** 2
        assert abs(err - (allv[D:] ** 2).sum()) < 1e-9, (D, err)


# ------------------------------------------------------------ FCC, eq. 9 ---

def _rand_rhat(seed, shape, N):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(shape + (N // 2 + 1,)) + 1j * rng.standard_normal(shape + (N // 2 + 1,))
    z[..., 0] = z[..., 0].real
    z[..., N // 2] = z[..., N // 2].real
    return z / np.abs(z)


def pin_fold_identity(o):
    for N, tm, r in ((512, 5, 1), (64, 4, 1), (512, 8, 2), (1024, 14, 1)):
        Rh = _rand_rhat(N + tm, (7,), N)
        I = 2 * r * tm + 1
        for D in sorted({1, 2, 3, (I + 1) // 2, I - 1, I}):
            try:
                B = o.fcc_basis(N, tm, D, r)
            except o.BasisAmbiguous:
                continue
            y1 = o.fcc_corr(Rh, B)
            y2 = o.fcc_corr_unfolded(Rh, B)
            assert np.abs(y1 - y2).max() < 1e-11 * max(1.0, np.abs(y2).max()), (N, tm, r, D)


def pin_full_rank_is_gcc(o):
    for N, tm in ((512, 5), (512, 4), (1024, 14), (64, 6)):
        Rh = _rand_rhat(tm, (5, 3), N)
        B = o.fcc_basis(N, tm, 2 * tm + 1, 1)
        y1 = o.fcc_corr(Rh, B)
        y2 = o.gcc_corr(Rh, N, tm, 1)
        assert np.abs(y1 - y2).max() < 1e-11 * np.abs(y2).max()


def pin_swap(o):
    """Swapping the pair conjugates R_hat, so y_ji(tau) = y_ij(-tau) at any rank."""
    N, tm = 512, 5
    Rh = _rand_rhat(1, (9,), N)
    for D in (1, 4, 6, 11):
        B = o.fcc_basis(N, tm, D, 1)
        y = o.fcc_corr(Rh, B)
        ys = o.fcc_corr(np.conj(Rh), B)
        assert np.abs(ys - y[..., ::-1]).max() < 1e-11 * np.abs(y).max()


def pin_flops(o):
    with open(os.path.join(GOLDEN, "table1_flops.json")) as fh:
        g = json.load(fh)
    N, I = g["N"], g["I"]
    for r, v in g["gcc"].items():
        assert o.flops_gcc(N, int(r)) == v
    for K, v in g["fcc"].items():
        assert o.flops_fcc(N, I, int(K)) == v
    assert o.flops_direct(N, I) == g["direct_I_33"]
    assert o.flops_lowrank(N, I, 8) == g["lowrank_K_8"]
    assert round(o.flops_gcc(N, 2) / o.flops_fcc(N, I, 8), 1) == g["fcc_reduction_vs_gcc_r2"]


def pin_paper_settings(o):
    with open(os.path.join(GOLDEN, "paper_settings.json")) as fh:
        g = json.load(fh)["results_setting"]
    xyz = np.array([[0, 0, 0], [g["d"], 0, 0]])
    tm = o.tau_max_from_geometry(xyz, g["fs"], g["c"])
    assert tm == g["tau_max"]
    assert o.lag_grid(tm, g["r"]).size == g["I"]


def pin_argmax(o):
    y = np.array([[0.0, 2.0, 2.0, 1.0], [3.0, 3.0, 3.0, 3.0], [-1.0, -2.0, -0.5, -0.5]])
    assert list(o.argmax_first(y)) == [1, 0, 2]
    assert list(o.tdoa_from_corr(y, 1, 1)) == [0, -1, 1]


def pin_parabola(o):
    for vertex in (-0.4, 0.0, 0.25, 0.49):
        a = -3.0
        ys = [a * (u - vertex) ** 2 + 7.0 for u in (-1, 0, 1)]
        assert abs(float(o.parabolic_offset(*ys)) - vertex) < 1e-14
    assert float(o.parabolic_offset(1.0, 1.0, 1.0)) == 0.0


ALL_PINS = [pin_window, pin_stft_bruteforce, pin_stft_tone, pin_frames, pin_pairs,
            pin_cross_and_phat, pin_recursion, pin_gcc_circular_xcorr,
            pin_gcc_closed_form, pin_gcc_r2_integer_lags, pin_basis_svd,
            pin_basis_symmetry, pin_dictionary_parity, pin_eckart_young,
            pin_fold_identity, pin_full_rank_is_gcc, pin_swap, pin_flops,
            pin_paper_settings, pin_argmax, pin_parabola]
