"""Plain FP64 CPU oracle for PHAT-weighted TDoA estimation.

TEST INFRASTRUCTURE ONLY.  The test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import this module; the GPU library and its
Python binding never do.  It shares no code, tables or helpers with the HIP
path: its basis comes from LAPACK (numpy.linalg.svd), its transforms from
numpy.fft, and every step is written out in the order the paper gives it.

Paper: F. Grondin, M.-A. Maheux, J.-S. Lauzon, J. Vincent, F. Michaud,
"Fast Cross-Correlation for TDoA Estimation on Small Aperture Microphone
Arrays", arXiv 2204.13622.  Each function cites the section / equation it
follows.  All floating-point work is float64 / complex128.

Readings taken where the paper is silent or inconsistent (each one is listed
with its reason in the design notes of the repository):

* Hann window is the periodic one, w[n] = 0.5 - 0.5 cos(2 pi n / N).
* Frames are not padded: T = floor((L - N) / hop) + 1, frame t covers samples
  [t hop, t hop + N).  The hop is a parameter (Sec. 2 uses 50 % overlap).
* Recursive cross-spectrum (eq. 1) starts from R = 0 before the first frame.
* PHAT of an exactly-zero cross-spectrum bin is 0.
* Eq. (2) is kept literally: the f = 0 and f = N/2 terms are inside 2 Re{.}.
* tau_max = ceil(d_max f_S / c) over all microphone pairs (Sec. 2, Sec. 5).
* The lag grid is tau_i = i / r - tau_max, i = 0 .. 2 r tau_max (Sec. 3).
* The SVD of W (Sec. 4) is taken separately on the subspaces of vectors that
  are symmetric / antisymmetric about f = N/4, and the components are ordered
  symmetric, antisymmetric, symmetric, ... as eq. (6) states (odd k even/real,
  even k odd/imaginary).  The paper's "real / purely imaginary" wording is a
  phase convention: the right singular vectors are taken real here.
* A rank cut that falls inside a cluster of (numerically) equal singular
  values of one parity is refused, because the rank-D result is not unique.
* Sign of each basis vector: its first entry of magnitude > 1e-6 max|v| is
  made positive (the correlation does not depend on it).
* argmax ties resolve to the lowest lag index.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "tau_max_from_geometry", "lag_grid", "num_frames", "hann_periodic",
    "frame_signal", "stft", "mic_pairs", "cross_spectrum", "phat",
    "gcc_corr", "FccBasis", "fcc_basis", "all_singular_values", "fold",
    "fcc_coefficients", "fcc_expand", "fcc_corr", "fcc_corr_unfolded",
    "argmax_first", "tdoa_from_corr", "parabolic_offset", "tdoa_parabolic_from_corr", "fcc_tdoa",
    "gcc_tdoa", "pipeline_spectra", "flops_gcc", "flops_direct",
    "flops_lowrank", "flops_fcc", "BasisAmbiguous",
]


class BasisAmbiguous(ValueError):
    """The requested rank cuts a cluster of equal singular values."""


# ---------------------------------------------------------------- Sec. 2 ---

def tau_max_from_geometry(mic_xyz, fs: float, c: float) -> int:
    """Largest TDoA in whole samples over all pairs (Sec. 2: tau_max = d f_S / c,
    rounded up so that every pair's lag window is covered)."""
    xyz = np.asarray(mic_xyz, dtype=np.float64)
    best = 0.0
    for i in range(xyz.shape[0]):
        for j in range(i + 1, xyz.shape[0]):
            dx, dy, dz = xyz[i] - xyz[j]
            d = math.sqrt(dx * dx + dy * dy + dz * dz)
            best = max(best, d)
    return int(math.ceil(best * fs / c))


def lag_grid(tau_max: int, r: int = 1) -> np.ndarray:
    """Candidate delays tau_1 .. tau_I, spaced 1/r sample (Sec. 3):
    I = 2 r tau_max + 1 (I = 4 tau_max + 1 for r = 2)."""
    I = 2 * r * tau_max + 1
    return np.arange(I, dtype=np.float64) / r - tau_max


def num_frames(L: int, N: int, hop: int) -> int:
    """Number of whole frames of N samples at the given hop (no padding)."""
    if L < N:
        return 0
    return (L - N) // hop + 1


def hann_periodic(N: int) -> np.ndarray:
    """Hann analysis window of the STFT (Sec. 2), periodic form."""
    n = np.arange(N, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * n / N)


def frame_signal(x, N: int, hop: int, frames=None) -> np.ndarray:
    """Cut x [M, L] into frames [T, M, N]; `frames` selects frame indices."""
    x = np.asarray(x, dtype=np.float64)
    T = num_frames(x.shape[-1], N, hop)
    t = np.arange(T) if frames is None else np.asarray(frames, dtype=np.int64)
    idx = t[:, None] * hop + np.arange(N)[None, :]          # [T, N]
    return np.transpose(x[:, idx], (1, 0, 2))                # [T, M, N]


def stft(x, N: int, hop: int, frames=None) -> np.ndarray:
    """STFT of every microphone (Sec. 2): X(t, f) for f = 0 .. N/2,
    X(t, f) = sum_n w[n] x[t hop + n] exp(-j 2 pi f n / N).  Returns
    complex128 [T, M, N/2 + 1]."""
    fr = frame_signal(x, N, hop, frames)
    return np.fft.rfft(fr * hann_periodic(N), axis=-1)


def mic_pairs(M: int):
    """All pairs (i, j), i < j, in lexicographic order."""
    return [(i, j) for i in range(M) for j in range(i + 1, M)]


def cross_spectrum(X, alpha: float = 1.0) -> np.ndarray:
    """Eq. (1): R(t, f) = (1 - alpha) R(t - 1, f) + alpha X_i(t, f) X_j(t, f)^*
    for every pair (i < j, lexicographic), with R = 0 before the first frame.
    X is [T, M, F]; returns [T, P, F]."""
    X = np.asarray(X)
    pr = mic_pairs(X.shape[1])
    ii = np.array([p[0] for p in pr], dtype=np.int64)
    jj = np.array([p[1] for p in pr], dtype=np.int64)
    C = X[:, ii, :] * np.conj(X[:, jj, :])
    if alpha == 1.0:
        return C
    R = np.empty_like(C)
    prev = np.zeros_like(C[0])
    for t in range(C.shape[0]):
        prev = (1.0 - alpha) * prev + alpha * C[t]
        R[t] = prev
    return R


def phat(R) -> np.ndarray:
    """Phase transform (Sec. 2): R_hat = R / |R|, and 0 where R is exactly 0."""
    R = np.asarray(R, dtype=np.complex128)
    mag = np.abs(R)
    out = np.zeros_like(R)
    nz = mag > 0
    out[nz] = R[nz] / mag[nz]
    return out


# ---------------------------------------------------------------- Sec. 3 ---

def gcc_corr(Rhat, N: int, tau_max: int, r: int = 1) -> np.ndarray:
    """GCC correlation of eq. (2) at the lag grid, through a full inverse DFT of
    size r N (Sec. 3: zero padding by r gives 1/r-sample resolution).

    y(tau) = 2 Re{ sum_{f=0}^{N/2} R_hat(f) exp(j 2 pi f tau / N) }.  Writing the
    real part as z + z^*, every bin f contributes R_hat(f) at index f and its
    conjugate at index -f (mod r N) of a Hermitian spectrum S; then
    y(n / r) = sum_k S[k] exp(j 2 pi k n / (r N)), the unnormalised inverse DFT.
    Returns float64 [..., I]."""
    Rhat = np.asarray(Rhat, dtype=np.complex128)
    F = N // 2 + 1
    assert Rhat.shape[-1] == F
    Lr = r * N
    S = np.zeros(Rhat.shape[:-1] + (Lr,), dtype=np.complex128)
    f = np.arange(F)
    S[..., f % Lr] += Rhat                  # indices 0 .. N/2, all distinct
    S[..., (-f) % Lr] += np.conj(Rhat)      # indices 0, rN-1 .. rN-N/2, distinct
    s = np.fft.ifft(S, axis=-1) * Lr
    n = np.rint(lag_grid(tau_max, r) * r).astype(np.int64) % Lr
    return s[..., n].real


# ---------------------------------------------------------------- Sec. 4 ---

@dataclass
class FccBasis:
    """Offline part of FCC (Sec. 4, Fig. 2): cropped bases and dictionary."""
    N: int
    tau_max: int
    r: int
    D: int
    sigma: np.ndarray          # [D] singular values, in basis order
    is_sym: np.ndarray         # [D] bool, True: p(k, f) = +p(k, N/2 - f)
    v_full: np.ndarray         # [D, N/2+1] real right singular vectors
    p_hat: np.ndarray          # [D, N/4+1] cropped rows of P = S V^H (eq. 7)
    Dc: np.ndarray             # [I, D] Re of the dictionary U
    Ds: np.ndarray             # [I, D] Im of the dictionary U
    tau: np.ndarray = field(default=None)   # [I] lag grid

    @property
    def I(self) -> int:
        return 2 * self.r * self.tau_max + 1


def _centred_matrices(N: int, tau_max: int, r: int):
    """W of eq. (3) times the unit-modulus row phase exp(-j pi tau / 2), restricted
    to real vectors symmetric (C) or antisymmetric (S) about f = N/4.  A
    symmetric v with v(f) = v(N/2 - f) = e(f)/sqrt(2) (f < N/4), v(N/4) = e(N/4)
    maps to C e; an antisymmetric one with v(f) = -v(N/2 - f) = e(f)/sqrt(2),
    v(N/4) = 0, maps to j S e."""
    m = N // 4
    tau = lag_grid(tau_max, r)
    g = np.arange(m, dtype=np.float64) - m                   # f - N/4, f < N/4
    ang = 2.0 * np.pi * np.outer(tau, g) / N
    C = np.empty((tau.size, m + 1))
    C[:, :m] = math.sqrt(2.0) * np.cos(ang)
    C[:, m] = 1.0
    S = math.sqrt(2.0) * np.sin(ang)
    return C, S, tau


def all_singular_values(N: int, tau_max: int, r: int = 1):
    """Every singular value of W (eq. 3), as (symmetric list, antisymmetric list)."""
    C, S, _ = _centred_matrices(N, tau_max, r)
    return (np.linalg.svd(C, compute_uv=False),
            np.linalg.svd(S, compute_uv=False))


def _fix_sign(e: np.ndarray) -> float:
    big = np.abs(e) > 1e-6 * np.abs(e).max()
    first = np.flatnonzero(big)[0]
    return 1.0 if e[first] > 0 else -1.0


def fcc_basis(N: int, tau_max: int, D: int, r: int = 1,
              gap_tol: float = 1e-9) -> FccBasis:
    """Truncated SVD of W (Sec. 4): W ~ U_D S_D V_D^H, P = S_D V_D^H (K x F rows
    p_k of eq. 5), dictionary U_D; cropped rows p_hat_k (eq. 7).

    Component order follows eq. (6): k = 1, 3, 5, ... symmetric about N/4,
    k = 2, 4, ... antisymmetric, so a rank D keeps ceil(D/2) symmetric and
    floor(D/2) antisymmetric components."""
    if N % 4 or N < 4:
        raise ValueError("N must be a multiple of 4")
    I = 2 * r * tau_max + 1
    if not 1 <= D <= I:
        raise ValueError("rank must lie in [1, I]")
    m = N // 4
    F = N // 2 + 1
    C, S, tau = _centred_matrices(N, tau_max, r)
    Uc, sc, Ect = np.linalg.svd(C, full_matrices=False)
    Us, ss, Est = np.linalg.svd(S, full_matrices=False)
    ds, da = (D + 1) // 2, D // 2
    for sv, cut in ((sc, ds), (ss, da)):
        if 0 < cut < sv.size and D < I:
            if sv[cut - 1] - sv[cut] <= gap_tol * max(sc[0], ss[0]):
                raise BasisAmbiguous(f"rank {D} cuts a singular-value cluster")
    sigma = np.empty(D)
    is_sym = np.empty(D, dtype=bool)
    v_full = np.zeros((D, F))
    Dc = np.empty((I, D))
    Dsn = np.empty((I, D))
    phase = np.exp(1j * np.pi * tau / 2.0)                    # exp(j pi tau / 2)
    if r == 1:                                               # exact quarter turns
        phase = np.array([1, 1j, -1, -1j])[np.rint(tau).astype(int) % 4]
    inv_r2 = 1.0 / math.sqrt(2.0)
    f_lo = np.arange(m)
    for k in range(D):
        sym = (k % 2 == 0)
        idx = k // 2
        if sym:
            e, u, s = Ect[idx].copy(), Uc[:, idx].copy(), sc[idx]
        else:
            e, u, s = Est[idx].copy(), Us[:, idx].copy(), ss[idx]
        sg = _fix_sign(e)
        e *= sg
        u *= sg
        v = np.zeros(F)
        v[f_lo] = e[:m] * inv_r2
        if sym:
            v[N // 2 - f_lo] = e[:m] * inv_r2
            v[m] = e[m]
            uk = phase * u                                   # W v = s exp(j pi tau/2) C e / s
        else:
            v[N // 2 - f_lo] = -e[:m] * inv_r2
            v[m] = 0.0
            uk = 1j * phase * u                              # W v = j exp(j pi tau/2) S e
        sigma[k], is_sym[k], v_full[k] = s, sym, v
        Dc[:, k], Dsn[:, k] = uk.real, uk.imag
    p_hat = sigma[:, None] * v_full[:, :m + 1]               # eq. (7)
    return FccBasis(N=N, tau_max=tau_max, r=r, D=D, sigma=sigma, is_sym=is_sym,
                    v_full=v_full, p_hat=p_hat, Dc=Dc, Ds=Dsn, tau=tau)


def fold(Rhat, N: int):
    """Eq. (8): x_s(f) = R_hat(f) + R_hat(N/2 - f), x_d(f) = R_hat(f) - R_hat(N/2 - f)
    for f = 0 .. N/4 - 1, plus the centre bin R_hat(N/4) (last entry of both)."""
    Rhat = np.asarray(Rhat, dtype=np.complex128)
    m = N // 4
    f = np.arange(m)
    head = Rhat[..., f]
    tail = Rhat[..., N // 2 - f]
    centre = Rhat[..., m]
    return head + tail, head - tail, centre


def fcc_coefficients(Rhat, B: FccBasis) -> np.ndarray:
    """Eq. (9): z_k = p_hat_k . x_s for symmetric k (plus the centre bin),
    z_k = p_hat_k . x_d for antisymmetric k.  Returns complex [..., D]."""
    m = B.N // 4
    x_s, x_d, centre = fold(Rhat, B.N)
    z = np.empty(np.shape(centre) + (B.D,), dtype=np.complex128)
    for k in range(B.D):
        if B.is_sym[k]:
            z[..., k] = x_s @ B.p_hat[k, :m] + centre * B.p_hat[k, m]
        else:
            z[..., k] = x_d @ B.p_hat[k, :m]
    return z


def fcc_expand(z, B: FccBasis) -> np.ndarray:
    """Sec. 4: y = 2 Re{D z}, i.e. y(tau_i) = 2 sum_k (Dc(i,k) Re z_k - Ds(i,k) Im z_k)."""
    z = np.asarray(z)
    return 2.0 * (z.real @ B.Dc.T - z.imag @ B.Ds.T)


def fcc_corr(Rhat, B: FccBasis) -> np.ndarray:
    """FCC correlation: fold (eq. 8), project (eq. 9), expand to lags."""
    return fcc_expand(fcc_coefficients(Rhat, B), B)


def fcc_corr_unfolded(Rhat, B: FccBasis) -> np.ndarray:
    """The same rank-D correlation without the fold: y = 2 Re{W V_D V_D^T x}
    (W of eq. 3 built directly; no division by any singular value)."""
    N = B.N
    f = np.arange(N // 2 + 1)
    W = np.exp(2j * np.pi * np.outer(B.tau, f) / N)
    Rhat = np.asarray(Rhat, dtype=np.complex128)
    proj = (Rhat @ B.v_full.T) @ B.v_full
    return 2.0 * (proj @ W.T).real


def argmax_first(y) -> np.ndarray:
    """Index of the largest correlation (Sec. 2); ties go to the lowest index."""
    return np.argmax(np.asarray(y), axis=-1)


def tdoa_from_corr(y, tau_max: int, r: int = 1) -> np.ndarray:
    """TDoA in units of 1/r sample: i* - r tau_max (int32)."""
    return (argmax_first(y) - r * tau_max).astype(np.int32)


def parabolic_offset(y_m, y_0, y_p) -> np.ndarray:
    """Closed-form quadratic interpolation around the peak (Sec. 2): offset of the
    vertex of the parabola through (-1, y_m), (0, y_0), (1, y_p); 0 where the
    three points are collinear."""
    y_m, y_0, y_p = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64)
                                          for a in (y_m, y_0, y_p)))
    den = y_m - 2.0 * y_0 + y_p
    num = y_m - y_p
    out = np.zeros(den.shape)
    ok = den != 0
    out[ok] = 0.5 * num[ok] / den[ok]
    return out


def tdoa_parabolic_from_corr(y, tau_max: int, r: int = 1) -> np.ndarray:
    """Argmax lag refined by quadratic interpolation (Sec. 2), in samples.
    No refinement at either end of the lag window."""
    y = np.asarray(y, dtype=np.float64)
    i = argmax_first(y)
    I = y.shape[-1]
    inner = (i > 0) & (i < I - 1)
    ic = np.clip(i, 1, I - 2)
    ym = np.take_along_axis(y, (ic - 1)[..., None], -1)[..., 0]
    y0 = np.take_along_axis(y, ic[..., None], -1)[..., 0]
    yp = np.take_along_axis(y, (ic + 1)[..., None], -1)[..., 0]
    d = np.where(inner, parabolic_offset(ym, y0, yp), 0.0)
    return (i - r * tau_max + d) / r


# ------------------------------------------------------------- pipelines ---

def pipeline_spectra(x, N: int, hop: int, alpha: float = 1.0, frames=None):
    """STFT -> cross-spectrum (eq. 1) -> PHAT, for every pair: [T, P, F]."""
    if alpha != 1.0 and frames is not None:
        raise ValueError("recursive smoothing needs every frame")
    return phat(cross_spectrum(stft(x, N, hop, frames), alpha))


def fcc_tdoa(x, N: int, hop: int, tau_max: int, D: int, r: int = 1,
             alpha: float = 1.0, frames=None, basis: FccBasis | None = None,
             return_corr: bool = False):
    """End-to-end FCC TDoA [T, P] (int32, units of 1/r sample)."""
    B = basis if basis is not None else fcc_basis(N, tau_max, D, r)
    y = fcc_corr(pipeline_spectra(x, N, hop, alpha, frames), B)
    t = tdoa_from_corr(y, tau_max, r)
    return (t, y) if return_corr else t


def gcc_tdoa(x, N: int, hop: int, tau_max: int, r: int = 1, alpha: float = 1.0,
             frames=None, return_corr: bool = False):
    """End-to-end GCC-PHAT TDoA [T, P] (int32, units of 1/r sample)."""
    y = gcc_corr(pipeline_spectra(x, N, hop, alpha, frames), N, tau_max, r)
    t = tdoa_from_corr(y, tau_max, r)
    return (t, y) if return_corr else t


# ------------------------------------------------------- flop accounting ---

def flops_gcc(N: int, r: int) -> int:
    """Real IFFT of r N points (Sec. 3).  The printed expression is garbled; the
    form 5 (r N / 2) log2(r N) reproduces every GCC entry of Table 1."""
    return int(5 * (r * N // 2) * round(math.log2(r * N)))


def flops_direct(N: int, I: int) -> int:
    """Direct y = 2 Re{W x} (Sec. 4): I (4 N + 6)."""
    return I * (4 * N + 6)


def flops_lowrank(N: int, I: int, K: int) -> int:
    """z = P x then 2 Re{D z} (Sec. 4): K (4 N + 6) + I (4 K - 1)."""
    return K * (4 * N + 6) + I * (4 * K - 1)


def flops_fcc(N: int, I: int, K: int) -> int:
    """Folded projection of eq. (9) plus the fold and the expansion (Sec. 4):
    K (N + 2) + N + I (4 K - 1)."""
    return K * (N + 2) + N + I * (4 * K - 1)
