"""Seeded synthetic microphone-array recordings.

This module only synthesises signals: geometry, sources, propagation delays,
reverberation and sensor noise.  It holds none of the TDoA method's
arithmetic (no framing, transforms, cross-spectra or correlation), so both the
oracle and the GPU path can be fed from it.

Workloads (the paper's own recordings come from a simulated-room dataset that
is not available here; these stand in for it with the shapes and statistics of
the benchmark configurations):

  1  M=4 on a 5 cm square, fs=16 kHz, 1 s, white source, integer far-field
     delays, sensor noise at 10 dB SNR.                   N=512, hop=128
  2  M=16 on a 5 cm-radius circle, fs=16 kHz, 60 s, AR(2) source gated on/off
     in 0.2-0.8 s bursts, per-mic exponentially decaying FIR reverb
     (RT60 0.3 s), sensor noise SNR ~ U[0, 20] dB per mic.  N=512, hop=128
  3  as 2 with fs=48 kHz, 120 s.                          N=1024, hop=256
  5  M=8 on a 4 cm-radius circle, fs=16 kHz, white source with fractional
     (sinc-interpolated) far-field delays, SNR ~ U[0, 20] dB.  N=512, hop=128

Seeds: numpy default_rng (PCG64).  Every quantity is drawn in a fixed order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SPEED_OF_SOUND = 343.0


@dataclass
class ArrayRecording:
    config: int
    seed: int
    mic_xyz: np.ndarray          # [M, 3] metres
    fs: float
    c: float
    N: int
    hop: int
    x: np.ndarray                # [M, L] float32
    delays: np.ndarray           # [M] arrival delay of the direct path, samples
    ranks: tuple = ()            # ranks the configuration is exercised at
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return self.x.shape[0]

    @property
    def L(self) -> int:
        return self.x.shape[1]


def square_array(side: float) -> np.ndarray:
    h = side / 2.0
    return np.array([[-h, -h, 0.0], [h, -h, 0.0], [h, h, 0.0], [-h, h, 0.0]])


def circular_array(M: int, radius: float) -> np.ndarray:
    a = 2.0 * np.pi * np.arange(M) / M
    return np.stack([radius * np.cos(a), radius * np.sin(a), np.zeros(M)], axis=1)


def far_field_delays(mic_xyz, azimuth: float, fs: float, c: float) -> np.ndarray:
    """Arrival delay in samples of a planar wave from `azimuth` at each mic,
    relative to the array origin (negative = earlier)."""
    u = np.array([np.cos(azimuth), np.sin(azimuth), 0.0])
    return -(np.asarray(mic_xyz) @ u) * fs / c


def _integer_delay(s: np.ndarray, d: int, L: int, pad: int) -> np.ndarray:
    """s is padded by `pad` samples on both sides; returns s[n - d], n = 0..L-1."""
    return s[pad - d: pad - d + L]


def _snr_noise(rng, sig: np.ndarray, snr_db: float) -> np.ndarray:
    p = float(np.mean(sig.astype(np.float64) ** 2))
    return rng.standard_normal(sig.shape) * np.sqrt(p * 10.0 ** (-snr_db / 10.0))


def _ar2(rng, L: int, pole_radius: float, angle: float) -> np.ndarray:
    from scipy.signal import lfilter
    a1 = 2.0 * pole_radius * np.cos(angle)
    a2 = -pole_radius ** 2
    e = rng.standard_normal(L)
    return lfilter([1.0], [1.0, -a1, -a2], e)


def _gate(rng, L: int, fs: float, lo: float = 0.2, hi: float = 0.8) -> np.ndarray:
    g = np.zeros(L)
    n, on = 0, True
    while n < L:
        seg = int(round(rng.uniform(lo, hi) * fs))
        if on:
            g[n:n + seg] = 1.0
        n += seg
        on = not on
    return g


def _reverb_fir(rng, fs: float, rt60: float) -> np.ndarray:
    """Exponentially decaying noise tail (60 dB over rt60) whose energy equals
    the unit direct path; index 0 is the direct path."""
    n_tail = int(round(rt60 * fs))
    n = np.arange(1, n_tail)
    tail = rng.standard_normal(n_tail - 1) * np.exp(-6.908 * n / (rt60 * fs))
    tail /= np.sqrt(np.sum(tail ** 2))
    return np.concatenate([[1.0], tail])


def make_recording(config: int, seed: int | None = None, seconds: float | None = None,
                   M: int | None = None) -> ArrayRecording:
    """Synthesise the recording of one benchmark configuration.

    `seconds` shortens (or lengthens) the recording; `M` overrides the mic
    count of the circular arrays (for reduced parity cases)."""
    if seed is None:
        seed = 1000 * config
    rng = np.random.default_rng(seed)
    c = SPEED_OF_SOUND
    if config == 1:
        fs, N, hop, dur = 16000.0, 512, 128, 1.0 if seconds is None else seconds
        xyz = square_array(0.05)
        L = int(round(dur * fs))
        az = rng.uniform(0.0, 2.0 * np.pi)
        delays = np.rint(far_field_delays(xyz, az, fs, c)).astype(np.int64)
        pad = 64
        s = rng.standard_normal(L + 2 * pad)
        clean = np.stack([_integer_delay(s, int(d), L, pad) for d in delays])
        noise = np.stack([_snr_noise(rng, clean[m], 10.0) for m in range(len(xyz))])
        x = clean + noise
        return ArrayRecording(1, seed, xyz, fs, c, N, hop, x.astype(np.float32),
                              delays.astype(np.float64), ranks=(9,),
                              meta={"azimuth": az})
    if config in (2, 3):
        from scipy.signal import fftconvolve
        if config == 2:
            fs, N, hop, dur = 16000.0, 512, 128, 60.0
            ranks = (6, 11)
        else:
            fs, N, hop, dur = 48000.0, 1024, 256, 120.0
            ranks = (15, 29)
        if seconds is not None:
            dur = seconds
        Mm = 16 if M is None else M
        xyz = circular_array(Mm, 0.05)
        L = int(round(dur * fs))
        az = rng.uniform(0.0, 2.0 * np.pi)
        delays = np.rint(far_field_delays(xyz, az, fs, c)).astype(np.int64)
        angle = rng.uniform(0.05 * np.pi, 0.45 * np.pi) * (16000.0 / fs)
        pad = 64
        s = _ar2(rng, L + 2 * pad, 0.95, angle)
        s[pad:pad + L] *= _gate(rng, L, fs)
        s[:pad] = 0.0
        s[pad + L:] = 0.0
        x = np.empty((Mm, L))
        snrs = rng.uniform(0.0, 20.0, size=Mm)
        for m in range(Mm):
            h = _reverb_fir(rng, fs, 0.3)
            direct = _integer_delay(s, int(delays[m]), L, pad)
            rev = fftconvolve(direct, h)[:L]
            x[m] = rev + _snr_noise(rng, rev, snrs[m])
        return ArrayRecording(config, seed, xyz, fs, c, N, hop, x.astype(np.float32),
                              delays.astype(np.float64), ranks=ranks,
                              meta={"azimuth": az, "snr_db": snrs, "ar_angle": angle})
    if config == 5:
        fs, N, hop, dur = 16000.0, 512, 128, 1.0 if seconds is None else seconds
        Mm = 8 if M is None else M
        xyz = circular_array(Mm, 0.04)
        L = int(round(dur * fs))
        az = rng.uniform(0.0, 2.0 * np.pi)
        delays = far_field_delays(xyz, az, fs, c)
        pad = 64
        s = rng.standard_normal(L + 2 * pad)
        x = np.stack([fractional_delay(s, d, pad, L) for d in delays])
        snrs = rng.uniform(0.0, 20.0, size=Mm)
        x = x + np.stack([_snr_noise(rng, x[m], snrs[m]) for m in range(Mm)])
        return ArrayRecording(5, seed, xyz, fs, c, N, hop, x.astype(np.float32),
                              delays, ranks=(5, 9), meta={"azimuth": az, "snr_db": snrs})
    raise ValueError(f"unknown configuration {config}")


def fractional_delay(s: np.ndarray, d: float, pad: int, L: int,
                     half_taps: int = 32) -> np.ndarray:
    """s[n - d] for n = 0..L-1 by a Hann-windowed sinc interpolator
    (s is padded by `pad` >= half_taps samples on both sides)."""
    k = np.arange(-half_taps, half_taps + 1)
    di = int(np.floor(d))
    frac = d - di
    taps = np.sinc(k - frac) * (0.5 + 0.5 * np.cos(np.pi * (k - frac) / (half_taps + 1)))
    out = np.zeros(L)
    for kk, w in zip(k, taps):
        start = pad - di - kk
        out += w * s[start:start + L]
    return out


def white_pair(seed: int, L: int, delay: int, snr_db: float | None = None):
    """Two-channel white-noise recording with x1[n] = x0[n - delay] (+ noise)."""
    rng = np.random.default_rng(seed)
    pad = abs(delay) + 8
    s = rng.standard_normal(L + 2 * pad)
    x = np.stack([_integer_delay(s, 0, L, pad), _integer_delay(s, delay, L, pad)])
    if snr_db is not None:
        x = x + np.stack([_snr_noise(rng, x[m], snr_db) for m in range(2)])
    return x.astype(np.float32)


def random_signals(seed: int, M: int, L: int, kind: str = "white") -> np.ndarray:
    """Unstructured test signals [M, L] float32 (white, or with exact zeros)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((M, L))
    if kind == "gated":
        x[:, L // 3: L // 3 + L // 4] = 0.0
    return x.astype(np.float32)


def fractional_delay_frames(seed: int, count: int, M: int = 8, radius: float = 0.04,
                            fs: float = 16000.0, N: int = 512, c: float = 343.0,
                            snr_db=(0.0, 20.0), chunk: int = 2048, rt60=None, drr_db=(0.0, 10.0)):
    """`count` independent single-frame recordings of a circular array with
    fractional (sub-sample) propagation delays.

    Each frame has its own far-field direction, uniform on the sphere, so the
    delay of every mic pair is uniform over that pair's physical range
    [-d_ij fs / c, d_ij fs / c].  The source is white and band-limited with
    period 2N; it is delayed in the frequency domain, which is exact
    band-limited (periodic sinc) interpolation, and the middle N samples are
    kept.  Each mic gets white sensor noise at an SNR uniform in `snr_db`
    relative to its own frame power.

    With rt60 = (lo, hi) seconds each mic also hears a reverberant tail: white
    noise decaying by 60 dB over an RT60 drawn from U[lo, hi], starting one
    sample after the direct path and wrapped onto the 2N-sample period
    (circular convolution), scaled to a direct-to-reverberant ratio drawn
    from U[drr_db].  The delays returned stay those of the direct path.

    Returns (x, delays, xyz): x [M][count * N] float32, frame e occupying
    samples [e N, (e + 1) N) (frame with hop N); delays [count][M] in samples
    (the arrival time at each mic relative to the array centre); xyz [M][3].
    """
    rng = np.random.default_rng(seed)
    xyz = circular_array(M, radius)
    Lp = 2 * N
    f = np.arange(Lp // 2 + 1)
    x = np.empty((M, count * N), dtype=np.float32)
    delays = np.empty((count, M))
    for e0 in range(0, count, chunk):
        E = min(chunk, count - e0)
        z = rng.uniform(-1.0, 1.0, E)
        phi = rng.uniform(0.0, 2.0 * np.pi, E)
        rho = np.sqrt(1.0 - z * z)
        u = np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)      # [E][3]
        d = -(u @ xyz.T) * fs / c                                           # [E][M]
        S = rng.standard_normal((E, f.size)) + 1j * rng.standard_normal((E, f.size))
        S[:, 0] = S[:, 0].real
        S[:, -1] = 0.0
        phase = np.exp(-2j * np.pi * f[None, None, :] * d[:, :, None] / Lp)  # [E][M][F]
        H = phase
        if rt60 is not None:
            n = np.arange(1, Lp)
            T60 = rng.uniform(rt60[0], rt60[1], (E, M, 1)) * fs
            tail = rng.standard_normal((E, M, Lp - 1)) * np.exp(-6.907755 * n[None, None, :] / T60)
            drr = rng.uniform(drr_db[0], drr_db[1], (E, M, 1))
            tail *= np.sqrt(10.0 ** (-drr / 10.0) / np.sum(tail * tail, axis=-1, keepdims=True))
            h = np.concatenate([np.zeros((E, M, 1)), tail], axis=-1)          # starts one sample late
            H = phase * (1.0 + np.fft.rfft(h, n=Lp, axis=-1))                  # tail follows the direct path
        sig = np.fft.irfft(S[:, None, :] * H, n=Lp, axis=-1)[:, :, N // 2: N // 2 + N]
        p = np.mean(sig * sig, axis=-1, keepdims=True)
        snr = rng.uniform(snr_db[0], snr_db[1], (E, M, 1))
        sig = sig + rng.standard_normal(sig.shape) * np.sqrt(p * 10.0 ** (-snr / 10.0))
        x[:, e0 * N:(e0 + E) * N] = sig.transpose(1, 0, 2).reshape(M, E * N)
        delays[e0:e0 + E] = d
    return x, delays, xyz


def pair_room(seed: int, d: float, seconds: float = 1.0, fs: float = 16000.0,
              c_range=(335.0, 350.0), rt60_range=(0.1, 0.6), drr_db=(0.0, 10.0),
              snr_db=(10.0, 30.0)):
    """Two microphones `d` metres apart on the x axis and a white far-field
    source at angle theta from that axis (uniform in (0, pi)), with a speed of
    sound uniform in `c_range`; each mic hears the fractionally delayed direct
    path plus its own exponentially decaying reverberant tail (RT60 and
    direct-to-reverberant ratio uniform in their ranges) and white sensor noise.

    Returns (x [2][L] float32, tdoa, theta, c) with tdoa = t_0 - t_1 =
    d cos(theta) fs / c in samples."""
    from scipy.signal import fftconvolve
    rng = np.random.default_rng(seed)
    L = int(round(seconds * fs))
    theta = rng.uniform(0.0, np.pi)
    c = rng.uniform(*c_range)
    tdoa = d * np.cos(theta) * fs / c
    pad = 64
    s = rng.standard_normal(L + 2 * pad)
    delays = (0.5 * tdoa, -0.5 * tdoa)                   # arrival times about the centre
    rt60 = rng.uniform(*rt60_range)
    x = np.empty((2, L))
    for m in range(2):
        direct = fractional_delay(s, delays[m], pad, L)
        h = _reverb_fir(rng, fs, rt60)                    # unit direct path, unit-energy tail
        h[1:] *= np.sqrt(10.0 ** (-rng.uniform(*drr_db) / 10.0))
        rev = fftconvolve(direct, h)[:L]
        x[m] = rev + _snr_noise(rng, rev, rng.uniform(*snr_db))
    return x.astype(np.float32), float(tdoa), float(theta), float(c)


def sphere_grid(G: int, upper: bool = False) -> np.ndarray:
    """G unit vectors spread evenly over the sphere (or the upper half, z >= 0)
    by the Fibonacci lattice; [G][3] float64."""
    k = np.arange(G, dtype=np.float64) + 0.5
    z = 1.0 - k / G if upper else 1.0 - 2.0 * k / G
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = np.pi * (3.0 - np.sqrt(5.0)) * k
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def random_planar_array(rng, M: int, aperture: float) -> np.ndarray:
    """M microphones uniformly in a disc, rescaled so that the largest
    distance between two of them is `aperture` metres; [M][3], z = 0."""
    r = np.sqrt(rng.uniform(0.0, 1.0, M))
    phi = rng.uniform(0.0, 2.0 * np.pi, M)
    xy = np.stack([r * np.cos(phi), r * np.sin(phi)], axis=1)
    d = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1)).max()
    xy *= aperture / d
    return np.concatenate([xy, np.zeros((M, 1))], axis=1)


def batch_arrays(seed: int, count: int, seconds: float):
    """`count` independent arrays: M uniform in {2..16} on random planar layouts
    of 2-10 cm aperture, f_S in {16, 48} kHz, N in {256, 512, 1024} with hop N/4,
    each hearing an AR(2) source from a random azimuth (integer delays) with
    sensor noise at an SNR uniform in [0, 20] dB.  Returns a list of dicts with
    xyz, fs, N, hop and x [M][L] float32."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        M = int(rng.integers(2, 17))
        xyz = random_planar_array(rng, M, rng.uniform(0.02, 0.10))
        fs = float(rng.choice([16000.0, 48000.0]))
        N = int(rng.choice([256, 512, 1024]))
        L = int(round(seconds * fs))
        az = rng.uniform(0.0, 2.0 * np.pi)
        delays = np.rint(far_field_delays(xyz, az, fs, 343.0)).astype(np.int64)
        pad = int(np.abs(delays).max()) + 8
        s = _ar2(rng, L + 2 * pad, 0.95, rng.uniform(0.05 * np.pi, 0.45 * np.pi) * (16000.0 / fs))
        x = np.stack([_integer_delay(s, int(d), L, pad) for d in delays])
        snr = rng.uniform(0.0, 20.0, M)
        x = x + np.stack([_snr_noise(rng, x[m], snr[m]) for m in range(M)])
        out.append({"xyz": xyz, "fs": fs, "N": N, "hop": N // 4, "x": x.astype(np.float32)})
    return out
