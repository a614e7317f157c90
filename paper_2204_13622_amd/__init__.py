"""MI355X (gfx950) Fast Cross-Correlation TDoA: Python binding of libfcc.so.

The binding only marshals arguments: every step of the path runs in the HIP
kernels of libfcc.so.  PyTorch provides device memory and the current stream.

    plan = Plan(mic_xyz, fs=16000, frame_size=512, hop=128, rank=6)
    tdoa = plan.tdoa(x)            # x: float32 [M, L] on a HIP device -> int32 [T, P]
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import FccError, PRECISIONS, METHODS

__all__ = ["Plan", "FccError", "PRECISIONS", "METHODS", "library_path"]


def library_path() -> str:
    return _lib.LIB_PATH


def _torch():
    import torch
    return torch


def _stream_handle(device) -> ctypes.c_void_p:
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _same_device(a, b) -> bool:
    torch = _torch()
    a, b = torch.device(a), torch.device(b)
    if a.type != b.type:
        return False
    if a.type != "cuda":
        return True
    cur = torch.cuda.current_device() if torch.cuda.is_available() else 0
    return (a.index if a.index is not None else cur) == (b.index if b.index is not None else cur)


def check_out(t, shape, dtype, device, name: str = "out"):
    """A caller-supplied output tensor: the exact shape, dtype, device and a
    contiguous layout, since the library writes every element of that shape
    through a bare pointer.  Raises ValueError before anything is launched."""
    torch = _torch()
    shape = tuple(int(v) for v in shape)
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if tuple(t.shape) != shape:
        raise ValueError(f"{name} must have shape {list(shape)}, got {list(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not _same_device(t.device, device):
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    return t


def check_workspace(ws, nbytes: int, device, name: str = "workspace"):
    """A caller-supplied scratch buffer: contiguous, on `device`, holding at
    least `nbytes` bytes.  Raises ValueError before anything is launched."""
    torch = _torch()
    if not isinstance(ws, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if not ws.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not _same_device(ws.device, device):
        raise ValueError(f"{name} must be on {device}, got {ws.device}")
    have = ws.numel() * ws.element_size()
    if have < int(nbytes):
        raise ValueError(f"{name} holds {have} bytes, {int(nbytes)} needed")
    return ws


class Plan:
    """One array geometry: FP64 basis built on the host, tables on each device.

    Arguments follow the problem statement of the paper (Sec. 2): microphone
    positions (metres), sample rate, speed of sound, frame size N, hop, lag
    range tau_max (0: from the geometry) and rank D (0: full rank).
    `operands` picks the matrix-core operand types of the 16- and 8-bit
    storage types: "fp16" (widened, the default) or "storage" (BF16 tiles for
    bf16 spectra, e4m3 tiles for fp8 spectra).
    """

    def __init__(self, mic_xyz, fs: float, c: float = 343.0, frame_size: int = 512,
                 hop: int = 128, tau_max: int = 0, rank: int = 0, interp: int = 1,
                 alpha: float = 1.0, precision: str = "fp32", method: str = "fcc",
                 operands: str = "fp16"):
        lib = _lib.load()
        self._lib = lib
        xyz = np.ascontiguousarray(np.asarray(mic_xyz, dtype=np.float64).reshape(-1, 3))
        self.mic_xyz = xyz
        self.precision = precision
        self.method = method
        cfg = _lib.FccConfig()
        cfg.num_mics = xyz.shape[0]
        cfg.mic_xyz = xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        cfg.fs, cfg.c = float(fs), float(c)
        cfg.frame_size, cfg.hop = int(frame_size), int(hop)
        cfg.tau_max, cfg.rank, cfg.interp = int(tau_max), int(rank), int(interp)
        cfg.alpha = float(alpha)
        if precision not in PRECISIONS or method not in METHODS or operands not in _lib.OPERANDS:
            raise ValueError(f"precision in {sorted(PRECISIONS)}, method in {sorted(METHODS)}, "
                             f"operands in {sorted(_lib.OPERANDS)}")
        cfg.precision = PRECISIONS[precision]
        cfg.method = METHODS[method]
        cfg.operands = _lib.OPERANDS[operands]
        self.operands = operands
        handle = ctypes.c_void_p()
        _lib.check(lib.fcc_plan_create(ctypes.byref(cfg), ctypes.byref(handle)))
        self._h = handle
        info = _lib.FccPlanInfo()
        _lib.check(lib.fcc_plan_query(self._h, ctypes.byref(info)))
        self.info = info
        self._basis = {}

    # ---- geometry / shapes -------------------------------------------------
    @property
    def M(self) -> int: return self.info.num_mics
    @property
    def P(self) -> int: return self.info.num_pairs
    @property
    def N(self) -> int: return self.info.frame_size
    @property
    def hop(self) -> int: return self.info.hop
    @property
    def F(self) -> int: return self.info.num_bins
    @property
    def tau_max(self) -> int: return self.info.tau_max
    @property
    def I(self) -> int: return self.info.num_lags
    @property
    def rank(self) -> int: return self.info.rank

    @staticmethod
    def pack_spectrum(e):
        """[..., N/2 + 1] complex bins -> [..., N/2, 2] packed real layout."""
        e = np.asarray(e)
        out = np.stack([e[..., :-1].real, e[..., :-1].imag], axis=-1)
        out[..., 0, 1] = e[..., -1].real
        return out

    @staticmethod
    def unpack_spectrum(a):
        """[..., N/2, 2] packed real layout -> [..., N/2 + 1] complex bins."""
        a = np.asarray(a, dtype=np.float64)
        e = np.empty(a.shape[:-2] + (a.shape[-2] + 1,), dtype=np.complex128)
        e[..., :-1] = a[..., 0] + 1j * a[..., 1]
        e[..., 0] = a[..., 0, 0]
        e[..., -1] = a[..., 0, 1]
        return e

    def pairs(self):
        return [(i, j) for i in range(self.M) for j in range(i + 1, self.M)]

    def num_frames(self, num_samples: int) -> int:
        out = ctypes.c_int64()
        _lib.check(self._lib.fcc_num_frames(self._h, int(num_samples), ctypes.byref(out)))
        return out.value

    def workspace_bytes(self, num_frames: int) -> int:
        out = ctypes.c_size_t()
        _lib.check(self._lib.fcc_workspace_bytes(self._h, int(num_frames), ctypes.byref(out)))
        return out.value

    def smooth_workspace_bytes(self, num_frames: int) -> int:
        out = ctypes.c_size_t()
        _lib.check(self._lib.fcc_smooth_workspace_bytes(self._h, int(num_frames), ctypes.byref(out)))
        return out.value

    @property
    def r(self) -> int:
        return self.info.interp

    @property
    def alpha(self) -> float:
        return self.info.alpha

    def new_state(self, device=None):
        """Zero smoothing state R [P, N/2 + 1, 2] float32 (alpha < 1)."""
        torch = _torch()
        return torch.zeros((self.P, self.N // 2 + 1, 2), dtype=torch.float32,
                           device=device if device is not None else "cuda")

    def tdoa_smoothed(self, spec, state=None, tdoa=True, tau=False, y=False, workspace=None):
        """Recursive smoothing (eq. 1, alpha < 1), per-pair PHAT and FCC over
        the frames of `spec` (raw spectra from ``spectra``), continuing from
        `state` [P, N/2 + 1, 2] (zeros when None), which is updated in place.
        Returns a dict with the requested outputs: 'tdoa' [T, P] int32
        (1/r sample), 'tau' [T, P] float32 (samples), 'y' [T, P, I] float32,
        and 'state'."""
        torch = _torch()
        T = self._check_spec(spec)
        dev = spec.device
        if state is None:
            state = self.new_state(dev)
        if (state.dtype != torch.float32 or not state.is_contiguous() or state.device != dev
                or tuple(state.shape) != (self.P, self.N // 2 + 1, 2)):
            raise ValueError(f"state must be contiguous float32 [{self.P}, {self.N // 2 + 1}, 2] on the device")
        out = {"state": state}
        if tdoa:
            out["tdoa"] = torch.empty((T, self.P), dtype=torch.int32, device=dev)
        if tau:
            out["tau"] = torch.empty((T, self.P), dtype=torch.float32, device=dev)
        if y:
            out["y"] = torch.empty((T, self.P, self.I), dtype=torch.float32, device=dev)
        if workspace is None:
            workspace = torch.empty(max(self.smooth_workspace_bytes(T), 256), dtype=torch.uint8, device=dev)
        else:
            check_workspace(workspace, self.smooth_workspace_bytes(T), dev)
        null = ctypes.c_void_p(0)
        basis = self.basis_tensor(dev)
        with torch.cuda.device(dev):
            _lib.check(self._lib.fcc_tdoa_smoothed(
                self._h, _ptr(basis), _ptr(spec), T, _ptr(state),
                _ptr(out["tdoa"]) if tdoa else null, _ptr(out["tau"]) if tau else null,
                _ptr(out["y"]) if y else null, _ptr(workspace), _stream_handle(dev)))
        return out

    def doa_table(self, dirs, device=None):
        """Fractional lag index of every pair for every unit direction,
        [P, G] float32 on `device` (built on the host in FP64)."""
        torch = _torch()
        d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        table = np.empty((self.P, d.shape[0]), dtype=np.float32)
        _lib.check(self._lib.fcc_doa_table(self._h, d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           d.shape[0], table.ctypes.data_as(ctypes.c_void_p)))
        return torch.from_numpy(table).to(device if device is not None else "cuda")

    def doa(self, y, table, score=False):
        """First best direction [T] int32 for correlations y [T, P, I]; with
        score=True also the scores [T, G].  Returns (doa, scores or None)."""
        torch = _torch()
        if y.dtype != torch.float32 or not y.is_contiguous() or y.dim() != 3 or \
                tuple(y.shape[1:]) != (self.P, self.I):
            raise ValueError(f"y must be contiguous float32 [T, {self.P}, {self.I}]")
        if table.dtype != torch.float32 or not table.is_contiguous() or table.dim() != 2 or \
                table.shape[0] != self.P or table.device != y.device:
            raise ValueError("table must be the plan's [P, G] float32 table on y's device")
        T, G = y.shape[0], table.shape[1]
        out = torch.empty(T, dtype=torch.int32, device=y.device)
        sc = torch.empty((T, G), dtype=torch.float32, device=y.device) if score else None
        with torch.cuda.device(y.device):
            _lib.check(self._lib.fcc_doa(self._h, _ptr(y), T, _ptr(table), G, _ptr(out),
                                         _ptr(sc) if score else ctypes.c_void_p(0),
                                         _stream_handle(y.device)))
        return out, sc

    def spectrum_dtype(self):
        torch = _torch()
        return {"fp32": torch.float32, "bf16": torch.bfloat16, "fp16": torch.float16,
                "fp8": torch.float8_e4m3fn, "fp8_e4m3": torch.float8_e4m3fn}[self.precision]

    # ---- device tables -------------------------------------------------------
    def basis_tensor(self, device=None):
        """The plan's packed tables on `device` (uploaded once per device)."""
        torch = _torch()
        dev = torch.device(device if device is not None else "cuda")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        buf = self._basis.get(dev.index)
        if buf is None:
            nbytes = self.info.basis_bytes
            raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
            off = (-raw.data_ptr()) % 256
            buf = raw[off:off + nbytes]
            with torch.cuda.device(dev):
                _lib.check(self._lib.fcc_plan_upload(self._h, _ptr(buf), _stream_handle(dev)))
            self._basis[dev.index] = buf
        return buf

    # ---- hot path ------------------------------------------------------------
    def _check_audio(self, x):
        torch = _torch()
        if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
            raise TypeError("x must be a torch tensor on a HIP device")
        if x.dtype != torch.float32 or x.dim() != 2 or x.shape[0] != self.M:
            raise ValueError(f"x must be float32 [M={self.M}, L]")
        if x.stride(1) != 1:
            raise ValueError("x rows must be contiguous")
        return x.shape[1], x.stride(0)

    def spectra(self, x, out=None):
        """Whitened spectra [T, M, N/2, 2] (re, im) in the plan's storage type,
        packed real layout: slot 0 holds (e(0), e(N/2)), slot f holds e(f)."""
        torch = _torch()
        L, ld = self._check_audio(x)
        T = self.num_frames(L)
        if out is None:
            out = torch.empty((T, self.M, self.N // 2, 2), dtype=self.spectrum_dtype(), device=x.device)
        else:
            check_out(out, (T, self.M, self.N // 2, 2), self.spectrum_dtype(), x.device)
        basis = self.basis_tensor(x.device)
        with torch.cuda.device(x.device):
            _lib.check(self._lib.fcc_spectra(self._h, _ptr(basis), _ptr(x), L, ld, _ptr(out),
                                             _stream_handle(x.device)))
        return out

    def tdoa(self, x, out=None, workspace=None):
        """Integer TDoA [T, P] (int32, samples) from audio x [M, L] float32."""
        torch = _torch()
        L, ld = self._check_audio(x)
        T = self.num_frames(L)
        if out is None:
            out = torch.empty((T, self.P), dtype=torch.int32, device=x.device)
        else:
            check_out(out, (T, self.P), torch.int32, x.device)
        if workspace is None:
            workspace = torch.empty(max(self.workspace_bytes(T), 256), dtype=torch.uint8,
                                    device=x.device)
        else:
            check_workspace(workspace, self.workspace_bytes(T), x.device)
        basis = self.basis_tensor(x.device)
        with torch.cuda.device(x.device):
            _lib.check(self._lib.fcc_tdoa(self._h, _ptr(basis), _ptr(x), L, ld, _ptr(out),
                                          _ptr(workspace), _stream_handle(x.device)))
        return out

    def tdoa_noalloc(self, x, out=None):
        """fcc_tdoa without a workspace: the library stages the spectra in its
        static per-GPU array (64 MiB) in chunks of frames.  Calls that overlap
        on one GPU race on that array."""
        torch = _torch()
        L, ld = self._check_audio(x)
        T = self.num_frames(L)
        if out is None:
            out = torch.empty((T, self.P), dtype=torch.int32, device=x.device)
        else:
            check_out(out, (T, self.P), torch.int32, x.device)
        basis = self.basis_tensor(x.device)
        with torch.cuda.device(x.device):
            _lib.check(self._lib.fcc_tdoa_noalloc(self._h, _ptr(basis), _ptr(x), L, ld, _ptr(out),
                                                  _stream_handle(x.device)))
        return out

    def _check_spec(self, spec):
        torch = _torch()
        if not isinstance(spec, torch.Tensor) or spec.device.type != "cuda":
            raise TypeError("spectra must be a torch tensor on a HIP device")
        if spec.dtype != self.spectrum_dtype() or not spec.is_contiguous():
            raise ValueError("spectra must be contiguous in the plan's storage type")
        if spec.dim() != 4 or tuple(spec.shape[1:]) != (self.M, self.N // 2, 2):
            raise ValueError(f"spectra must be [T, {self.M}, {self.N // 2}, 2]")
        return spec.shape[0]

    def tdoa_from_spectra(self, spec, out=None):
        torch = _torch()
        T = self._check_spec(spec)
        if out is None:
            out = torch.empty((T, self.P), dtype=torch.int32, device=spec.device)
        else:
            check_out(out, (T, self.P), torch.int32, spec.device)
        basis = self.basis_tensor(spec.device)
        with torch.cuda.device(spec.device):
            _lib.check(self._lib.fcc_tdoa_from_spectra(self._h, _ptr(basis), _ptr(spec), T,
                                                       _ptr(out), _stream_handle(spec.device)))
        return out

    def correlation(self, spec, out=None):
        """y [T, P, I] float32 at lags tau_i = i - tau_max."""
        torch = _torch()
        T = self._check_spec(spec)
        if out is None:
            out = torch.empty((T, self.P, self.I), dtype=torch.float32, device=spec.device)
        else:
            check_out(out, (T, self.P, self.I), torch.float32, spec.device)
        basis = self.basis_tensor(spec.device)
        with torch.cuda.device(spec.device):
            _lib.check(self._lib.fcc_correlation(self._h, _ptr(basis), _ptr(spec), T, _ptr(out),
                                                 _stream_handle(spec.device)))
        return out

    def coefficients(self, spec, out=None):
        """Projection coefficients of eq. (9): [T, P, 2D] float32, (a_k, b_k) interleaved."""
        torch = _torch()
        T = self._check_spec(spec)
        if out is None:
            out = torch.empty((T, self.P, 2 * self.rank), dtype=torch.float32, device=spec.device)
        else:
            check_out(out, (T, self.P, 2 * self.rank), torch.float32, spec.device)
        basis = self.basis_tensor(spec.device)
        with torch.cuda.device(spec.device):
            _lib.check(self._lib.fcc_coefficients(self._h, _ptr(basis), _ptr(spec), T, _ptr(out),
                                                  _stream_handle(spec.device)))
        return out

    def tdoa_parabolic(self, spec, out=None):
        """Argmax lag refined by quadratic interpolation: [T, P] float32, samples."""
        torch = _torch()
        T = self._check_spec(spec)
        if out is None:
            out = torch.empty((T, self.P), dtype=torch.float32, device=spec.device)
        else:
            check_out(out, (T, self.P), torch.float32, spec.device)
        basis = self.basis_tensor(spec.device)
        with torch.cuda.device(spec.device):
            _lib.check(self._lib.fcc_tdoa_parabolic(self._h, _ptr(basis), _ptr(spec), T, _ptr(out),
                                                    _stream_handle(spec.device)))
        return out

    # ---- host-side inspection ------------------------------------------------
    def basis_export(self) -> dict:
        D, I, Bs = self.rank, self.I, self.N // 4 + 1
        sigma = np.zeros(D)
        is_sym = np.zeros(D, dtype=np.int32)
        p_hat = np.zeros((D, Bs))
        dc = np.zeros((I, D))
        ds = np.zeros((I, D))
        dp = ctypes.POINTER(ctypes.c_double)
        _lib.check(self._lib.fcc_basis_export(
            self._h, sigma.ctypes.data_as(dp), is_sym.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            p_hat.ctypes.data_as(dp), dc.ctypes.data_as(dp), ds.ctypes.data_as(dp)))
        return {"sigma": sigma, "is_sym": is_sym.astype(bool), "p_hat": p_hat, "Dc": dc, "Ds": ds}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fcc_plan_destroy(self._h)
            self._h = None
        self._basis = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


from .batch import Batch  # noqa: E402,F401

__all__.append("Batch")
