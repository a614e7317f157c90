"""Learned sub-sample TDoA on top of FCC (binding of the fcc_mlp_* and
fcc_tdoa_learned calls of libfcc.so).

A small MLP maps the rank-D projection coefficients of one pair-frame
(eq. 9, from ``Plan.coefficients``) to a TDoA in samples and a confidence:

    u = c / ||c||,  h1 = gelu(u W1 + b1),  h2 = gelu(h1 W2 + b2),  (mu, s) = h2 W3 + b3

with s (clipped to [-8, 8]) the log-variance of a Gaussian error model and
exp(-s / 2) the confidence.  Forward, backward and the Adam update are HIP
kernels (FP16 matrix cores, FP32 elsewhere); this module only allocates
tensors, orders the calls and picks minibatches.  Below a confidence
threshold the estimate falls back to the FCC argmax refined by quadratic
interpolation (Sec. 2), which is also the yardstick of its error.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _lib
from . import _ptr, _stream_handle, _torch, check_out, check_workspace

__all__ = ["Mlp", "num_params", "init_params", "tdoa_learned", "learned_workspace_bytes",
           "choose_threshold"]


def num_params(in_dim: int, hidden: int) -> int:
    return int(_lib.load().fcc_mlp_num_params(in_dim, hidden))


def init_params(in_dim: int, hidden: int, seed: int = 0) -> np.ndarray:
    """He-style normal initialisation, zero biases; flat float32 in the
    library's layout W1 [in][H], b1, W2 [H][H], b2, W3 [H][2], b3."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal((in_dim, hidden)) * math.sqrt(2.0 / in_dim), np.zeros(hidden),
             rng.standard_normal((hidden, hidden)) * math.sqrt(2.0 / hidden), np.zeros(hidden),
             rng.standard_normal((hidden, 2)) * math.sqrt(1.0 / hidden), np.zeros(2)]
    theta = np.concatenate([p.ravel() for p in parts]).astype(np.float32)
    assert theta.size == num_params(in_dim, hidden)
    return theta


class Mlp:
    """Parameters and Adam state of one network on one HIP device."""

    def __init__(self, in_dim: int, hidden: int = 128, params=None, seed: int = 0, device="cuda"):
        torch = _torch()
        self._lib = _lib.load()
        self.in_dim, self.hidden = int(in_dim), int(hidden)
        n = num_params(self.in_dim, self.hidden)
        if n == 0:
            raise ValueError("invalid network shape")
        host = init_params(self.in_dim, self.hidden, seed) if params is None else \
            np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        if host.size != n:
            raise ValueError(f"expected {n} parameters, got {host.size}")
        self.params = torch.from_numpy(host).to(torch.device(device))
        self.device = self.params.device              # with its index
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss_sum = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.step = 0
        self._ws = None

    @property
    def num_params(self) -> int:
        return self.params.numel()

    def _workspace(self, rows: int):
        torch = _torch()
        nbytes = ctypes.c_size_t()
        _lib.check(self._lib.fcc_mlp_workspace_bytes(self.in_dim, self.hidden, rows, ctypes.byref(nbytes)))
        need = max(nbytes.value, 256)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def _check_rows(self, coef):
        torch = _torch()
        if not isinstance(coef, torch.Tensor) or coef.device != self.params.device:
            raise TypeError("coefficients must be a torch tensor on the network's device")
        if coef.dtype != torch.float32 or not coef.is_contiguous():
            raise ValueError("coefficients must be contiguous float32")
        if coef.dim() < 1 or coef.shape[-1] != self.in_dim:
            raise ValueError(f"coefficients must end in a dimension of {self.in_dim}")
        return coef.numel() // self.in_dim

    def forward(self, coef, out=None):
        """coef [..., in_dim] -> [..., 2] = (mu, s)."""
        torch = _torch()
        R = self._check_rows(coef)
        if out is None:
            out = torch.empty(tuple(coef.shape[:-1]) + (2,), dtype=torch.float32, device=self.device)
        else:
            check_out(out, tuple(coef.shape[:-1]) + (2,), torch.float32, self.device)
        ws = self._workspace(R)
        with torch.cuda.device(self.device):
            _lib.check(self._lib.fcc_mlp_forward(_ptr(self.params), self.in_dim, self.hidden, _ptr(coef), R,
                                                 _ptr(out), _ptr(ws), _stream_handle(self.device)))
        return out

    def loss_and_grad(self, coef, target, out=None):
        """Mean Gaussian NLL of the rows against `target` (samples); the
        gradient lands in ``self.grad``.  Returns (loss tensor [1], out)."""
        torch = _torch()
        R = self._check_rows(coef)
        if target.dtype != torch.float32 or not target.is_contiguous() or target.numel() != R:
            raise ValueError("target must be contiguous float32 with one value per row")
        if target.device != self.device:
            raise ValueError("target must be on the network's device")
        if out is None:
            out = torch.empty((R, 2), dtype=torch.float32, device=self.device)
        else:
            check_out(out, (R, 2), torch.float32, self.device)
        ws = self._workspace(R)
        self.loss_sum.zero_()
        with torch.cuda.device(self.device):
            _lib.check(self._lib.fcc_mlp_backward(_ptr(self.params), self.in_dim, self.hidden, _ptr(coef),
                                                  _ptr(target), R, _ptr(self.grad), _ptr(self.loss_sum),
                                                  _ptr(out), _ptr(ws), _stream_handle(self.device)))
        return self.loss_sum / max(R, 1), out

    def adam(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        """One Adam step with the gradient currently in ``self.grad``."""
        torch = _torch()
        self.step += 1
        with torch.cuda.device(self.device):
            _lib.check(self._lib.fcc_mlp_adam(_ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(self.grad),
                                              self.num_params, lr, beta1, beta2, eps, self.step,
                                              _stream_handle(self.device)))

    def fit(self, coef, target, epochs: int = 10, batch: int = 1024, lr: float = 2e-3,
            lr_final: float | None = None, seed: int = 0):
        """Minibatch Adam over contiguous row blocks in a fresh random block
        order each epoch (rows are expected in random order already).  The
        learning rate decays by cosine from `lr` to `lr_final` (default lr/20).
        Returns the mean loss of each epoch."""
        torch = _torch()
        R = self._check_rows(coef)
        coef = coef.reshape(R, self.in_dim)
        target = target.reshape(R)
        nb = (R + batch - 1) // batch
        rng = np.random.default_rng(seed)
        lr_final = lr / 20.0 if lr_final is None else lr_final
        total = epochs * nb
        history = []
        done = 0
        for _ in range(epochs):
            acc = torch.zeros(1, dtype=torch.float32, device=self.device)
            for b in rng.permutation(nb):
                lo, hi = int(b) * batch, min(R, (int(b) + 1) * batch)
                loss, _ = self.loss_and_grad(coef[lo:hi], target[lo:hi])
                acc += loss * (hi - lo)
                rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * done / total))
                self.adam(rate)
                done += 1
            history.append(float(acc.item()) / R)
        return history


def learned_workspace_bytes(plan, hidden: int, num_frames: int) -> int:
    nbytes = ctypes.c_size_t()
    _lib.check(plan._lib.fcc_learned_workspace_bytes(plan._h, hidden, num_frames, ctypes.byref(nbytes)))
    return nbytes.value


def tdoa_learned(plan, spec, mlp: Mlp, min_confidence: float, tau=None, confidence=None, workspace=None):
    """Learned TDoA [T, P] float32 (samples) from the plan's spectra, falling
    back to the interpolated FCC lag where the confidence is below
    `min_confidence`.  Returns (tau, confidence)."""
    torch = _torch()
    T = plan._check_spec(spec)
    if mlp.in_dim != 2 * plan.rank or mlp.device != spec.device:
        raise ValueError("network input must be 2 * rank on the spectra's device")
    if tau is None:
        tau = torch.empty((T, plan.P), dtype=torch.float32, device=spec.device)
    else:
        check_out(tau, (T, plan.P), torch.float32, spec.device, "tau")
    if confidence is None:
        confidence = torch.empty((T, plan.P), dtype=torch.float32, device=spec.device)
    else:
        check_out(confidence, (T, plan.P), torch.float32, spec.device, "confidence")
    if workspace is None:
        workspace = torch.empty(max(learned_workspace_bytes(plan, mlp.hidden, T), 256), dtype=torch.uint8,
                                device=spec.device)
    else:
        check_workspace(workspace, learned_workspace_bytes(plan, mlp.hidden, T), spec.device)
    basis = plan.basis_tensor(spec.device)
    with torch.cuda.device(spec.device):
        _lib.check(plan._lib.fcc_tdoa_learned(plan._h, _ptr(basis), _ptr(spec), T, _ptr(mlp.params),
                                              mlp.hidden, float(min_confidence), _ptr(tau), _ptr(confidence),
                                              _ptr(workspace), _stream_handle(spec.device)))
    return tau, confidence


def choose_threshold(mu, confidence, fallback, target, candidates=None) -> float:
    """Confidence threshold with the least mean absolute error on a
    validation set (host arrays); +inf means always fall back."""
    mu, confidence, fallback, target = (np.asarray(a, dtype=np.float64).ravel()
                                        for a in (mu, confidence, fallback, target))
    if candidates is None:
        candidates = np.concatenate([[0.0], np.quantile(confidence, np.linspace(0.0, 0.99, 100)), [np.inf]])
    best, best_c = np.inf, np.inf
    for c in candidates:
        err = np.abs(np.where(confidence >= c, mu, fallback) - target).mean()
        if err < best:
            best, best_c = err, float(c)
    return best_c
