"""Batches of independent arrays (binding of the fcc_batch_* calls).

    batch = Batch([plan_a, plan_b, ...], [L_a, L_b, ...])
    audio = batch.pack([x_a, x_b, ...])       # one device buffer, each [M_a, L_a]
    tdoa = batch.tdoa(audio)                  # one int32 buffer
    per_array = batch.split(tdoa)             # [T_a, P_a] views
    batch.tune(audio)                         # pick tile shapes by timing them

The library runs the front end in one launch per frame size present and the
pair stage in one launch per class of arrays sharing a matrix-core tile
shape, optionally captured once into a graph and replayed; this module only
allocates the buffers and marshals the calls.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from . import _ptr, _stream_handle, _torch

__all__ = ["Batch"]


class Batch:
    def __init__(self, plans, num_samples, device="cuda"):
        torch = _torch()
        self._lib = _lib.load()
        self.plans = list(plans)
        n = len(self.plans)
        if n == 0 or len(num_samples) != n:
            raise ValueError("one length per plan")
        handles = (ctypes.c_void_p * n)(*[p._h for p in self.plans])
        lengths = (ctypes.c_int64 * n)(*[int(v) for v in num_samples])
        h = ctypes.c_void_p()
        _lib.check(self._lib.fcc_batch_create(handles, n, lengths, ctypes.byref(h)))
        self._h = h
        self.info = _lib.FccBatchInfo()
        _lib.check(self._lib.fcc_batch_query(self._h, ctypes.byref(self.info)))
        ao, to, nf = (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)()
        _lib.check(self._lib.fcc_batch_layout(self._h, ao, to, nf))
        self.num_samples = [int(v) for v in num_samples]
        self.audio_offset, self.tdoa_offset, self.frames = list(ao), list(to), list(nf)
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.image = self._aligned(self.info.image_bytes)
        with torch.cuda.device(self.device):
            _lib.check(self._lib.fcc_batch_upload(self._h, _ptr(self.image), _stream_handle(self.device)))
        self.workspace = self._aligned(self.info.workspace_bytes)

    def _aligned(self, nbytes):
        torch = _torch()
        raw = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        return raw[off:off + int(nbytes)]

    def pack(self, signals):
        """One device buffer holding every array's [M_a, L_a] audio."""
        torch = _torch()
        out = torch.empty(max(self.info.audio_floats, 1), dtype=torch.float32, device=self.device)
        for a, (x, p) in enumerate(zip(signals, self.plans)):
            x = torch.as_tensor(x, dtype=torch.float32)
            if tuple(x.shape) != (p.M, self.num_samples[a]):
                raise ValueError(f"array {a}: expected [{p.M}, {self.num_samples[a]}]")
            o = self.audio_offset[a]
            out[o:o + x.numel()].copy_(x.reshape(-1).to(self.device))
        return out

    def _check_audio(self, audio):
        torch = _torch()
        if (not isinstance(audio, torch.Tensor) or audio.dtype != torch.float32 or not audio.is_contiguous()
                or audio.device != self.device):
            raise ValueError("audio must be the packed float32 buffer on the batch's device")
        if audio.numel() < self.info.audio_floats:
            raise ValueError("audio buffer too small")

    def _check_out(self, out):
        torch = _torch()
        if (not isinstance(out, torch.Tensor) or out.dtype != torch.int32 or not out.is_contiguous()
                or out.device != self.device):
            raise ValueError("out must be a contiguous int32 tensor on the batch's device")
        if out.numel() < self.info.tdoa_count:
            raise ValueError(f"out holds {out.numel()} values, {self.info.tdoa_count} needed")

    def tdoa(self, audio, out=None, graph=True):
        torch = _torch()
        self._check_audio(audio)
        if out is not None:
            self._check_out(out)
        if out is None:
            # one output buffer per batch, so a captured graph is reused; the
            # next call overwrites it unless `out` is given
            if getattr(self, "_out", None) is None:
                self._out = torch.empty(max(self.info.tdoa_count, 1), dtype=torch.int32, device=self.device)
            out = self._out
        with torch.cuda.device(self.device):
            _lib.check(self._lib.fcc_batch_tdoa(self._h, _ptr(self.image), _ptr(audio), _ptr(out),
                                                _ptr(self.workspace), 1 if graph else 0,
                                                _stream_handle(self.device)))
        return out

    def tune(self, audio, out=None):
        """Times candidate pair-stage tile shapes on these buffers and keeps
        the fastest; returns the shapes in use."""
        torch = _torch()
        self._check_audio(audio)
        if out is None:
            out = torch.empty(max(self.info.tdoa_count, 1), dtype=torch.int32, device=self.device)
        else:
            self._check_out(out)
        with torch.cuda.device(self.device):
            _lib.check(self._lib.fcc_batch_tune(self._h, _ptr(self.image), _ptr(audio), _ptr(out),
                                                _ptr(self.workspace), _stream_handle(self.device)))
        return self.tuning()

    def tuning(self):
        cap = 2 + 3 * self.info.num_classes
        v = (ctypes.c_int32 * cap)()
        _lib.check(self._lib.fcc_batch_tuning(self._h, v, cap))
        v = list(v)
        return {"front_end": {"launches": v[0]},
                "pair_classes": [{"workgroups": v[2 + 3 * c], "waves": v[3 + 3 * c],
                                  "blocks_per_cu": v[4 + 3 * c]} for c in range(self.info.num_classes)]}

    def split(self, tdoa):
        """Per-array [T_a, P_a] views of a batch output."""
        return [tdoa[o:o + T * p.P].view(T, p.P)
                for o, T, p in zip(self.tdoa_offset, self.frames, self.plans)]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fcc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
