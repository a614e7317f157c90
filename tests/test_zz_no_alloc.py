"""fcc_tdoa_noalloc (the entry point that allocates nothing) against fcc_tdoa:
the same kernels on the same frames, so the integer lags must be equal bit
for bit.  Two calls in a row on one GPU, the second with a smaller input,
since every call shares the GPU's static scratch array."""
import sys

import numpy as np
import pytest

from gen import make_recording

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


@pytest.mark.parametrize("precision,D", [("fp16", 11), ("fp32", 6), ("fp8", 6)])
def test_noalloc_equals_workspace_path(torch, fcc, precision, D):
    rec = make_recording(2)                      # 60 s: T = 7497 frames, 120 pairs
    p = fcc.Plan(rec.mic_xyz, rec.fs, rec.c, frame_size=rec.N, hop=rec.hop, rank=D, precision=precision)
    frame_bytes = p.info.spectrum_bytes_per_frame
    chunk = fcc._lib.NOALLOC_SCRATCH_BYTES // frame_bytes
    x = torch.from_numpy(rec.x).cuda()
    # first call: the whole recording (several chunks); second: a ragged
    # prefix of fewer frames than one chunk holds, on the same scratch
    for L in (rec.L, 1000 * rec.hop + rec.N + 77):
        T = p.num_frames(L)
        _say(f"noalloc {precision} D={D} T={T} chunk={chunk} frames")
        xs = x[:, :L]
        t_ref = p.tdoa(xs)
        t = p.tdoa_noalloc(xs)
        torch.cuda.synchronize()
        assert tuple(t.shape) == (T, 120)
        assert torch.equal(t, t_ref), int((t != t_ref).sum())
    assert p.num_frames(rec.L) > chunk or precision == "fp8"   # the first call spans chunks


def test_noalloc_refusals(torch, fcc):
    _say("noalloc refusals")
    rec = make_recording(1)
    p = fcc.Plan(rec.mic_xyz, rec.fs, rec.c, frame_size=rec.N, hop=rec.hop, alpha=0.5)
    with pytest.raises(fcc.FccError) as ei:
        p.tdoa_noalloc(torch.from_numpy(rec.x).cuda())
    assert ei.value.name == "FCC_ERR_UNSUPPORTED"
    q = fcc.Plan(rec.mic_xyz, rec.fs, rec.c, frame_size=rec.N, hop=rec.hop)
    x = torch.from_numpy(rec.x).cuda()
    with pytest.raises(ValueError):
        q.tdoa_noalloc(x, out=torch.empty((3, q.P), dtype=torch.int32, device="cuda"))
    assert tuple(q.tdoa_noalloc(x[:, :100]).shape) == (0, q.P)     # no frame: nothing enqueued
