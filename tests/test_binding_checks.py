"""Caller-supplied outputs and workspaces are checked by the binding before
anything is launched: the library writes through bare pointers, so a tensor
of the wrong shape, type, layout or device, or a workspace that is too small,
must be refused on the host."""
import numpy as np
import pytest
import torch

from paper_2204_13622_amd import check_out, check_workspace


def test_check_out_accepts_exact_tensor():
    t = torch.empty((7, 120), dtype=torch.int32)
    assert check_out(t, (7, 120), torch.int32, "cpu") is t


@pytest.mark.parametrize("bad", [
    torch.empty((7, 119), dtype=torch.int32),            # one pair short
    torch.empty((8, 120), dtype=torch.int32),            # one frame too many
    torch.empty((7 * 120,), dtype=torch.int32),          # right size, wrong shape
    torch.empty((7, 120), dtype=torch.float32),          # wrong type
    torch.empty((120, 7), dtype=torch.int32).t(),        # not contiguous
    np.empty((7, 120), dtype=np.int32),                  # not a tensor
])
def test_check_out_refuses(bad):
    with pytest.raises(ValueError):
        check_out(bad, (7, 120), torch.int32, "cpu")


def test_check_out_refuses_other_device():
    t = torch.empty((2, 3), dtype=torch.float32, device="meta")
    with pytest.raises(ValueError):
        check_out(t, (2, 3), torch.float32, "cpu")


def test_check_workspace():
    ws = torch.empty(1024, dtype=torch.uint8)
    assert check_workspace(ws, 1024, "cpu") is ws
    assert check_workspace(torch.empty(256, dtype=torch.float32), 1024, "cpu") is not None   # 1024 bytes
    with pytest.raises(ValueError):
        check_workspace(ws, 1025, "cpu")
    with pytest.raises(ValueError):
        check_workspace(torch.empty((64, 32), dtype=torch.uint8).t(), 16, "cpu")
    with pytest.raises(ValueError):
        check_workspace(torch.empty(4096, dtype=torch.uint8, device="meta"), 16, "cpu")
