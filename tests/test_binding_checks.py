"""The binding rejects bad buffers before any launch (CPU only).

A device-pointer entry point reads and writes ``B * n * 2 * L`` doubles of x and
y (and n times that of the Jacobian); a host tensor, a float32 tensor or a
buffer that is too small would become an out-of-bounds access on the GPU, so
the wrappers raise ``QdpError`` first.  No handle is created and no kernel is
launched here: the stand-in handle below only carries n.
"""

import types

import numpy as np
import pytest
import torch

from paper_1109_0545_amd import binding as b

H = types.SimpleNamespace(n=4, handle=None, system=None)
SYS = types.SimpleNamespace(n=4, handle=None)


def _raises(fn, *a, **k):
    with pytest.raises(b.QdpError) as e:
        fn(*a, **k)
    assert e.value.status == 1
    return str(e.value)


def test_dev_checks_each_property():
    msg = _raises(b._dev, torch.zeros(8, dtype=torch.float64), "x", 8)
    assert "not on the GPU" in msg
    assert "torch tensor" in _raises(b._dev, np.zeros(8), "x", 8)
    assert "required" in _raises(b._dev, None, "x", 8)
    assert b._dev(None, "scale", 8, nullable=True) is None


def test_device_wrappers_reject_host_tensors_before_launch():
    x = torch.zeros(4 * 2 * 2, dtype=torch.float64)
    y = torch.zeros(4 * 2 * 2, dtype=torch.float64)
    jac = torch.zeros(4 * 4 * 2 * 2, dtype=torch.float64)
    _raises(b.newton_step_dev, H, 0.5, x, 2)
    _raises(b.newton_batch_dev, H, 0.5, x, 1, 2)
    _raises(b.eval_homotopy_dev, H, 0.5, x, 2, y, jac)
    _raises(b.eval_homotopy_batch_dev, H, 0.5, x, 1, 2, y, jac)
    _raises(b.eval_jacobian_dev, SYS, x, 2, y, jac)


def test_batch_size_must_be_positive():
    x = torch.zeros(16, dtype=torch.float64)
    assert "batch size" in _raises(b.newton_batch_dev, H, 0.5, x, 0, 2)


def test_host_entry_points_check_shapes():
    assert "shape" in _raises(b.newton_step, H, 0.5, np.zeros((3, 2, 2)), 2)
    assert "shape" in _raises(b.eval_homotopy, H, 0.5, np.zeros((4, 2, 1)), 2)
    assert "shape" in _raises(b.track_paths, H, np.zeros((4, 2, 2)), 2)


def test_system_shapes_are_checked_before_the_library_reads_them():
    off = np.array([0, 2, 3], dtype=np.int32)
    exps = np.zeros((3, 2), dtype=np.uint8)
    coefs = np.zeros((3, 2, 2))
    assert "poly_offsets" in _raises(b.System, 3, off, exps, coefs, 2)
    assert "exps" in _raises(b.System, 2, off, np.zeros((2, 2), dtype=np.uint8), coefs, 2)
    assert "coefs" in _raises(b.System, 2, off, exps, np.zeros((3, 2, 1)), 2)


def test_noncontiguous_host_array_is_rejected():
    a = np.zeros((4, 4))[:, ::2]
    assert "contiguous" in _raises(b._ptr, a)


def test_set_elimination_accepts_the_layouts_and_rejects_others():
    # qdp_set_elimination only records a process-wide choice (no device call)
    for policy in (b.ELIM_POINT, b.ELIM_COLUMNS, b.ELIM_BLOCKS, b.ELIM_AUTO):
        b.set_elimination(policy)
    for bad in (-1, 4):
        assert "policy" in _raises(b.set_elimination, bad)
    b.set_elimination(b.ELIM_AUTO)
