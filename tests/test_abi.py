"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, and its host-only defaults match the readings the oracle uses.  No
GPU work is launched here."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qdpath.h")


def _lib_path():
    from paper_1109_0545_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        from paper_1109_0545_amd.build import build

        build()
    return binding.LIB_PATH


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qdp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("qdp_eval_jacobian", "qdp_newton_step", "qdp_track_path", "qdp_system_create",
                 "qdp_homotopy_create", "qdp_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", _lib_path()], capture_output=True, text=True).stdout
    for n in declared_functions():
        assert re.search(rf"\bT {n}$", out, flags=re.M), n


def test_binding_covers_every_symbol():
    from paper_1109_0545_amd.binding import SIGNATURES

    assert set(declared_functions()) <= set(SIGNATURES)


def test_track_defaults_match_oracle_readings():
    _lib_path()
    import paper_1109_0545_amd as q
    from oracle.track import TrackParams

    p = q.default_track_params()
    o = TrackParams()
    for f in ("lambda0", "lambda_min", "lambda_max", "shrink", "expand", "expand_after", "eps_path",
              "max_it_path", "max_it_end", "max_steps"):
        assert getattr(p, f) == getattr(o, f), f
    assert p.predictor == q.PRED_SECANT and p.mode == q.SOLVE_FULL


def test_errors_are_reported_without_gpu_work():
    _lib_path()
    import numpy as np

    import paper_1109_0545_amd as q

    # invalid arguments are rejected before any device call
    with pytest.raises(q.QdpError) as e:
        q.System(0, np.zeros(1, np.int32), np.zeros((0, 0), np.uint8), np.zeros((0, 2, 2)), 2)
    assert e.value.status == 1
    with pytest.raises(q.QdpError) as e:
        q.System(2, np.array([0, 1, 1], np.int32), np.zeros((1, 2), np.uint8), np.zeros((1, 2, 2)), 2)
    assert "at least one term" in str(e.value)
    with pytest.raises(q.QdpError) as e:
        q.System(1, np.array([0, 1], np.int32), np.zeros((1, 1), np.uint8), np.full((1, 2, 2), np.nan), 2)
    assert e.value.status == 4
    with pytest.raises(q.QdpError) as e:
        q.System(1, np.array([0, 1], np.int32), np.zeros((1, 1), np.uint8), np.zeros((1, 2, 3)), 3)
    assert e.value.status == 1


def test_batch_entry_points_reject_null_arguments():
    # errors found before any GPU work: NULL handles and buffers
    from paper_1109_0545_amd import binding as B

    lib = B.lib()
    assert lib.qdp_newton_batch_dev(None, 0.5, None, 4, 2, 0, 1e-10, 4, None) == 1
    assert lib.qdp_eval_homotopy_batch_dev(None, 0.5, None, 1, 2, None, None, None, None) == 1
    assert lib.qdp_homotopy_last_info_batch(None, 2, 1, None, None) == 1
    assert b"NULL" in lib.qdp_last_error()
