"""The Newton entry point that allocates nothing (qdp_newton_step_noalloc_dev)
against qdp_newton_step_dev on the same inputs: bit for bit equal points and
equal Newton info, on two calls in a row, the second with a smaller system;
and the rejection of a system too large for its static workspace."""

import numpy as np
import pytest

from synth.systems import CONFIGS, config_system, make_system, random_point
from tests.gpu_helpers import fixture, say

pytestmark = pytest.mark.gpu


def _case(name):
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS[name])
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    fix = fixture(name)
    x = np.zeros((s.n, 2, 2))
    for v, (re, im) in enumerate(fix["x_half_f64"]):
        x[v, 0, 0] = re * (1 + 1e-6)
        x[v, 1, 0] = im
    return s, H, x


def _compare(H, x, t, mode, max_it):
    import torch

    import paper_1109_0545_amd as q

    stream = torch.cuda.current_stream()
    xa = torch.from_numpy(x.copy()).cuda()
    xb = torch.from_numpy(x.copy()).cuda()
    info_b = torch.zeros(64, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    q.newton_step_dev(H, t, xa, 2, mode=mode, eps=0.0, max_it=max_it, stream=stream)
    ia = q.last_info(H, 2, stream=stream)
    q.newton_step_noalloc_dev(H, t, xb, 2, mode=mode, eps=0.0, max_it=max_it, info=info_b, stream=stream)
    torch.cuda.synchronize()
    ib = q.info_from_bytes(info_b.cpu().numpy())
    assert np.array_equal(xa.cpu().numpy(), xb.cpu().numpy())
    assert ia == ib, (ia, ib)
    assert ib["iterations"] == max_it and not ib["singular"]
    return ib


def test_noalloc_matches_newton_step_dev_twice_then_smaller():
    say("no-alloc newton: n64_dd full, then n64_dd mixed, then n8_dd full")
    s, H, x = _case("n64_dd")
    _compare(H, x, 0.5, 0, 2)
    info = _compare(H, x, 0.5, 1, 2)
    assert info["refine_steps"] >= 1
    s8, H8, x8 = _case("n8_dd")  # second system, smaller: the scratch keeps the last call's contents
    _compare(H8, x8, 0.5, 0, 3)


def test_noalloc_common_support_system():
    # a common-support system also takes the monomial-partials scratch
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS["c40_dd"])
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    x = s.zstar.copy()
    x[:, :, 0] += 1e-6
    x[:, :, 1] = 0.0
    say("no-alloc newton: c40_dd common support")
    _compare(H, x, 1.0, 0, 2)


def test_noalloc_rejects_a_system_beyond_its_workspace():
    import torch

    import paper_1109_0545_amd as q

    s = make_system(256, 4, 2, 2, 77)
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    x = torch.from_numpy(random_point(256, 2, seed=3, spread=0.1)).cuda()
    say("no-alloc newton: n=256 rejected")
    with pytest.raises(q.QdpError) as e:
        q.newton_step_noalloc_dev(H, 0.5, x, 2, eps=0.0, max_it=1)
    assert e.value.status == 1 and "workspace" in str(e.value)
