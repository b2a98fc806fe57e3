"""Mixed-precision Newton correction (FP64 factorization + iterative
refinement in double or quad double) beside the full elimination: each
against the oracle's Newton iterations (fixtures written by
tests/golden/make_fixtures.py from oracle.newton), and the n = 128 path tracked
to its endpoint in both modes."""

import json
import os

import mpmath
import numpy as np
import pytest

from oracle.newton import newton_tolerance
from oracle.numbers import mpc_of
from oracle.track import correct_digits
from synth.systems import CONFIGS, config_system
from tests.gpu_helpers import HERE, say
from tests.test_gpu_track import track_config

pytestmark = pytest.mark.gpu

MODES = {0: "full", 1: "mixed"}


def newton_fixture(name):
    with open(os.path.join(HERE, "golden", f"newton_{name}.json")) as fh:
        return json.load(fh)


def iteration_errors(name, mode):
    """One GPU Newton iteration from each stored input point; per iteration the
    distance to the oracle's z + dz*, the one-step bound, |dz_gpu - dz*| and
    the GPU's residual."""
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS[name])
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    fix = newton_fixture(name)
    L = fix["L"]
    out = []
    for k, row in enumerate(fix["iterations"]):
        x = np.array(row["x_limbs"])
        say("newton iteration vs oracle", name, MODES[mode], "iteration", k)
        xg, info = q.newton_step(H, fix["t"], x, L, mode=mode, eps=0.0, max_it=1)
        with mpmath.workprec(700):
            xs = [mpc_of(x[v]) for v in range(s.n)]
            dz = [mpc_of(np.array(d)) for d in row["dz_limbs"]]
            zg = [mpc_of(xg[v]) for v in range(s.n)]
            err = max(float(abs(zg[v] - (xs[v] + dz[v]))) for v in range(s.n))
        tol = newton_tolerance(s.n, row["kappa"], L, row["dz_inf"], row["z_inf"], row["jinv"], row["h_scale"])
        out.append({"iteration": k, "err": err, "tol": tol, "dz_inf": row["dz_inf"], "info": info,
                    "rho_oracle": row["rho"]})
    return out


@pytest.mark.parametrize("name", ["n64_dd", "n128_dd", "n64_qd"])
@pytest.mark.parametrize("mode", [0, 1])
def test_newton_iterations_match_oracle(name, mode):
    # three iterations from a point 1e-6 off the path at t = 1/2: the
    # correction falls from ~1e-6 to ~1e-16; each GPU step lands within the
    # one-step bound of the oracle's z + dz*, in both solve modes
    for e in iteration_errors(name, mode):
        say(f"  {name} {MODES[mode]} it {e['iteration']}: |z - z*| = {e['err']:.3e}  bound {e['tol']:.3e}  "
            f"|dz*| = {e['dz_inf']:.3e}  refinements {e['info']['refine_steps']}")
        assert not e["info"]["singular"] and e["info"]["iterations"] == 1
        assert e["err"] <= e["tol"], e
        rho = e["rho_oracle"]
        L = newton_fixture(name)["L"]
        assert abs(e["info"]["residual_first"] - rho) <= 1e-6 * rho + 64 * 128 * 2.0 ** (-53 * L)
        if mode == 1:
            assert 1 <= e["info"]["refine_steps"] <= (3 if L == 2 else 6)


@pytest.mark.parametrize("mode", [0, 1])
def test_track_n128_endpoint_digits(mode):
    # the n = 128 workload tracked from its stored start root to t = 1 with
    # the full double-double solve and with FP64 LU + double-double refinement
    z, st, zss = track_config("n128_dd", mode=mode)
    q_digits = correct_digits(z, zss)
    say(f"  n128 {MODES[mode]}: {q_digits} correct digits, {st['corrections']} corrections, "
        f"{st['newton_iterations']} Newton iterations, {st['seconds']:.2f} s")
    assert not st["fail"] and st["t_final"] == 1.0
    assert q_digits >= 28
