"""Learned step control on held-out systems: what the trained network gains
over the plain step-size control, with the Newton test as judge."""

import os

import numpy as np
import pytest

from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_learned_control_beats_plain_on_held_out_systems():
    # all 50 held-out n=32 systems: fewer corrector stages than both plain
    # controllers, and less wall time per path than the stronger one (the
    # network runs on the device inside each corrector stage, so a stage
    # costs about the same with and without it)
    from paper_1109_0545_amd import policy

    say("learned vs plain on the 50 held-out n=32 systems")
    r = policy.evaluate(os.path.join(ROOT, "tests", "golden", "family_heldout.json"),
                        os.path.join(ROOT, "paper_1109_0545_amd", "policy_n32.npz"))
    s = r["summary"]
    assert s["systems"] == 50
    for base in ("plain_quadratic", "plain"):
        wins = sum(1 for row in r["rows"] if row["learned"]["corrections"] < row[base]["corrections"])
        assert s[f"{base}_fails"] == 0 and s[f"{base}_min_digits"] >= 28
        assert s["learned_mean_corrections"] < s[f"{base}_mean_corrections"]
        assert wins >= 40, (base, wins)
    assert s["learned_fails"] == 0 and s["learned_min_digits"] >= 28
    say(f"  mean s/path: plain {s['plain_mean_seconds']:.4f}, quadratic {s['plain_quadratic_mean_seconds']:.4f}, "
        f"learned {s['learned_mean_seconds']:.4f}; corrections {s['plain_mean_corrections']:.1f} / "
        f"{s['plain_quadratic_mean_corrections']:.1f} / {s['learned_mean_corrections']:.1f}")
    assert s["learned_mean_seconds"] < s["plain_quadratic_mean_seconds"]


def test_learned_control_falls_back_when_the_network_is_wrong():
    # an over-confident network (every multiplier "accepted") proposes the
    # largest step each time; the Newton test rejects what does not converge,
    # the plain rule takes over until the next success, and the path still
    # ends at the same point
    import paper_1109_0545_amd as q
    from paper_1109_0545_amd import policy
    from synth.policy import init_params

    fam = os.path.join(ROOT, "tests", "golden", "family_heldout.json")
    seed, S, H, x0, fix = next(policy.family_jobs(fam))
    params = np.zeros_like(init_params(1, policy.WIDTHS))
    # output biases: logits +20 (always accepted), quadratic weight 1
    params[-policy.WIDTHS[-1]:] = [20, 20, 20, 20, 20, 1.0]
    pol = q.Policy(policy.WIDTHS, params, np.zeros(16), np.ones(16))
    say("learned fallback")
    p = q.default_track_params(predictor=q.PRED_LEARNED, policy=pol)
    z, st, _ = q.track_path(H, x0, 2, p)
    assert st["fail"] == 0 and st["policy_used"] > 0 and st["policy_rejected"] > 0
    assert policy.correct_digits(z, fix["zss_limbs"]) >= 28
