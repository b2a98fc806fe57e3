"""The bench's quality-up arithmetic (Section 2), pinned to the paper's
worked example: 4.818 s in double double on one core against 8.076 s in quad
double on eight cores gives 13.410 cores for equal time, 14 whole cores, and
a quality up of 1 + 7/13 ~ 1.538 at eight cores (tests/golden/quality_up.json,
which the oracle's quality module is pinned to as well)."""

import json
import os

import bench

HERE = os.path.dirname(os.path.abspath(__file__))


def test_bench_quality_up_matches_the_papers_worked_example():
    with open(os.path.join(HERE, "golden", "quality_up.json")) as fh:
        fix = json.load(fh)
    ps = bench.equal_time_units(fix["t_dd_1core"], fix["t_qd_pcores"], fix["p"])
    assert abs(ps - fix["p_star"]) < 5e-4
    y = bench.quality_up_linear(fix["p"], ps, 2.0)
    assert abs(y - fix["y_num"] / fix["y_den"]) < 1e-12
    assert round(y, 3) == fix["y_rounded"]
    # the estimate's ends: one unit gives 1, ceil(p*) units the full ratio
    assert bench.quality_up_linear(1, ps, 2.0) == 1.0
    assert bench.quality_up_linear(fix["cores"], ps, 2.0) == 2.0
    assert bench.quality_up_linear(fix["cores"] + 10, ps, 2.0) == 2.0
