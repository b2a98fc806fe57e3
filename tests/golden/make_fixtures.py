"""Write the path fixtures used by the tracker tests and the benchmark.

For each workload shape: draw the seeded system (``synth``), refine its
planted root to the exact regular root z** in high precision
(``oracle.track.refine_root``), track backward from z** to t = 0 in FP64 to
name the start root x_v = exp(2 pi i k_v / d_v) whose path ends at z**, and
confirm the pair by tracking forward.  Also stores the FP64 point of that
path at t = 1/2 (a starting point for fixed-t Newton timing).

Newton sequences (``newton <name>...``): from the path point at t = 1/2,
moved off the path by a seeded relative 1e-6, three oracle Newton iterations
(``oracle.newton.newton_step``), each from the previous oracle iterate rounded
to the workload's limbs; per iteration the input bits, the oracle's correction
dz* (8 limbs), its residual and the terms of the one-step tolerance
(``oracle.newton``: kappa, ||J^-1||, the largest scale).

Calls only ``oracle/`` and ``synth/``.  Usage:

    python tests/golden/make_fixtures.py n8_dd n32_dd n64_qd n64_dd n128_dd
    python tests/golden/make_fixtures.py newton n64_dd n128_dd
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import mpmath  # noqa: E402

from oracle.evaluate import eval_homotopy  # noqa: E402
from oracle.newton import cond_inf, inv_norm_inf, newton_step  # noqa: E402
from oracle.numbers import prec_bits, to_limbs_complex  # noqa: E402
from oracle.track import F64Homotopy, refine_root, start_root_index, track_f64  # noqa: E402
from synth.systems import CONFIGS, config_system, make_system  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ZSS_LIMBS = 8  # 424 bits: far below the quad-double unit roundoff


def fixture_for(sysm, name: str, meta: dict, refine: bool = True) -> dict:
    """``refine=False`` skips the high-precision z** (training systems only
    need the start root); the FP64 target root then comes from an FP64 Newton
    polish of the planted point."""
    t0 = time.time()
    H = F64Homotopy(sysm)
    if refine:
        rr = refine_root(sysm, sysm.zstar)
        zss64 = np.array([complex(v) for v in rr.z])
    else:
        rr = None
        zss64 = sysm.zstar[:, 0, 0] + 1j * sysm.zstar[:, 1, 0]
        for _ in range(4):
            h, J, _ = H.eval(zss64, 1.0)
            zss64 = zss64 + np.linalg.solve(J, -h)
    t_ref = time.time() - t0
    k, x0 = start_root_index(H, zss64)
    start = np.exp(2j * np.pi * k / H.deg)
    x_half, _ = track_f64(H, start, 0.0, 0.5)
    x1, nsteps = track_f64(H, start, 0.0, 1.0)
    fwd_err = float(np.max(np.abs(x1 - zss64)))
    if fwd_err > 1e-8:
        raise RuntimeError(f"{name}: forward FP64 track missed z** by {fwd_err}")
    zss = [to_limbs_complex(v, ZSS_LIMBS).tolist() for v in rr.z] if refine else None
    out = dict(meta)
    out.update(
        {
            "name": name,
            "source": "written by tests/golden/make_fixtures.py from oracle.track (refine_root, FP64 tracker)",
            "n": sysm.n,
            "L": sysm.L,
            "degrees": [int(d) for d in H.deg],
            "start_k": [int(v) for v in k],
            "zss_limbs": zss,
            "refine_corrections": rr.corrections if refine else None,
            "fp64_forward_steps": int(nsteps),
            "fp64_forward_err": fwd_err,
            "x_half_f64": [[float(v.real), float(v.imag)] for v in x_half],
            "seconds": time.time() - t0,
            "refine_seconds": t_ref,
        }
    )
    return out


def main(names):
    for name in names:
        cfg = CONFIGS[name]
        s = config_system(cfg)
        meta = {"config": name, "m": cfg.m, "E": cfg.E, "seed": cfg.seed}
        out = fixture_for(s, name, meta)
        path = os.path.join(HERE, f"path_{name}.json")
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        print(name, "k[:4] =", out["start_k"][:4], "seconds", round(out["seconds"], 1), flush=True)


NEWTON_T = 0.5
NEWTON_PERTURB = 1e-6
NEWTON_ITERS = 3


def newton_sequence(name: str) -> dict:
    cfg = CONFIGS[name]
    s = config_system(cfg)
    L = s.L
    with open(os.path.join(HERE, f"path_{name}.json")) as fh:
        fix = json.load(fh)
    base = np.array([complex(a, b) for a, b in fix["x_half_f64"]])
    rng = np.random.Generator(np.random.PCG64(1000 + cfg.seed))
    pert = rng.standard_normal(s.n) + 1j * rng.standard_normal(s.n)
    x = np.stack([to_limbs_complex(mpmath.mpc(v), L) for v in base * (1 + NEWTON_PERTURB * pert)])
    prec = prec_bits(L)
    rows = []
    for k in range(NEWTON_ITERS):
        t0 = time.time()
        st = newton_step(s.exps, s.coefs, s.poly_offsets, s.gamma, NEWTON_T, x, form="quotient")
        hs = eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, NEWTON_T, x, form="quotient")
        with mpmath.workprec(prec):
            row = {
                "x_limbs": x.tolist(),
                "dz_limbs": [to_limbs_complex(d, ZSS_LIMBS).tolist() for d in st.dz],
                "rho": float(st.rho),
                "kappa": cond_inf(st.J, 300),
                "jinv": inv_norm_inf(st.J, 300),
                "h_scale": float(max(hs.S)),
                "dz_inf": max(float(abs(d)) for d in st.dz),
                "z_inf": max(float(abs(z)) for z in st.z),
            }
            x = np.stack([to_limbs_complex(z, L) for z in st.z])
        row["seconds"] = time.time() - t0
        rows.append(row)
        print(name, "iteration", k, "rho", row["rho"], "|dz|", row["dz_inf"], "kappa", row["kappa"],
              round(row["seconds"], 1), flush=True)
    return {
        "name": name,
        "source": "written by tests/golden/make_fixtures.py from oracle.newton (newton_step, cond_inf, inv_norm_inf)",
        "n": s.n, "L": L, "t": NEWTON_T, "perturb": NEWTON_PERTURB, "perturb_seed": 1000 + cfg.seed,
        "form": "quotient", "iterations": rows,
    }


def main_family(prefix: str, n: int, m: int, E: int, L: int, seeds, refine: bool):
    """Fixtures for a family of systems (learned step control): one JSON with all of them."""
    rows = []
    for seed in seeds:
        s = make_system(n, m, E, L, seed)
        try:
            out = fixture_for(s, f"{prefix}_{seed}", {"seed": seed, "m": m, "E": E}, refine=refine)
        except RuntimeError as e:  # keep going; the family records which seeds failed
            print("skip", seed, e, flush=True)
            continue
        out.pop("x_half_f64")
        rows.append(out)
        print(prefix, seed, round(out["seconds"], 1), flush=True)
    with open(os.path.join(HERE, f"family_{prefix}.json"), "w") as fh:
        json.dump(rows, fh)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "newton":
        for nm in sys.argv[2:]:
            out = newton_sequence(nm)
            with open(os.path.join(HERE, f"newton_{nm}.json"), "w") as fh:
                json.dump(out, fh)
    elif len(sys.argv) > 1 and sys.argv[1] == "family":
        # family <prefix> <first_seed> <count> <refine 0|1>: n=32 systems shaped like the n32 workload
        prefix, first, count = sys.argv[2], int(sys.argv[3]), int(sys.argv[4])
        refine = len(sys.argv) > 5 and sys.argv[5] == "1"
        main_family(prefix, 32, 32, 3, 2, range(first, first + count), refine)
    else:
        main(sys.argv[1:] or ["n8_dd", "n32_dd", "n64_qd", "n64_dd", "n128_dd"])
