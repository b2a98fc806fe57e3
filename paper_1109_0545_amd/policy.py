"""Learned step control: data collection, training and evaluation driver.

Everything numeric runs in the library: probe tracking (``qdp_track_path``
with ``probe = 1``), training (``qdp_policy_train_step``: the FP32 forward,
backward and Adam kernels) and inference (BF16 kernel inside the tracker).
This module only assembles batches and reports.

Data: at every accepted state of a plain path (quadratic predictor), the
tracker tries the step multipliers 2^-1, 2^0, 2^1, 2^2, 2^3 of the last
accepted step and records which ones the Newton test accepts, plus the
least-squares weight of the quadratic predictor against the secant for the
2^0 step (``qdp_step_record`` of kind 1).  Targets: the five accept flags
(binary cross-entropy) and that weight (squared error, masked when
unavailable or outside [-1, 3]).

Command line (n = 32 systems described by a family file of seeds and start
roots):
    python -m paper_1109_0545_amd.policy collect  --family F --out data.npz
    python -m paper_1109_0545_amd.policy train    --data data.npz --out policy.npz
    python -m paper_1109_0545_amd.policy evaluate --family F --policy policy.npz
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Dict, List

import numpy as np

from . import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WIDTHS = [B.N_FEATURES, 128, 128, 128, B.N_MULT + 1]


def family_jobs(path: str, L: int = 2):
    """(seed, System, Homotopy, start point, fixture row) for every system of a family file."""
    sys.path.insert(0, ROOT)
    from synth.systems import make_system, start_root

    rows = json.load(open(path))
    for r in rows:
        s = make_system(32, r["m"], r["E"], L, r["seed"])
        S = B.System.from_synth(s)
        H = B.Homotopy(S, s.gamma)
        x0 = start_root(np.array(r["degrees"]), np.array(r["start_k"]), L)
        yield r["seed"], S, H, x0, r


def records_to_dataset(recs: List[dict]):
    X, Y, M = [], [], []
    for r in recs:
        if r["kind"] != 1:
            continue
        y = np.zeros(B.N_MULT + 1, dtype=np.float32)
        m = np.ones(B.N_MULT + 1, dtype=np.float32)
        for k in range(B.N_MULT):
            y[k] = 1.0 if (r["probe_ok"] >> k) & 1 else 0.0
        bl = r["blend_label"]
        if math.isfinite(bl) and -1.0 <= bl <= 3.0:
            y[-1] = bl
        else:
            m[-1] = 0.0
        X.append(np.asarray(r["features"], dtype=np.float32))
        Y.append(y)
        M.append(m)
    return np.array(X, dtype=np.float32), np.array(Y, dtype=np.float32), np.array(M, dtype=np.float32)


def collect(family: str, out: str, log_cap: int = 40000) -> Dict:
    Xs, Ys, Ms = [], [], []
    t0 = time.time()
    params = B.default_track_params(probe=1, predictor=B.PRED_QUADRATIC)
    for seed, S, H, x0, _ in family_jobs(family):
        _, st, recs = B.track_path(H, x0, 2, params, log_cap=log_cap)
        X, Y, M = records_to_dataset(recs)
        Xs.append(X)
        Ys.append(Y)
        Ms.append(M)
        print(f"collect seed {seed}: {len(X)} states, fail {st['fail']}", flush=True)
    X, Y, M = np.concatenate(Xs), np.concatenate(Ys), np.concatenate(Ms)
    np.savez(out, X=X, Y=Y, M=M)
    return {"states": int(len(X)), "samples": int(len(X) * B.N_MULT), "seconds": time.time() - t0}


def train(data: str, out: str, epochs: int = 60, batch: int = 1024, lr: float = 2e-3, seed: int = 7) -> Dict:
    import torch

    sys.path.insert(0, ROOT)
    from synth.policy import init_params

    d = np.load(data)
    X, Y, M = d["X"], d["Y"], d["M"]
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std[std < 1e-6] = 1.0
    pol = B.Policy(WIDTHS, init_params(seed, WIDTHS), mean, std)
    rng = np.random.Generator(np.random.PCG64(seed))
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.from_numpy(Y).cuda()
    Md = torch.from_numpy(M).cuda()
    n = len(X)
    hist = []
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        losses = []
        for i in range(0, n - batch + 1, batch):
            idx = perm[i: i + batch]
            xb, yb, mb = Xd[idx].contiguous(), Yd[idx].contiguous(), Md[idx].contiguous()
            want = i + 2 * batch > n
            lval = pol.train_step(xb, yb, mb, lr=lr * (0.5 ** (ep // 20)), want_loss=want)
            if want:
                losses.append(lval)
        hist.append(float(np.mean(losses)) if losses else float("nan"))
    torch.cuda.synchronize()
    params = pol.params()
    np.savez(out, widths=np.array(WIDTHS, dtype=np.int32), params=params, mean=mean, std=std,
             loss_history=np.array(hist))
    return {"samples": int(n), "epochs": epochs, "final_loss": hist[-1], "seconds": time.time() - t0}


def load(path: str) -> B.Policy:
    d = np.load(path)
    return B.Policy(d["widths"], d["params"], d["mean"], d["std"])


def correct_digits(z: np.ndarray, zss_limbs) -> int:
    """floor(-log10(max |z - z**| / max(1, ||z**||))) from stored limbs (mpmath at 800 bits)."""
    import mpmath

    with mpmath.workprec(800):
        def val(limbs):
            return mpmath.mpc(mpmath.fsum(mpmath.mpf(float(a)) for a in limbs[0]),
                              mpmath.fsum(mpmath.mpf(float(a)) for a in limbs[1]))

        err = max(abs(val(z[v]) - val(np.array(zss_limbs[v]))) for v in range(len(z)))
        nrm = max(mpmath.mpf(1), max(abs(val(np.array(w))) for w in zss_limbs))
        return 99 if err == 0 else int(mpmath.floor(-mpmath.log10(err / nrm)))


def evaluate(family: str, policy_path: str, limit: int = 0, rule: int = 0, threshold: float = 0.3,
             cap: float = 0.32) -> Dict:
    pol = load(policy_path)
    plain = B.default_track_params()
    plain_q = B.default_track_params(predictor=B.PRED_QUADRATIC)
    learned = B.default_track_params(predictor=B.PRED_LEARNED, policy=pol, policy_rule=rule,
                                     accept_threshold=threshold, lambda_max_learned=cap)
    rows = []
    for i, (seed, S, H, x0, fix) in enumerate(family_jobs(family)):
        if limit and i >= limit:
            break
        row = {"seed": seed}
        for key, prm in (("plain", plain), ("plain_quadratic", plain_q)):
            zp, sp, _ = B.track_path(H, x0, 2, prm)
            row[key] = {"corrections": sp["corrections"], "succ": sp["succ_corrections"], "seconds": sp["seconds"],
                        "newton_iterations": sp["newton_iterations"], "fail": sp["fail"],
                        "digits": correct_digits(zp, fix["zss_limbs"]) if not sp["fail"] else -1}
        zl, sl, _ = B.track_path(H, x0, 2, learned)
        row.update({
            "learned": {"corrections": sl["corrections"], "succ": sl["succ_corrections"], "seconds": sl["seconds"],
                        "newton_iterations": sl["newton_iterations"], "fail": sl["fail"],
                        "policy_used": sl["policy_used"], "policy_rejected": sl["policy_rejected"],
                        "digits": correct_digits(zl, fix["zss_limbs"]) if not sl["fail"] else -1},
        })
        rows.append(row)
    def agg(key, f):
        return float(np.mean([r[key][f] for r in rows]))

    summary = {"systems": len(rows)}
    for key in ("plain", "plain_quadratic", "learned"):
        summary.update({
            f"{key}_mean_corrections": agg(key, "corrections"),
            f"{key}_median_corrections": float(np.median([r[key]["corrections"] for r in rows])),
            f"{key}_mean_newton_iterations": agg(key, "newton_iterations"),
            f"{key}_mean_seconds": agg(key, "seconds"),
            f"{key}_fails": int(sum(r[key]["fail"] for r in rows)),
            f"{key}_min_digits": int(min(r[key]["digits"] for r in rows)),
        })
    summary.update({
        "learned_rejected_fraction": float(sum(r["learned"]["policy_rejected"] for r in rows) /
                                           max(1, sum(r["learned"]["policy_used"] for r in rows))),
    })
    summary.update({"rule": rule, "threshold": threshold, "cap": cap})
    return {"summary": summary, "rows": rows}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["collect", "train", "evaluate"])
    ap.add_argument("--family")
    ap.add_argument("--data")
    ap.add_argument("--out")
    ap.add_argument("--policy")
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--limit", type=int, default=0)
    ap.add_argument("--rule", type=int, default=0)
    ap.add_argument("--threshold", type=float, default=0.3)
    ap.add_argument("--cap", type=float, default=0.32)
    a = ap.parse_args(argv)
    if a.cmd == "collect":
        print(json.dumps(collect(a.family, a.out)))
    elif a.cmd == "train":
        print(json.dumps(train(a.data, a.out, epochs=a.epochs)))
    else:
        r = evaluate(a.family, a.policy, a.limit, a.rule, a.threshold, a.cap)
        if a.out:
            json.dump(r, open(a.out, "w"), indent=1)
        print(json.dumps(r["summary"]))


if __name__ == "__main__":
    main()
