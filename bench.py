"""Benchmark: complex double-double Newton steps per second at n = 64.

Workload: the n = 64 system (64 monomials per polynomial, exponents uniform
in {0..4}, unit-circle coefficients, seed 2) stored in double double, the
total-degree homotopy at t = 1/2, starting at the point of the tracked path
at t = 1/2 (stored fixture).  One step = one Newton iteration of Algorithm
4.1 = evaluation of h and its full Jacobian + Gaussian elimination with
partial pivoting + back substitution + update, with the convergence exit
disabled (eps = 0) so that every step does the full work.  Inputs are
resident in HBM before the timed region; the timed region is K iterations
enqueued back to back on one stream, bracketed by device synchronisation.

Prints one JSON line (see the keys below).  ``--gpus N`` with N > 1 exits:
this build runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "complex-DD Newton steps/s at n=64; full-path time at 28 correct digits"
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector
HBM_PEAK_GBS = 8000.0

# algorithmic flops per complex operation in double double, counted from the
# textbook double-double formulas: complex multiply 80, add 40, fma 120
CMUL, CADD, CFMA = 80, 40, 120
# quad double: FP64 operations (FMA = 2) of this library's quad-double routines:
# real add 70 (level-by-level sums, renormalisation), real multiply 129, so
# complex multiply 4*129 + 2*70 = 656, add 140, fma 796
QD_CMUL, QD_CADD, QD_CFMA = 656, 140, 796
FLOPS = {2: (CMUL, CADD, CFMA), 4: (QD_CMUL, QD_CADD, QD_CFMA), 1: (6, 2, 8)}


def ge_cfma(n: int) -> int:
    """Complex fused multiply-adds of elimination on [A b]: sum_{r=1}^{n-1} r (r+1)."""
    return sum(r * (r + 1) for r in range(1, n))


def bs_cfma(n: int) -> int:
    return n * (n - 1) // 2


def eval_ops(exps, offsets):
    """(cmults, cadds) of one evaluation: per monomial with k active variables
    and k2 of them with exponent >= 2: 4k + k2 - 5 products and k + 1 sums."""
    import numpy as np

    e = np.asarray(exps)
    k = (e > 0).sum(axis=1)
    k2 = (e > 1).sum(axis=1)
    cm = np.where(k >= 2, 4 * k + k2 - 5, np.where(k == 1, k2 + 1, 0)).sum()
    ca = (k + 1).sum()
    return int(cm), int(ca)


def path_point(fix, L):
    import numpy as np

    x = np.zeros((len(fix["x_half_f64"]), 2, L))
    for v, (re, im) in enumerate(fix["x_half_f64"]):
        x[v, 0, 0] = re
        x[v, 1, 0] = im
    return x


def _oracle_rows(args):
    """Worker of the multi-process oracle leg: h, J and scales of a block of
    polynomial rows (a fresh interpreter; imports only the oracle)."""
    import numpy as np

    from oracle.evaluate import eval_homotopy

    exps, coefs, offsets, gamma, t, x, rows = args
    r = eval_homotopy(np.asarray(exps), np.asarray(coefs), np.asarray(offsets), np.asarray(gamma), t,
                      np.asarray(x), rows=rows, form="quotient")
    return r.y, r.J


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sysm, x, t, budget_s: float = 20.0, max_workers: int = 16):
    """Time the oracle's Newton step (plain mpmath evaluation + lu_solve) on
    this host: single process, then with the evaluation's polynomial rows
    spread over a pool of worker processes (at most 16, the host share of one
    GPU; the library linear solve stays in one process).  Each leg runs as
    many steps as fit in about half the budget (at least one)."""
    import multiprocessing as mp

    import mpmath

    from oracle.newton import newton_step, solve

    t0 = time.perf_counter()
    steps = 0
    while True:
        newton_step(sysm.exps, sysm.coefs, sysm.poly_offsets, sysm.gamma, t, x, form="quotient")
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s * 0.5 or steps >= 50:
            break
    single = steps / el
    ncpu = os.cpu_count() or 1
    workers = max(1, min(ncpu, max_workers))
    n = sysm.n
    blocks = [list(range(i, n, workers)) for i in range(workers)]
    args = [(sysm.exps, sysm.coefs, sysm.poly_offsets, sysm.gamma, t, x, rows) for rows in blocks]
    ctx = mp.get_context("spawn")  # fresh interpreters: nothing of the GPU runtime is inherited
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_rows, args[:1])  # start-up and imports outside the timed region
        t0 = time.perf_counter()
        psteps = 0
        while True:
            parts = pool.map(_oracle_rows, args)
            J = [None] * n
            y = [None] * n
            for rows, (ys, Js) in zip(blocks, parts):
                for k, i in enumerate(rows):
                    y[i], J[i] = ys[k], Js[k]
            with mpmath.workprec(488):
                solve(J, [-v for v in y], 488)
            psteps += 1
            el = time.perf_counter() - t0
            if el > budget_s * 0.5 or psteps >= 50:
                break
    return {
        "value": psteps / el,
        "unit": "Newton steps/s",
        "cores": workers,
        "kind": "oracle",
        "sample": f"{psteps} oracle Newton step(s) of the same n=64 double-double workload at t=0.5 (mpmath at 488 "
                  f"bits: plain evaluation with its {n} polynomial rows spread over {workers} worker processes, "
                  f"then lu_solve in one process), {el:.1f} s; single process: {steps} step(s), "
                  f"{single:.3f} steps/s",
        "single_process_value": single,
        "host_cpu_count": ncpu,
        "host_cpu_model": cpu_model(),
    }


def track_case(q, name, L, mode=0):
    """Full path of a stored workload: seconds and correct digits vs the stored z**."""
    import mpmath
    import numpy as np

    from synth.systems import CONFIGS, config_system, start_root

    with open(os.path.join(ROOT, "tests", "golden", f"path_{name}.json")) as fh:
        fix = json.load(fh)
    s = config_system(CONFIGS[name])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x0 = start_root(np.array(fix["degrees"]), np.array(fix["start_k"]), L)
    z, st, _ = q.track_path(H, x0, L, q.default_track_params(mode=mode))
    with mpmath.workprec(800):
        def val(limbs):
            return mpmath.mpc(mpmath.fsum(mpmath.mpf(float(a)) for a in limbs[0]),
                              mpmath.fsum(mpmath.mpf(float(a)) for a in limbs[1]))

        err = max(abs(val(z[v]) - val(np.array(fix["zss_limbs"][v]))) for v in range(s.n))
        nrm = max(mpmath.mpf(1), max(abs(val(np.array(w))) for w in fix["zss_limbs"]))
        digits = 99 if err == 0 else int(mpmath.floor(-mpmath.log10(err / nrm)))
    return {"workload": name, "solve": "full" if mode == 0 else "mixed",
            "seconds": round(st["seconds"], 4), "correct_digits": digits,
            "succ_corrections": st["succ_corrections"], "corrections": st["corrections"],
            "newton_iterations": st["newton_iterations"], "avg_step": st["avg_step"], "min_step": st["min_step"],
            "fail": st["fail"]}


def limbs_value(limbs):
    """Exact value of [2][L] limbs as an mpc (at the caller's working precision)."""
    import mpmath

    return mpmath.mpc(mpmath.fsum(mpmath.mpf(float(a)) for a in limbs[0]),
                      mpmath.fsum(mpmath.mpf(float(a)) for a in limbs[1]))


def newton_vs_oracle(q, name, mode):
    """One GPU Newton iteration from each point of the stored oracle Newton
    sequence (tests/golden/newton_<name>.json: three iterations from 1e-6 off
    the path at t = 1/2): per iteration the oracle's ||dz*||, the GPU's
    ||z_gpu - (z + dz*)||_inf and that error in units of u ||z|| (u = 2^-53L)."""
    import mpmath
    import numpy as np

    from synth.systems import CONFIGS, config_system

    with open(os.path.join(ROOT, "tests", "golden", f"newton_{name}.json")) as fh:
        fix = json.load(fh)
    s = config_system(CONFIGS[name])
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    rows = []
    L = fix["L"]
    for k, row in enumerate(fix["iterations"]):
        x = np.array(row["x_limbs"])
        xg, info = q.newton_step(H, fix["t"], x, L, mode=mode, eps=0.0, max_it=1)
        with mpmath.workprec(700):
            err = max(abs(limbs_value(xg[v]) - limbs_value(x[v]) - limbs_value(np.array(row["dz_limbs"][v])))
                      for v in range(s.n))
        rows.append({"iteration": k, "dz_oracle_inf": row["dz_inf"], "err_inf": float(err),
                     "err_over_u_z": float(err) / (2.0 ** (-53 * L) * row["z_inf"]), "kappa": row["kappa"],
                     "refine_steps": info["refine_steps"]})
    return {"workload": name, "solve": "full" if mode == 0 else "mixed", "iterations": rows}


def common_support_case(q, steps: int = 1000, warmup: int = 20):
    """The shape of the paper's Table 1 (1,000 Newton iterations on a 40 x 40
    system whose polynomials share one support of 200 monomials, average
    degree 40): the seeded stand-in c40_dd, complex double double, t = 1 (the
    target system) from 1e-6 off its planted root, convergence exit off."""
    import numpy as np
    import torch

    from synth.systems import CONFIGS, config_system

    sysm = config_system(CONFIGS["c40_dd"])
    S = q.System.from_synth(sysm)
    H = q.Homotopy(S, sysm.gamma)
    rng = np.random.default_rng(0)
    x0 = sysm.zstar.copy()
    x0[:, :, 0] += 1e-6 * rng.standard_normal((sysm.n, 2))
    x0[:, :, 1] = 0.0
    x = torch.from_numpy(x0[None].copy()).cuda()
    stream = torch.cuda.current_stream()
    q.newton_batch_dev(H, 1.0, x, 1, 2, 0, eps=0.0, max_it=warmup, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q.newton_batch_dev(H, 1.0, x, 1, 2, 0, eps=0.0, max_it=steps, stream=stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    info = q.last_info_batch(H, 2, 1, stream=stream)[0]
    q.binding.set_timing(True)
    q.newton_batch_dev(H, 1.0, x, 1, 2, 0, eps=0.0, max_it=min(steps, 500), stream=stream)
    torch.cuda.synchronize()
    q.binding.set_timing(False)
    eval_ms, solve_ms, launches = q.binding.last_timing(H, 2, stream=stream)
    n, M = sysm.n, int(sysm.poly_offsets[1])
    cm, ca = eval_ops(sysm.exps[:M], np.array([0, M]))  # the support's partials, once
    ev_flops = cm * CMUL + ca * CADD + n * (n + 1) * M * CFMA  # + the coefficient product
    ev_us = eval_ms / launches * 1e3
    return {"workload": "c40_dd: 40 x 40, common support of 200 monomials, exponents in {0,1,2} (average "
                        "degree 40), seed 4; complex double double, t = 1, from 1e-6 off the planted root",
            "newton_iterations": steps, "seconds": el, "steps_per_s": steps / el,
            "residual_last": info["residual_last"], "singular": info["singular"],
            "eval_us": ev_us, "solve_us": solve_ms / launches * 1e3,
            "eval_flops": ev_flops, "eval_frac_fp64_peak": ev_flops / ev_us / 1e6 / FP64_PEAK_TFLOPS,
            "paper_table1_seconds": {"1 thread": 40.778, "8 threads": 6.177,
                                     "context": "two quad-core 3.2 GHz Xeons, the paper's earlier evaluation "
                                                "scheme, precision not stated; their system and generator "
                                                "are not published"}}


def equal_time_units(t_lo_1: float, t_hi_p: float, p: float) -> float:
    """Section 2: the units (cores, here CUs) that bring a run taking t_hi_p on
    p units down to t_lo_1, under optimal speedup: (t_hi_p / t_lo_1) p."""
    return t_hi_p / t_lo_1 * p


def quality_up_linear(p: int, p_star: float, ratio: float) -> float:
    """Section 2's quality-up estimate at p units: y(1) = 1 and y = ratio
    (Q_hi / Q_lo) at p* rounded up to whole units, linear in between (capped
    at ratio beyond)."""
    pc = math.ceil(p_star - 1e-9)
    if pc <= 1:
        return ratio
    return min(ratio, 1 + (ratio - 1) * (p - 1) / (pc - 1))


def cu_study(q, B: int = 256, q_dd: int = 30, q_qd: int = 63):
    """Speedup and quality up with p compute units (Section 2's notions, p =
    CUs instead of cores): Newton iterations of B points of the n=64 path (the
    batched line) in double double and quad double on a stream restricted to
    p CUs (hipExtStreamCreateWithCUMask; the runtime accepts masks of at least
    8 CUs, one per XCD, so p = 8 .. all).  speedup(p) = T(8) / T(p), and the
    single-CU time is estimated as 8 T(8) (optimal speedup below 8 CUs, the
    paper's own assumption for its cores).  Quality up at fixed time T_DD(1):
    p* = the CUs with T_QD(p*) = T_DD(1) (log-interpolated between measured p,
    optimal speedup below 8), and the paper's linear estimate y(p) = 1 +
    (Q_QD/Q_DD - 1)(p - 1)/(ceil(p*) - 1), capped at Q_QD/Q_DD; q_dd, q_qd are
    the correct decimal places of the n=64 path endpoint in each precision."""
    import ctypes as ct
    import math

    import numpy as np
    import torch

    from synth.systems import CONFIGS, config_system

    q.binding.lib()
    hip_path = next((ln.split()[-1] for ln in open("/proc/self/maps") if "libamdhip64" in ln), None)
    if hip_path is None:
        raise RuntimeError("HIP runtime not mapped")
    hip = ct.CDLL(hip_path)  # the runtime copy the library and torch already use
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    ps = [p for p in (8, 16, 32, 64, 128, 256) if p < ncu] + [ncu]
    with open(os.path.join(ROOT, "tests", "golden", "path_n64_dd.json")) as fh:
        fix = json.load(fh)
    times = {}
    for L, K, name in ((2, 2, "n64_dd"), (4, 1, "n64_qd")):
        s_l = config_system(CONFIGS[name])
        H = q.Homotopy(q.System.from_synth(s_l), s_l.gamma)
        p0 = path_point(fix, L)
        x0 = torch.from_numpy(np.stack([p0 * (1.0 + 1e-6 * b) for b in range(B)])).cuda()
        q.newton_batch_dev(H, 0.5, x0.clone(), B, L, 0, eps=0.0, max_it=1)  # workspace, code load
        torch.cuda.synchronize()
        for p in ps:
            mask = (ct.c_uint32 * ((ncu + 31) // 32))()
            for c in range(p):
                mask[c // 32] |= 1 << (c % 32)
            st = ct.c_void_p()
            rc = hip.hipExtStreamCreateWithCUMask(ct.byref(st), len(mask), mask)
            if rc != 0:
                raise RuntimeError(f"hipExtStreamCreateWithCUMask({p} CUs) returned {rc}")
            x = x0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            q.newton_batch_dev(H, 0.5, x, B, L, 0, eps=0.0, max_it=K, stream=st.value)
            rc = hip.hipStreamSynchronize(st)
            times[(L, p)] = (time.perf_counter() - t0) / K
            hip.hipStreamDestroy(st)
            if rc != 0:
                raise RuntimeError(f"hipStreamSynchronize returned {rc}")
    p0 = ps[0]
    rows = [{"cus": p, "dd_s_per_iteration": times[(2, p)], "qd_s_per_iteration": times[(4, p)],
             "dd_speedup_vs_8": times[(2, p0)] / times[(2, p)], "qd_speedup_vs_8": times[(4, p0)] / times[(4, p)]}
            for p in ps]
    t_dd1 = p0 * times[(2, p0)]  # single-CU estimate
    if times[(4, p0)] <= t_dd1:
        pstar = equal_time_units(t_dd1, times[(4, p0)], p0)
    else:
        pstar = None
        for a, b in zip(ps, ps[1:]):
            if times[(4, a)] > t_dd1 >= times[(4, b)]:
                la, lb = math.log(times[(4, a)]), math.log(times[(4, b)])
                f = (la - math.log(t_dd1)) / (la - lb)
                pstar = math.exp(math.log(a) + f * (math.log(b) - math.log(a)))
    cap = q_qd / q_dd

    def y(p):
        return None if pstar is None else quality_up_linear(p, pstar, cap)

    return {"workload": f"n=64 (seed 2), {B} points of the path at t = 0.5 per launch, full elimination; "
                        "seconds per Newton iteration on a stream masked to p CUs",
            "rows": rows, "dd_single_cu_estimate_s": t_dd1, "Q_dd": q_dd, "Q_qd": q_qd,
            "p_star_cus": pstar, "quality_up_8_cus": y(8), "quality_up_all_cus": y(ncu)}


def track_batch_case(q, name, L, B, single):
    """B copies of the stored path tracked together (one launch per kernel per
    round): paths per second against the single-path run `single`."""
    import numpy as np

    from synth.systems import CONFIGS, config_system, start_root

    with open(os.path.join(ROOT, "tests", "golden", f"path_{name}.json")) as fh:
        fix = json.load(fh)
    s = config_system(CONFIGS[name])
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    x0 = start_root(np.array(fix["degrees"]), np.array(fix["start_k"]), L)
    z, st = q.track_paths(H, np.stack([x0] * B), L)
    same = all(np.array_equal(z[b], z[0]) for b in range(B))
    secs = st[0]["seconds"]
    return {"workload": name, "B": B, "seconds": round(secs, 4), "paths_per_s": B / secs,
            "single_path_seconds": single["seconds"], "speedup_per_path": single["seconds"] * B / secs,
            "fails": sum(x["fail"] for x in st), "all_endpoints_equal": same,
            "corrections": st[0]["corrections"], "newton_iterations": st[0]["newton_iterations"]}


def quality_report(dd, qd, cpu):
    """Quality up of Section 2 on the n = 64 workload: the same path tracked in
    double double and in quad double on the GPU.  Q = correct decimal places
    against the exact root; the fixed-time reference is the oracle's double
    double Newton step on one host core, times the Newton iterations of the
    GPU double-double path (an extrapolation: the oracle does not track the
    whole path)."""
    rep = {
        "workload": "n=64, 64 monomials per polynomial, exponents in {0..4}, seed 2; the same draws rounded to "
                    "2 limbs (double double) and 4 limbs (quad double)",
        "Q_dd": dd["correct_digits"], "T_dd_s": dd["seconds"],
        "Q_qd": qd["correct_digits"], "T_qd_s": qd["seconds"],
        "quality_up": qd["correct_digits"] / dd["correct_digits"],
        "time_ratio_qd_over_dd": qd["seconds"] / dd["seconds"],
    }
    if cpu:
        t1 = dd["newton_iterations"] / cpu["value"]
        rep["oracle_dd_path_s_extrapolated"] = t1
        rep["qd_gpu_faster_than_oracle_dd"] = qd["seconds"] < t1
    return rep


def measured_traffic(kernel_file: str):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary of
    the dominant kernel, or None when the kernel's sources changed since the
    counters were taken (the record stores a hash of those sources)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", kernel_file)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    return rec["bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def newton_rate(q, name: str, L: int, mode: int, steps: int, warmup: int, t: float = 0.5, B: int = 1):
    """Newton steps/s of one workload at fixed t with the convergence exit off;
    returns (steps/s summed over the B points, ms per iteration, eval us/launch,
    solve us/launch, system, info of point 0).  B > 1: B points of the path
    (the stored point scaled by 1 + 1e-6 b) in one launch per kernel."""
    import numpy as np
    import torch

    from synth.systems import CONFIGS, config_system

    sysm = config_system(CONFIGS[name])
    with open(os.path.join(ROOT, "tests", "golden", f"path_{name}.json")) as fh:
        fix = json.load(fh)
    S = q.System.from_synth(sysm)
    H = q.Homotopy(S, sysm.gamma)
    stream = torch.cuda.current_stream()
    p0 = path_point(fix, L)
    x = torch.from_numpy(np.stack([p0 * (1.0 + 1e-6 * b) for b in range(B)])).cuda()
    q.newton_batch_dev(H, t, x, B, L, mode, eps=0.0, max_it=warmup, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q.newton_batch_dev(H, t, x, B, L, mode, eps=0.0, max_it=steps, stream=stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    infos = q.last_info_batch(H, L, B, stream=stream)
    if any(i["iterations"] != steps for i in infos):
        raise RuntimeError(f"{name}: not every point ran {steps} Newton iterations: {infos[:2]}")
    # per-kernel durations from HIP events between the kernels, in a separate
    # run (the events add gaps between launches, so the timed run has none)
    q.binding.set_timing(True)
    q.newton_batch_dev(H, t, x, B, L, mode, eps=0.0, max_it=min(steps, 500), stream=stream)
    torch.cuda.synchronize()
    q.binding.set_timing(False)
    eval_ms, solve_ms, launches = q.binding.last_timing(H, L, stream=stream)
    return B * steps / el, el / steps * 1e3, eval_ms / launches * 1e3, solve_ms / launches * 1e3, sysm, infos[0]


def eval_flops(sysm, L: int) -> int:
    cm, ca = eval_ops(sysm.exps, sysm.poly_offsets)
    fm, fa, _ = FLOPS[L]
    return cm * fm + ca * fa


def rate_entry(name, L, B, mode, rate, ms, ev_us, ge_us, sysm):
    """Per-kernel algorithmic rates of one Newton timing run (B points per launch)."""
    n = sysm.n
    evf = B * eval_flops(sysm, L)
    gef = B * (ge_cfma(n) + bs_cfma(n)) * FLOPS[L][2]
    return {"workload": name, "B": B, "solve": "full" if mode == 0 else "mixed", "steps_per_s": rate,
            "ms_per_iteration": ms, "eval_us": ev_us, "solve_us": ge_us,
            "eval_tflops": evf / ev_us / 1e6, "eval_frac_fp64_peak": evf / ev_us / 1e6 / FP64_PEAK_TFLOPS,
            "solve_tflops": gef / ge_us / 1e6 if mode == 0 else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--mode", choices=["full", "mixed"], default="full")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paths", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the mixed-precision / n=128 comparison lines")
    ap.add_argument("--batch", type=int, default=256, help="points per launch of the batched comparison line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 256 MiB device copy (for HBM counter calibration)")
    ap.add_argument("--cu-study", action="store_true",
                    help="run only the speedup / quality-up study over compute units and print it")
    ap.add_argument("--profile-common", action="store_true",
                    help="run only the common-support line (--steps Newton iterations) and print it")
    ap.add_argument("--profile-line", choices=["n64_dd", "n128_dd", "n64_qd"],
                    help="run only this one-path Newton line (--mode, --steps iterations) and print its rates "
                         "(for profiling the mixed-precision and quad-double kernels)")
    ap.add_argument("--batch-workload", choices=["n64_dd", "n64_qd"], default="n64_dd",
                    help="workload of --profile-batch")
    ap.add_argument("--profile-batch", action="store_true",
                    help="run only the batched Newton line (--batch-workload, --batch points per launch, "
                         "--steps iterations) and print its rates (for profiling the batched evaluation)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    if args.copy_calibration:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8, "launches": 5}))
        return

    import paper_1109_0545_amd as q
    from synth.systems import CONFIGS

    L = 2
    t = 0.5
    mode = q.SOLVE_FULL if args.mode == "full" else q.SOLVE_MIXED_IR
    if args.profile_line:
        lim = 4 if args.profile_line.endswith("qd") else 2
        r, m_, e_, g_, sy, inf = newton_rate(q, args.profile_line, lim, mode, args.steps, args.warmup, t)
        ent = rate_entry(args.profile_line, lim, 1, mode, r, m_, e_, g_, sy)
        ent["refine_steps"] = inf["refine_steps"]
        print(json.dumps(ent))
        return
    if args.cu_study:
        print(json.dumps(cu_study(q, B=args.batch)))
        return
    if args.profile_common:
        print(json.dumps(common_support_case(q, steps=args.steps)))
        return
    if args.profile_batch:
        wl = args.batch_workload
        lim = 4 if wl.endswith("qd") else 2
        r = newton_rate(q, wl, lim, mode, args.steps, args.warmup, t, B=args.batch)
        print(json.dumps(rate_entry(wl, lim, args.batch, mode, *r[:5])))
        return
    rate, ms, ev_us, ge_us, sysm, info = newton_rate(q, "n64_dd", L, mode, args.steps, args.warmup, t)

    n = sysm.n
    cm, ca = eval_ops(sysm.exps, sysm.poly_offsets)
    ge_flops = (ge_cfma(n) + bs_cfma(n)) * CFMA
    ev_flops = cm * CMUL + ca * CADD
    # the elimination of one n = 64 double-double point runs in blocks of 16
    # columns, the last one taking b and up to 24 columns, one workgroup (one
    # CU) per block (k_ge_mcb); the mixed solve is one workgroup
    rest = n + 1 - 8
    cus = (1 if rest <= 16 else -(-rest // 16)) if mode == 0 else 1
    if ge_us >= ev_us:
        dom = f"elimination (k_ge_mcb, {cus} workgroups)" if mode == 0 else "mixed solve (k_mixed)"
        dom_flops, dom_us = ge_flops, ge_us
    else:
        dom, dom_flops, dom_us = "evaluation (k_eval)", ev_flops, ev_us
    achieved = dom_flops / (dom_us * 1e-6) / 1e12
    cfg = CONFIGS["n64_dd"]
    out = {
        "metric": METRIC,
        "value": rate,
        "unit": "Newton steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "dd",
        "data": "synthetic",
        "config": {
            "workload": "n=64 sparse system, 64 monomials per polynomial, exponents uniform in {0..4}, "
                        "unit-circle coefficients, seed 2, complex double double, total-degree homotopy at t=0.5, "
                        f"one path, {'full double-double elimination' if mode == 0 else 'FP64 LU + DD refinement'}",
            "n": n, "monomials_per_polynomial": cfg.m, "max_exponent": cfg.E, "limbs": L, "solve": args.mode,
        },
        "roofline": {
            "bound": "alu",
            "kernel": dom,
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": measured_traffic("traffic_k_ge_n64_dd.json") if dom.startswith("elimination") else None,
            "algorithmic_flops_per_launch": dom_flops,
            "avg_launch_us": dom_us,
            # one path's solve occupies `cus` of the 256 CUs (one workgroup
            # each): its rate against those CUs' share of the FP64 peak
            "cus_used": cus,
            "frac_of_used_cus": achieved / (FP64_PEAK_TFLOPS * cus / 256),
        },
        "kernels": {"eval_us": ev_us, "solve_us": ge_us, "eval_flops": ev_flops, "solve_flops": ge_flops},
    }
    if not args.no_extra:
        extra = [rate_entry("n64_dd", L, 1, mode, rate, ms, ev_us, ge_us, sysm)]
        for name, lim, md, k, B in (("n64_dd", 2, 1 - mode, max(args.steps // 2, 10), 1),
                                    ("n128_dd", 2, 0, 200, 1), ("n128_dd", 2, 1, 200, 1),
                                    ("n64_qd", 4, 0, 200, 1), ("n64_qd", 4, 1, 200, 1),
                                    ("n64_dd", 2, 0, 100, args.batch)):
            r, m_, e_, g_, sy, inf = newton_rate(q, name, lim, md, k, 10, t, B=B)
            ent = rate_entry(name, lim, B, md, r, m_, e_, g_, sy)
            ent["refine_steps"] = inf["refine_steps"]
            extra.append(ent)
        # B points per launch: independent paths at one t (the rate summed over points)
        out["solve_modes"] = extra
        out["common_support"] = common_support_case(q)
    paths = {}
    if not args.no_paths:
        try:
            for name, lim in (("n8_dd", 2), ("n32_dd", 2), ("n64_dd", 2), ("n64_qd", 4)):
                paths[name] = track_case(q, name, lim)
            out["paths"] = list(paths.values())
            out["paths_batch"] = [track_batch_case(q, "n64_dd", 2, args.batch, paths["n64_dd"])]
        except Exception as e:  # report, never hide, a failing path
            out["paths"] = [{"error": str(e)}]
    if not args.no_paths and not args.no_extra:
        # mixed precision (FP64 factorization + refinement in double or quad double)
        # beside the full elimination: error per Newton iteration against the oracle
        # and the n = 128 double-double and n = 64 quad-double path endpoints in both modes
        try:
            out["mixed_vs_full"] = {
                "per_iteration": [newton_vs_oracle(q, nm, md) for nm in ("n64_dd", "n128_dd", "n64_qd")
                                  for md in (0, 1)],
                "paths": [track_case(q, "n128_dd", 2, md) for md in (0, 1)] + [track_case(q, "n64_qd", 4, 1)],
            }
        except Exception as e:  # report, never hide
            out["mixed_vs_full"] = {"error": str(e)}
    if not args.no_cpu_baseline:
        from synth.systems import config_system

        with open(os.path.join(ROOT, "tests", "golden", "path_n64_dd.json")) as fh:
            fix = json.load(fh)
        out["cpu_baseline"] = cpu_baseline(config_system(cfg), path_point(fix, L), t)
    if "n64_dd" in paths and "n64_qd" in paths:
        out["quality_up"] = quality_report(paths["n64_dd"], paths["n64_qd"], out.get("cpu_baseline"))
    if not args.no_extra:
        qu = out.get("quality_up") or {}
        try:
            out["cu_study"] = cu_study(q, B=args.batch, q_dd=qu.get("Q_dd", 30), q_qd=qu.get("Q_qd", 63))
        except Exception as e:  # report, never hide
            out["cu_study"] = {"error": str(e)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
