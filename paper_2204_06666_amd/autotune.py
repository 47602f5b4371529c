"""Exhaustive tuning of the preprocessing parameters of one matrix, and the
sweep over the tuning set that trains the parameter predictor.

For every matrix the grid is partition size x ELL width cap x rows per wave
(6 x 4 x 4 points, FP32 values and x, one right-hand side; the values are in
``predictor``).  The matrix is
partitioned once per partition size; the 16 encodings of that size reuse the
partition (ehyb_preprocess_partitioned).  Each point is timed on the device
as the best of several rounds of back-to-back launches (HIP events).  The
rule-based default (Eq. 1 partition size, no cap, 64 rows per wave) is timed
beside the grid.

    python -m paper_2204_06666_amd.autotune --start 0 --count 50 --out sweep.jsonl
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import EHYB_F32, Plan, features
from .predictor import ROWS_PER_WAVE, SLICE_ROWS, WIDTH_QUANTILES, lds_max_rows, width_cap


def time_spmv(torch, plan, x, y, launches: int = 20, rounds: int = 3) -> float:
    """Seconds per launch: the best of `rounds` means over `launches` launches."""
    plan.spmv(x, y)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(rounds):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(launches):
            plan.spmv(x, y)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3 / launches)
    return best


def sweep_matrix(A, device="cuda:0", launches: int = 20, rounds: int = 3) -> dict:
    """Times (us) of every grid point, as times_us[slice][width][rows per
    wave] in the order of the grid tuples, and of the Eq. 1 default."""
    import torch
    x = torch.from_numpy(np.random.Generator(np.random.PCG64(7)).uniform(-1, 1, A.n_rows)
                         .astype(np.float32)).to(device)
    y = torch.empty_like(x)
    lens = np.diff(A.row_ptr)
    times = []
    t_pre = 0.0
    for s in SLICE_ROWS:
        rows = s if s else lds_max_rows()
        t0 = time.perf_counter()
        base = Plan(A, value_dtype=EHYB_F32, slice_rows=rows)
        part = base.partition()
        t_pre += time.perf_counter() - t0
        per_s = []
        for q in WIDTH_QUANTILES:
            per_q = []
            for rpw in ROWS_PER_WAVE:
                t0 = time.perf_counter()
                if q is None and rpw == 64:
                    p = base
                else:
                    p = Plan(A, value_dtype=EHYB_F32, partition=part, ell_width_cap=width_cap(lens, q),
                             rows_per_wave=rpw)
                t_pre += time.perf_counter() - t0
                p.upload(device)
                per_q.append(round(time_spmv(torch, p, x, y, launches, rounds) * 1e6, 2))
                if p is not base:
                    del p
            per_s.append(per_q)
        times.append(per_s)
        del base
    d = Plan(A, value_dtype=EHYB_F32).upload(device)
    eq1 = {"slice_rows": d.stats()["slice_rows"], "time_us": round(time_spmv(torch, d, x, y, launches, rounds) * 1e6, 2)}
    return {"slice_rows": list(SLICE_ROWS), "width_q": list(WIDTH_QUANTILES), "rows_per_wave": list(ROWS_PER_WAVE),
            "times_us": times, "eq1": eq1, "preprocess_s": round(t_pre, 2)}


def plan_for_point(A, point) -> Plan:
    """The FP32 plan of grid point (partition size, width quantile, rows per
    wave), built as the sweep builds it: a partition of that size, then the
    encoding with that ELL cap and lane count."""
    s, q, r = point
    base = Plan(A, value_dtype=EHYB_F32, slice_rows=s or lds_max_rows())
    return Plan(A, value_dtype=EHYB_F32, partition=base.partition(), ell_width_cap=width_cap(np.diff(A.row_ptr), q),
                rows_per_wave=r)


def choose_plan(predictor, A, device="cuda:0") -> Plan:
    """The FP32 plan of the point the predictor chooses for A, or the Eq. 1
    default plan where A lies outside the predictor's training range."""
    pt = predictor.choose([features(A)], [A.n_rows], device)[0]
    return plan_for_point(A, pt) if pt is not None else Plan(A, value_dtype=EHYB_F32)


def grid_points(rec: dict):
    """[(slice_rows, width_q, rows_per_wave, time_us)] of a sweep record."""
    out = []
    for i, s in enumerate(rec["slice_rows"]):
        for j, q in enumerate(rec["width_q"]):
            for k, r in enumerate(rec["rows_per_wave"]):
                out.append((s, q, r, rec["times_us"][i][j][k]))
    return out


def best_point(rec: dict):
    return min(grid_points(rec), key=lambda g: g[3])


# the batched product: launch shape and plan parameters shared by the batch
BATCH_GRID = {"lds_bytes": (40 * 1024, 54 * 1024, 80 * 1024, 160 * 1024), "rows_per_wave": (64, 16),
              "halo_rows": (0, -1)}


def tune_batch(mats, n_rhs: int = 8, device="cuda:0", launches: int = 20, rounds: int = 3, log=None) -> dict:
    """Exhaustive tuning of the batched product (FP32 values): every point of
    BATCH_GRID builds the batch's plans and times one launch over all of
    them.  Returns {"best": params, "points": [[params, us], ...]}."""
    import itertools

    import torch

    from . import Batch
    g = np.random.Generator(np.random.PCG64(4999))
    X0 = [g.uniform(-1.0, 1.0, (A.n_rows, n_rhs)).astype(np.float32) for A in mats]
    points = []
    keys = list(BATCH_GRID)
    for combo in itertools.product(*(BATCH_GRID[k] for k in keys)):
        prm = dict(zip(keys, combo))
        plans = [Plan(A, value_dtype=EHYB_F32, n_rhs=n_rhs, **prm).upload(device) for A in mats]
        B = Batch(plans, n_rhs, device)
        Xd = [torch.from_numpy(x[p.perm()]).to(device) for x, p in zip(X0, plans)]
        Yd = [torch.empty_like(x) for x in Xd]
        B.spmm(Xd, Yd)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(rounds):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(launches):
                B.spmm(Xd, Yd)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e3 / launches)
        points.append([prm, round(best, 2)])
        if log:
            log(f"batch point {prm}: {best:.1f} us")
        del B, plans, Xd, Yd
    best = min(points, key=lambda q: q[1])
    return {"n_rhs": n_rhs, "best": best[0], "best_us": best[1], "points": points}


def main(argv=None):
    import matgen

    ap = argparse.ArgumentParser()
    ap.add_argument("--start", type=int, default=0)
    ap.add_argument("--count", type=int, default=10)
    ap.add_argument("--n-lo", type=int, default=10_000)
    ap.add_argument("--n-hi", type=int, default=250_000)
    ap.add_argument("--out", required=True)
    ap.add_argument("--indices", type=int, nargs="*", default=None,
                    help="sweep these matrix indices instead of --start/--count")
    ap.add_argument("--batch", action="store_true",
                    help="tune the batched product of the 64-matrix batch instead (writes JSON)")
    args = ap.parse_args(argv)
    if args.batch:
        mats = [A for _, A in matgen.batch_matrices(64)]
        res = tune_batch(mats, log=lambda m: print(f"[autotune] {m}", flush=True))
        json.dump(res, open(args.out, "w"), indent=1)
        print(f"[autotune] batch best {res['best']} {res['best_us']} us", flush=True)
        return 0
    with open(args.out, "a") as f:
        for i in (args.indices if args.indices else range(args.start, args.start + args.count)):
            t0 = time.perf_counter()
            desc, A = matgen.tuning_matrix(i, n_lo=args.n_lo, n_hi=args.n_hi)
            t_gen = time.perf_counter() - t0
            rec = {"i": i, "desc": desc, "n": int(A.n_rows), "nnz": int(A.nnz),
                   "features": [float(f"{v:.7g}") for v in features(A)]}
            rec.update(sweep_matrix(A))
            f.write(json.dumps(rec) + "\n")
            f.flush()
            s, q, r, t = best_point(rec)
            print(f"[autotune] {i} {desc} n={A.n_rows} nnz={A.nnz} best=({s},{q},{r}) {t:.1f}us "
                  f"eq1 {rec['eq1']['time_us']:.1f}us gen {t_gen:.1f}s pre {rec['preprocess_s']:.1f}s "
                  f"total {time.perf_counter() - t0:.1f}s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
