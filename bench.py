"""Benchmark of the EHYB FP64 SpMV on one MI355X.

One step = one y = A x of the headline workload (27-point stencil, 100^3 grid,
randomly relabelled, 1e6 rows, 26,463,592 entries) with x and y in the plan's
permuted order (the solver use: preprocess once, then many products).  The
plain CSR comparator runs on the same GPU on the matrix as given.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0   # MI355X published HBM3E bandwidth
METRIC = "EHYB SpMV GFLOP/s & % HBM peak vs plain CSR, same MI355X, FP64 at 1e-12"


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    p = os.path.join(ROOT, "paper_2204_06666_amd", "csrc", "ehyb_device.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def load_traffic(kernel_hash):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, only if
    they were taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "ehyb_spmv_f64_stencil27_traffic.json")
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_hash:
        return None
    return d.get("bytes_per_launch")


def time_launches(torch, fn, steps, warmup):
    """Wall-clock and HIP-event time of `steps` back-to-back launches on the
    current stream, bracketed by device synchronisation."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    return wall, ev0.elapsed_time(ev1) * 1e-3 / steps


def time_cold(torch, fn, flush, reps):
    """Median per-launch time with L2 and the 256 MB Infinity Cache flushed
    first by reading (not writing) a larger buffer, so no dirty lines are left
    to be written back during the timed launch."""
    ts = []
    for i in range(reps):
        flush.sum()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        fn()
        ev1.record()
        torch.cuda.synchronize()
        ts.append(ev0.elapsed_time(ev1) * 1e-3)
    return statistics.median(ts)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall-clock budget of the CPU oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="stencil27", choices=["stencil27", "knn-fem"],
                    help="stencil27: the headline FP64 product (default); knn-fem: the "
                         "unstructured-FEM matrix in FP64, FP32 and BF16 values")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="knn-fem only: fraction of the 1e6 points")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the EHYB kernel runs on one device, "
              "multi-GPU sharding is a design note, not a benchmark here", file=sys.stderr)
        sys.exit(2)
    if args.workload == "knn-fem":
        return run_precision(args)

    import numpy as np
    import torch

    import matgen
    from paper_2204_06666_amd import Plan, csr_spmv, device_info, probe_read
    from paper_2204_06666_amd.workloads import HEADLINE, HEADLINE_PARAMS, PAPER_SPLIT_PARAMS

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    info = device_info()
    log(f"device {info['arch']} CUs={info['num_cus']} LDS/block={info['lds_per_block']}")

    log("generating the headline matrix")
    A = matgen.config_matrix(HEADLINE["config"])
    x = matgen.uniform_vector(A.n_rows, HEADLINE["x_seed"])
    n, nnz = A.n_rows, A.nnz
    flops = 2.0 * nnz

    log("preprocessing (partition, reorder, encode)")
    t0 = time.perf_counter()
    plan = Plan(A, **HEADLINE_PARAMS)
    t_pre = time.perf_counter() - t0
    st = plan.stats()
    log(f"plan: {st['nparts']} parts, ER fraction {st['nnz_er'] / nnz:.4f}, "
        f"{st['algorithmic_bytes'] / 1e6:.1f} MB/SpMV, preprocess {t_pre:.1f}s")
    plan.upload(dev)
    perm = plan.perm()
    xp = torch.from_numpy(x[perm]).to(dev)
    yp = torch.empty(n, dtype=torch.float64, device=dev)
    xo = torch.from_numpy(x).to(dev)
    yo = torch.empty(n, dtype=torch.float64, device=dev)

    # --- headline: EHYB in permuted space
    log(f"timing EHYB: {args.warmup} warm-up + {args.steps} steps")
    wall, kern = time_launches(torch, lambda: plan.spmv(xp, yp), args.steps, args.warmup)
    gflops = flops / wall / 1e9
    algo = st["algorithmic_bytes"]
    achieved = algo / kern / 1e9
    log(f"EHYB: {wall * 1e6:.1f} us/step wall, {kern * 1e6:.1f} us/launch (events), "
        f"{gflops:.1f} GFLOP/s, {achieved:.0f} GB/s algorithmic")

    # --- the paper's split: no halo, every outside entry in the residual part
    log("timing EHYB with the paper's split (no halo)")
    plan_ps = Plan(A, **PAPER_SPLIT_PARAMS).upload(dev)
    st_ps = plan_ps.stats()
    xps = torch.from_numpy(x[plan_ps.perm()]).to(dev)
    wall_ps, kern_ps = time_launches(torch, lambda: plan_ps.spmv(xps, yp), args.steps, args.warmup)

    # --- EHYB including the permutation of x and y (vectors in original order)
    wall_u, kern_u = time_launches(torch, lambda: plan.spmv(xo, yo, permuted=False), args.steps,
                                   args.warmup)

    # --- plain CSR comparator on the matrix as given: best lanes-per-row
    log("timing plain CSR comparator")
    rp = torch.from_numpy(A.row_ptr.astype(np.int32)).to(dev)
    ci = torch.from_numpy(A.col).to(dev)
    cv = torch.from_numpy(A.val).to(dev)
    csr = {}
    for lanes in (4, 8, 16, 32):
        w, k = time_launches(torch, lambda: csr_spmv(rp, ci, cv, xo, yo, lanes), args.steps,
                             args.warmup)
        csr[lanes] = (w, k)
    best_l = min(csr, key=lambda k: csr[k][0])
    csr_wall, csr_kern = csr[best_l]
    csr_bytes = nnz * 12 + (n + 1) * 4 + 2 * n * 8
    log(f"CSR best lanes={best_l}: {csr_wall * 1e6:.1f} us/step, {flops / csr_wall / 1e9:.1f} GFLOP/s")

    # --- ablation: CSR on the reordered matrix P A P^T
    drp, dci, dval = plan.decode()
    rp2 = torch.from_numpy(drp.astype(np.int32)).to(dev)
    ci2 = torch.from_numpy(dci).to(dev)
    cv2 = torch.from_numpy(dval).to(dev)
    csr_re = {}
    for lanes in (8, 16, 32):
        csr_re[lanes] = time_launches(torch, lambda: csr_spmv(rp2, ci2, cv2, xp, yo, lanes),
                                      args.steps, args.warmup)
    best_re = min(csr_re, key=lambda k: csr_re[k][0])

    # --- HBM bandwidth probe (read stream over 4 GiB, best of 10)
    log("bandwidth probe")
    buf = torch.empty(4 << 30, dtype=torch.uint8, device=dev)
    buf.fill_(1)
    sink = torch.empty(65536, dtype=torch.int64, device=dev)
    bw = []
    for _ in range(10):
        w, k = time_launches(torch, lambda: probe_read(buf, sink), 1, 1 if not bw else 0)
        bw.append(buf.numel() / k / 1e9)
    hbm_meas = max(bw)
    del buf

    # --- cold runs: flush L2 and the 256 MB Infinity Cache before each launch
    log("cold timing")
    flush = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
    cold_ehyb = time_cold(torch, lambda: plan.spmv(xp, yp), flush, 30)
    cold_csr = time_cold(torch, lambda: csr_spmv(rp, ci, cv, xo, yo, best_l), flush, 30)
    del flush

    # --- CPU oracle baseline (bounded sample: whole matrix, repeated ~cpu-seconds)
    cpu = None
    if not args.no_cpu:
        import oracle
        log("CPU oracle baseline")
        oracle.spmv(A, x)
        reps, t0 = 0, time.perf_counter()
        while True:
            oracle.spmv(A, x)
            reps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds:
                break
        cpu = {"value": round(flops * reps / el / 1e9, 3), "unit": "GFLOP/s",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"whole headline matrix, {reps} products in {el:.1f} s "
                         f"(plain FP64 CSR, OpenMP over rows)"}

    kh = kernel_source_hash()
    traffic = load_traffic(kh)
    out = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": HEADLINE["workload"], "n": n, "nnz": nnz,
                   "vectors": "permuted order (x, y as the plan stores them)",
                   "plan": {k: st[k] for k in ("nparts", "slice_rows", "max_part_rows",
                                               "rows_per_slice", "lanes_per_row", "nnz_er",
                                               "nnz_halo", "n_halo", "max_halo", "ell_slots",
                                               "er_slots", "lds_bytes_used")}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBPS, 4),
                     "traffic": traffic, "kernel": "ehyb_spmv_f64_kernel<1>",
                     "algorithmic_bytes_per_launch": algo, "launch_us": round(kern * 1e6, 2)},
        "cpu_baseline": cpu,
        "hbm_probe_GBps": round(hbm_meas, 1),
        "pct_of_measured_hbm": round(100 * achieved / hbm_meas, 2),
        "csr": {"lanes_per_row": best_l, "GFLOPs": round(flops / csr_wall / 1e9, 2),
                "us_per_step": round(csr_wall * 1e6, 2),
                "algorithmic_GBps": round(csr_bytes / csr_kern / 1e9, 1),
                "all": {str(k): round(v[0] * 1e6, 2) for k, v in csr.items()}},
        "speedup_vs_csr": round(csr_wall / wall, 3),
        "csr_on_reordered": {"lanes_per_row": best_re,
                             "GFLOPs": round(flops / csr_re[best_re][0] / 1e9, 2)},
        "ehyb_paper_split": {"GFLOPs": round(flops / wall_ps / 1e9, 2),
                             "us_per_step": round(wall_ps * 1e6, 2),
                             "algorithmic_GBps": round(st_ps["algorithmic_bytes"] / kern_ps / 1e9, 1),
                             "nnz_er": st_ps["nnz_er"], "er_slots": st_ps["er_slots"]},
        "ehyb_with_permutation": {"GFLOPs": round(flops / wall_u / 1e9, 2),
                                  "us_per_step": round(wall_u * 1e6, 2)},
        "cold": {"ehyb_us": round(cold_ehyb * 1e6, 2), "csr_us": round(cold_csr * 1e6, 2),
                 "ehyb_GFLOPs": round(flops / cold_ehyb / 1e9, 2),
                 "ehyb_pct_measured_hbm": round(100 * algo / cold_ehyb / 1e9 / hbm_meas, 2)},
        "preprocess_s": round(t_pre, 2),
        "preprocess_over_spmv": round(t_pre / wall, 0),
        "kernel_source_sha256_16": kh,
    }
    print(json.dumps(out), flush=True)


def run_precision(args):
    """Unstructured-FEM matrix (mutual kNN, 3x3 blocks): FP64 values against
    FP32 and BF16 values with binary32 x and accumulation, each with its error
    against the FP64 oracle."""
    import numpy as np
    import torch

    import matgen
    import oracle
    from oracle.precision import quantize
    from paper_2204_06666_amd import EHYB_BF16, EHYB_F32, EHYB_F64, Plan

    dev = torch.device("cuda:0")
    log(f"generating the kNN-FEM matrix (scale {args.scale})")
    A = matgen.config_matrix(3, scale=args.scale)
    x = matgen.uniform_vector(A.n_rows, matgen.CONFIG_SEEDS[3] + 2)
    n, nnz = A.n_rows, A.nnz
    flops = 2.0 * nnz
    log(f"n={n} nnz={nnz}; FP64 oracle")
    y64 = oracle.spmv(A, x)
    s64 = oracle.abs_scale(A, x)
    res = {}
    for name, dt in (("f64", EHYB_F64), ("f32", EHYB_F32), ("bf16", EHYB_BF16)):
        log(f"preprocessing {name}")
        t0 = time.perf_counter()
        plan = Plan(A, value_dtype=dt).upload(dev)
        t_pre = time.perf_counter() - t0
        st = plan.stats()
        perm = plan.perm()
        xt = torch.from_numpy(x[perm].astype(np.float64 if dt == EHYB_F64 else np.float32)).to(dev)
        yt = torch.empty_like(xt)
        wall, kern = time_launches(torch, lambda: plan.spmv(xt, yt), args.steps, args.warmup)
        yp = yt.cpu().numpy().astype(np.float64)
        y = np.empty_like(yp)
        y[perm] = yp
        e = oracle.scaled_error(y, y64, s64)
        res[name] = {"GFLOPs": round(flops / wall / 1e9, 2), "us_per_step": round(wall * 1e6, 2),
                     "algorithmic_bytes": st["algorithmic_bytes"],
                     "algorithmic_GBps": round(st["algorithmic_bytes"] / kern / 1e9, 1),
                     "pct_of_8TBps": round(100 * st["algorithmic_bytes"] / kern / 8e12, 2),
                     "max_row_scaled_error_vs_fp64": float(e.max()),
                     "normwise_rel_error_vs_fp64": float(np.linalg.norm(y - y64) / np.linalg.norm(y64)),
                     "nparts": st["nparts"], "nnz_er": st["nnz_er"], "nnz_halo": st["nnz_halo"],
                     "preprocess_s": round(t_pre, 2)}
        if dt != EHYB_F64:
            Aq = matgen.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, quantize(A.val, name))
            xq = x.astype(np.float32).astype(np.float64)
            eq = oracle.scaled_error(y, oracle.spmv(Aq, xq), oracle.abs_scale(Aq, xq))
            res[name]["max_row_scaled_error_vs_quantized"] = float(eq.max())
        log(f"{name}: {res[name]}")
        del plan, xt, yt
    out = {
        "metric": METRIC, "value": res["f64"]["GFLOPs"], "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res["f64"]["us_per_step"] / 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"mutual-kNN FEM stand-in, {int(1_000_000 * args.scale)} points ~U[0,1]^3, "
                               f"k ~ U{{12..40}}, 3x3 blocks (seeds 3000-3003)", "n": n, "nnz": nnz},
        "precision": res,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
