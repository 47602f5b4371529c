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


def load_traffic(kernel_hash, name="ehyb_spmv_f64_stencil27_traffic.json"):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, only if
    they were taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", name)
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
    """Median time of single launches, each after a cache flush (`flush`
    reads 1 GiB with cache-allocating loads, evicting L2 and the 256 MB
    Infinity Cache and leaving no dirty lines), bracketed by HIP events."""
    ts = []
    for _ in range(reps):
        flush()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        fn()
        ev1.record()
        torch.cuda.synchronize()
        ts.append(ev0.elapsed_time(ev1) * 1e-3)
    return statistics.median(ts)


def time_cold_graph(torch, fn, flush, n=20, reps=7):
    """What a product adds to a stream after a cache flush: a HIP graph of n
    (flush, product) pairs against one of n flushes, median of `reps` replays
    each, difference per product.  `fn` and `flush` take the capture stream."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        flush(s)
        fn(s)
    torch.cuda.synchronize()
    graphs = []
    for with_product in (True, False):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            for _ in range(n):
                flush(s)
                if with_product:
                    fn(s)
        graphs.append(g)
    out = []
    for g in graphs:
        ts = []
        for _ in range(reps):
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            g.replay()
            ev1.record()
            torch.cuda.synchronize()
            ts.append(ev0.elapsed_time(ev1) * 1e-3)
        out.append(statistics.median(ts))
    del graphs
    return (out[0] - out[1]) / n


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_oracle_baseline(oracle, A, x, flops, what):
    """The CPU oracle (plain FP64 CSR, OpenMP over rows) on the whole matrix:
    one warm-up product, then the median of 5, on 1 thread and on all the
    threads OpenMP is given."""
    nthr = oracle.max_threads()
    legs = {}
    for th in sorted({1, nthr}):
        oracle.spmv(A, x, threads=th)
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            oracle.spmv(A, x, threads=th)
            ts.append(time.perf_counter() - t0)
        legs[th] = statistics.median(ts)
    return {"value": round(flops / legs[nthr] / 1e9, 3), "unit": "GFLOP/s", "cores": nthr, "kind": "oracle",
            "sample": f"{what}: one warm-up product, then the median of 5, on {nthr} threads "
                      f"(and on 1: single_thread_GFLOPs)",
            "single_thread_GFLOPs": round(flops / legs[1] / 1e9, 3),
            "ms_per_product": {str(k): round(v * 1e3, 3) for k, v in legs.items()},
            "cpu_model": cpu_model()}


class RocsparseSpmv:
    """The vendor CSR product as a comparator: rocSPARSE's generic SpMV
    (the copy bundled with torch, so that it shares torch's HIP runtime),
    FP64, int32 indices, one algorithm (adaptive by default), its buffer
    sizing and preprocessing done once, so that a call is the compute stage
    alone, on torch's current stream."""
    ALG = {"adaptive": 2, "rowsplit": 3, "lrb": 7, "nnzsplit": 8}

    def __init__(self, torch, row_ptr, col, val, x, y, alg="adaptive"):
        import ctypes
        self.ct = ctypes
        self.lib = ctypes.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "librocsparse.so"))
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        n = len(row_ptr) - 1
        dev = x.device
        self.keep = [torch.from_numpy(row_ptr.astype("int32")).to(dev), torch.from_numpy(col.astype("int32")).to(dev),
                     torch.from_numpy(val).to(dev), x, y]
        rp, ci, v = self.keep[:3]
        self.h, self.A, self.X, self.Y = vp(), vp(), vp(), vp()
        self._ok(self.lib.rocsparse_create_handle(ctypes.byref(self.h)), "create_handle")
        self._ok(self.lib.rocsparse_set_stream(self.h, vp(torch.cuda.current_stream().cuda_stream)), "set_stream")
        self._ok(self.lib.rocsparse_create_csr_descr(ctypes.byref(self.A), i64(n), i64(n), i64(len(col)),
                                                     vp(rp.data_ptr()), vp(ci.data_ptr()), vp(v.data_ptr()),
                                                     2, 2, 0, 152), "create_csr_descr")
        self._ok(self.lib.rocsparse_create_dnvec_descr(ctypes.byref(self.X), i64(n), vp(x.data_ptr()), 152), "dnvec x")
        self._ok(self.lib.rocsparse_create_dnvec_descr(ctypes.byref(self.Y), i64(n), vp(y.data_ptr()), 152), "dnvec y")
        self.alpha, self.beta = ctypes.c_double(1.0), ctypes.c_double(0.0)
        self.alg = self.ALG[alg]
        size = ctypes.c_size_t(0)
        self._stage(1, size, None)
        self.buf = torch.empty(max(int(size.value), 256), dtype=torch.uint8, device=dev)
        self._stage(2, size, self.buf)
        torch.cuda.synchronize()
        self.size = size

    def _ok(self, st, what):
        if st != 0:
            raise RuntimeError(f"rocsparse {what}: status {st}")

    def _stage(self, stage, size, buf):
        ct = self.ct
        self._ok(self.lib.rocsparse_spmv(self.h, 111, ct.byref(self.alpha), self.A, self.X, ct.byref(self.beta),
                                         self.Y, 152, self.alg, stage, ct.byref(size),
                                         ct.c_void_p(buf.data_ptr() if buf is not None else 0)), f"spmv stage {stage}")

    def __call__(self):
        self._stage(3, self.size, self.buf)

    def close(self):
        for f, o in (("rocsparse_destroy_dnvec_descr", self.X), ("rocsparse_destroy_dnvec_descr", self.Y),
                     ("rocsparse_destroy_spmat_descr", self.A), ("rocsparse_destroy_handle", self.h)):
            getattr(self.lib, f)(o)


def rocsparse_time(torch, row_ptr, col, val, x, steps, warmup):
    """rocSPARSE (adaptive CSR) per product: wall-clock and HIP-event time,
    and its result; None and the error if the library cannot be used."""
    y = torch.empty_like(x)
    try:
        op = RocsparseSpmv(torch, row_ptr, col, val, x, y)
    except (OSError, AttributeError, RuntimeError) as e:
        return None, None, None, str(e)
    wall, kern = time_launches(torch, op, steps, warmup)
    torch.cuda.synchronize()
    op.close()
    return wall, kern, y, None


def fp64_products(row_ptr, col, val, X):
    """A X and |A| |X| in FP64 by scipy's CSR product: the reference of the
    errors this benchmark reports (the row-by-row checks against the oracle
    are the tests' job)."""
    import numpy as np
    import scipy.sparse as sp
    n = len(row_ptr) - 1
    S = sp.csr_matrix((val, col, row_ptr), shape=(n, n))
    return S @ X, abs(S) @ np.abs(X)


def scaled_error(y, ref, scale):
    """|y - ref| / scale per entry; 0 where both are exact zeros of a zero scale."""
    import numpy as np
    err = np.abs(y - ref)
    return np.where(scale > 0, err / np.where(scale > 0, scale, 1.0), np.where(err == 0, 0.0, np.inf))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall-clock budget of the CPU oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="stencil27",
                    choices=["stencil27", "knn-fem", "batched", "predictor", "powerlaw"],
                    help="stencil27: the headline FP64 product (default); knn-fem: the "
                         "unstructured-FEM matrix in FP64, FP32 and BF16 values; batched: 64 "
                         "uneven FP32 matrices x 8 right-hand sides in one launch; predictor: the "
                         "learned preprocessing parameters on held-out matrices; powerlaw: "
                         "power-law graphs with hub rows against plain CSR")
    ap.add_argument("--count", type=int, default=64, help="batched only: number of matrices")
    ap.add_argument("--lds-bytes", type=int, default=None,
                    help="batched only: LDS budget per partition (default: the autotuner's choice)")
    ap.add_argument("--halo-rows", type=int, default=None, help="batched only: halo_rows of the plans")
    ap.add_argument("--rows-per-wave", type=int, default=None, help="batched only: rows_per_wave (64, 16 or 4)")
    ap.add_argument("--live", type=int, default=16, help="predictor only: held-out matrices re-timed live")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="knn-fem only: fraction of the 1e6 points")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the EHYB kernel runs on one device, "
              "multi-GPU sharding is a design note, not a benchmark here", file=sys.stderr)
        sys.exit(2)
    if args.workload == "knn-fem":
        return run_precision(args)
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "predictor":
        return run_predictor(args)
    if args.workload == "powerlaw":
        return run_powerlaw(args)

    import numpy as np
    import torch

    import matgen
    from paper_2204_06666_amd import (EHYB_LOAD_AUTO, EHYB_LOAD_CACHED, EHYB_LOAD_STREAM, Plan, cache_flush, csr_spmv,
                                      device_info, probe_read)
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

    # --- the same product recorded in a HIP graph: 50 launches per graph, 7
    # replays, median per launch (graph replays must give the eager bits)
    log("timing EHYB replayed from a HIP graph of 50 launches")
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(gs):
        plan.spmv(xp, yp, stream=gs)
    torch.cuda.current_stream().wait_stream(gs)
    torch.cuda.synchronize()
    y_eager = yp.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gs):
        for _ in range(50):
            plan.spmv(xp, yp, stream=gs)
    graph.replay()
    torch.cuda.synchronize()
    reps = []
    for _ in range(7):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1) * 1e-3 / 50)
    graph_s = statistics.median(reps)
    if not torch.equal(yp.view(torch.int64), y_eager.view(torch.int64)):
        raise SystemExit("graph replay differs from the eager product")
    del graph
    log(f"EHYB in a graph: {graph_s * 1e6:.2f} us/launch")

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
    for lanes in (2, 4, 8, 16, 32):
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
    for lanes in (2, 4, 8, 16):
        csr_re[lanes] = time_launches(torch, lambda: csr_spmv(rp2, ci2, cv2, xp, yo, lanes),
                                      args.steps, args.warmup)
    best_re = min(csr_re, key=lambda k: csr_re[k][0])

    # --- the vendor CSR product (rocSPARSE, through torch's sparse CSR), as context
    log("timing rocSPARSE (torch sparse CSR) on the matrix as given and on P A P^T")
    rs_wall, rs_kern, y_rs, rs_err = rocsparse_time(torch, A.row_ptr, A.col, A.val, xo, args.steps, args.warmup)
    rs2_wall, rs2_kern, _, _ = rocsparse_time(torch, drp, dci, dval, xp, args.steps, args.warmup)
    del drp, dci, dval, rp2, ci2, cv2

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

    # --- cold runs: L2 and the 256 MB Infinity Cache flushed before each launch
    log("cold timing")
    fbuf = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
    flush = lambda st=None: cache_flush(fbuf, sink, stream=st)  # noqa: E731
    cold = {}
    for mode_name, mode in (("plain", EHYB_LOAD_CACHED), ("stream", EHYB_LOAD_STREAM)):
        plan.set_load_mode(mode)
        cold[mode_name] = {
            "single_launch_us": time_cold(torch, lambda: plan.spmv(xp, yp), flush, 30),
            "after_flush_in_graph_us": time_cold_graph(torch, lambda st: plan.spmv(xp, yp, stream=st), flush)}
    plan.set_load_mode(EHYB_LOAD_AUTO)
    cold_csr = time_cold(torch, lambda: csr_spmv(rp, ci, cv, xo, yo, best_l), flush, 30)
    # a plain streaming read of the product's algorithmic bytes, timed the same
    # way: what HBM delivers cold to a launch of this size
    pbuf = torch.ones(algo // 64 * 64, dtype=torch.uint8, device=dev)
    cold_read = time_cold_graph(torch, lambda st: probe_read(pbuf, sink, stream=st), flush)
    del fbuf, pbuf
    # the cold headline: streaming loads (a product that reuses nothing from the
    # caches), the incremental time in a stream after other work
    cold_s = cold["stream"]["after_flush_in_graph_us"]
    log(f"cold: {json.dumps(cold)}")

    # --- CPU oracle baseline (the whole matrix; about a second of CPU work)
    cpu = None
    if not args.no_cpu:
        import oracle
        log("CPU oracle baseline")
        cpu = cpu_oracle_baseline(oracle, A, x, flops, "the whole headline matrix")

    # the vendor product's result against the plain CSR kernel's (both FP64)
    rocsparse = {"what": "rocSPARSE generic SpMV, CSR adaptive algorithm, FP64, int32 indices; buffer sizing "
                         "and preprocessing once, compute stage timed", "error": rs_err}
    if rs_err is None:
        y_csr = torch.empty_like(xo)
        csr_spmv(rp, ci, cv, xo, y_csr, best_l)
        rocsparse.update({"us_per_step": round(rs_wall * 1e6, 2), "GFLOPs": round(flops / rs_wall / 1e9, 2),
                          "algorithmic_GBps": round(csr_bytes / rs_kern / 1e9, 1),
                          "on_reordered_us_per_step": round(rs2_wall * 1e6, 2),
                          "on_reordered_GFLOPs": round(flops / rs2_wall / 1e9, 2),
                          "max_abs_diff_vs_csr_kernel": float(torch.max(torch.abs(y_rs - y_csr)).item())})

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
                     "traffic": traffic, "kernel": "ehyb_spmv_kernel<EHYB_F64, L=1, plain loads>",
                     "algorithmic_bytes_per_launch": algo, "launch_us": round(kern * 1e6, 2),
                     "timing": "warm: back-to-back launches, HIP events",
                     "cold": {"us": round(cold_s * 1e6, 2), "achieved": round(algo / cold_s / 1e9, 1),
                              "frac": round(algo / cold_s / 1e9 / PEAK_HBM_GBPS, 4),
                              "pct_of_measured_hbm": round(100 * algo / cold_s / 1e9 / hbm_meas, 2),
                              "same_size_read_cold_us": round(cold_read * 1e6, 2),
                              "pct_of_same_size_cold_read": round(100 * cold_read / cold_s, 2),
                              "load_mode": "stream",
                              "protocol": "L2 and Infinity Cache flushed (1 GiB read with cache-allocating "
                                          "loads) before each product; HIP graph of 20 (flush, product) pairs "
                                          "minus one of 20 flushes, median of 7 replays"}},
        "cpu_baseline": cpu,
        "hbm_probe_GBps": round(hbm_meas, 1),
        "pct_of_measured_hbm": round(100 * achieved / hbm_meas, 2),
        "csr": {"kernel": "CSR-vector, 4 entries per lane per batch, lanes per row swept",
                "lanes_per_row": best_l, "GFLOPs": round(flops / csr_wall / 1e9, 2),
                "us_per_step": round(csr_wall * 1e6, 2),
                "algorithmic_GBps": round(csr_bytes / csr_kern / 1e9, 1),
                "pct_of_8TBps": round(100 * csr_bytes / csr_kern / 8e12, 2),
                "all_us": {str(k): round(v[0] * 1e6, 2) for k, v in csr.items()}},
        "speedup_vs_csr": round(csr_wall / wall, 3),
        "csr_on_reordered": {"lanes_per_row": best_re, "GFLOPs": round(flops / csr_re[best_re][0] / 1e9, 2),
                             "us_per_step": round(csr_re[best_re][0] * 1e6, 2),
                             "algorithmic_GBps": round(csr_bytes / csr_re[best_re][1] / 1e9, 1),
                             "pct_of_8TBps": round(100 * csr_bytes / csr_re[best_re][1] / 8e12, 2)},
        "rocsparse_context": rocsparse,
        "speedup_vs_rocsparse": round(rs_wall / wall, 3) if rs_err is None else None,
        "ehyb_paper_split": {"GFLOPs": round(flops / wall_ps / 1e9, 2),
                             "us_per_step": round(wall_ps * 1e6, 2),
                             "algorithmic_GBps": round(st_ps["algorithmic_bytes"] / kern_ps / 1e9, 1),
                             "nnz_er": st_ps["nnz_er"], "er_slots": st_ps["er_slots"]},
        "warm_graph": {"us_per_launch": round(graph_s * 1e6, 2), "GFLOPs": round(flops / graph_s / 1e9, 2),
                       "protocol": "HIP graph of 50 launches, median of 7 replays"},
        "ehyb_with_permutation": {"GFLOPs": round(flops / wall_u / 1e9, 2),
                                  "us_per_step": round(wall_u * 1e6, 2)},
        "cold": {k: {kk: round(vv * 1e6, 2) for kk, vv in v.items()} for k, v in cold.items()},
        "cold_csr_us": round(cold_csr * 1e6, 2),
        "preprocess_s": round(t_pre, 2),
        "preprocess_breakdown_s": {k: round(st[k], 3) for k in ("t_graph_s", "t_partition_s", "t_reorder_s",
                                                                "t_encode_s")},
        "preprocess_over_spmv": round(t_pre / wall, 0),
        "kernel_source_sha256_16": kh,
    }
    print(json.dumps(out), flush=True)


KNN_TRAFFIC = {"f64": "ehyb_spmv_f64_knnfem_traffic.json", "f32": "ehyb_spmv_f32_knnfem_traffic.json",
               "bf16": "ehyb_spmv_bf16_knnfem_traffic.json"}


def run_precision(args):
    """Unstructured-FEM matrix (mutual kNN, 3x3 blocks): FP64 values against
    FP32 and BF16 values with binary32 x and accumulation, each with its error
    against the FP64 product of the original values (scipy's CSR product), its
    roofline (algorithmic bytes over the HIP-event time per product) and the
    committed rocprofv3 traffic of its kernel; the CPU oracle (FP64) on the
    whole matrix as the CPU baseline."""
    import numpy as np
    import torch

    import matgen
    from paper_2204_06666_amd import EHYB_BF16, EHYB_BF16_ACC64, EHYB_F32, EHYB_F32_ACC64, EHYB_F64, Plan

    dev = torch.device("cuda:0")
    log(f"generating the kNN-FEM matrix (scale {args.scale})")
    A = matgen.config_matrix(3, scale=args.scale)
    x = matgen.uniform_vector(A.n_rows, matgen.CONFIG_SEEDS[3] + 2)
    n, nnz = A.n_rows, A.nnz
    flops = 2.0 * nnz
    log(f"n={n} nnz={nnz}; FP64 reference product")
    y64, s64 = fp64_products(A.row_ptr, A.col, A.val, x)
    res = {}
    for name, dt in (("f64", EHYB_F64), ("f32", EHYB_F32), ("bf16", EHYB_BF16), ("f32_acc64", EHYB_F32_ACC64),
                     ("bf16_acc64", EHYB_BF16_ACC64)):
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
        e = scaled_error(y, y64, s64)
        res[name] = {"GFLOPs": round(flops / wall / 1e9, 2), "us_per_step": round(wall * 1e6, 2),
                     "algorithmic_bytes": st["algorithmic_bytes"],
                     "algorithmic_GBps": round(st["algorithmic_bytes"] / kern / 1e9, 1),
                     "pct_of_8TBps": round(100 * st["algorithmic_bytes"] / kern / 8e12, 2),
                     "roofline": {"bound": "hbm", "achieved": round(st["algorithmic_bytes"] / kern / 1e9, 1),
                                  "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                                  "frac": round(st["algorithmic_bytes"] / kern / 1e9 / PEAK_HBM_GBPS, 4),
                                  "traffic": load_traffic(kernel_source_hash(), KNN_TRAFFIC[name])
                                  if name in KNN_TRAFFIC else None,
                                  "launch_us": round(kern * 1e6, 2)},
                     "max_row_scaled_error_vs_fp64": float(e.max()),
                     "normwise_rel_error_vs_fp64": float(np.linalg.norm(y - y64) / np.linalg.norm(y64)),
                     "nparts": st["nparts"], "nnz_er": st["nnz_er"], "nnz_halo": st["nnz_halo"],
                     "preprocess_s": round(t_pre, 2)}
        if dt != EHYB_F64:
            # against the FP64 product of the values as the plan stores them
            # (P A P^T decoded) and x as the kernel reads it, in plan order
            rp, ci, v = plan.decode()
            yq, sq = fp64_products(rp, ci, v, xt.cpu().numpy().astype(np.float64))
            res[name]["max_row_scaled_error_vs_quantized"] = float(scaled_error(yp, yq, sq).max())
            del rp, ci, v
        log(f"{name}: {res[name]}")
        del plan, xt, yt
    cpu = None
    if not args.no_cpu:
        import oracle
        log("CPU oracle baseline")
        cpu = cpu_oracle_baseline(oracle, A, x, flops, "the whole kNN-FEM matrix (FP64)")
    r64 = res["f64"]["roofline"]
    out = {
        "metric": METRIC, "value": res["f64"]["GFLOPs"], "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res["f64"]["us_per_step"] / 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"mutual-kNN FEM stand-in, {int(1_000_000 * args.scale)} points ~U[0,1]^3, "
                               f"k ~ U{{12..40}}, 3x3 blocks (seeds 3000-3003)", "n": n, "nnz": nnz},
        "roofline": dict(r64, kernel="ehyb_spmv_kernel<EHYB_F64, L=1, streaming loads>",
                         algorithmic_bytes=res["f64"]["algorithmic_bytes"]),
        "cpu_baseline": cpu,
        "precision": res,
    }
    print(json.dumps(out), flush=True)


def run_batched(args):
    """64 matrices of uneven sizes (2-D Poisson, 27-point stencil, kNN-FEM),
    8 right-hand sides each, FP32 values, x and accumulation: one persistent
    launch over all (matrix, partition) work items, recorded in a HIP graph,
    against 64 x 8 separate single-vector products of plans built for one
    right-hand side."""
    import numpy as np
    import torch

    import matgen
    from paper_2204_06666_amd import EHYB_F32, Batch, Plan

    nrhs = 8
    dev = torch.device("cuda:0")
    # plan parameters: the committed batch autotuning result, unless given
    from paper_2204_06666_amd.workloads import BATCHED_PARAMS, batched_tuned
    tuned = batched_tuned() or BATCHED_PARAMS
    for k in ("lds_bytes", "halo_rows", "rows_per_wave"):
        if getattr(args, k) is None:
            setattr(args, k, tuned[k])
    log(f"plan parameters {dict(lds_bytes=args.lds_bytes, halo_rows=args.halo_rows, rows_per_wave=args.rows_per_wave)}")
    log(f"generating {args.count} matrices")
    mats = []
    for i, fm in enumerate(matgen.batch_matrices(args.count)):
        mats.append(fm)
        if i % 16 == 15:
            log(f"  {i + 1} matrices generated")
    sum_n = sum(A.n_rows for _, A in mats)
    sum_nnz = sum(A.nnz for _, A in mats)
    log(f"sum n={sum_n} sum nnz={sum_nnz}; preprocessing (n_rhs={nrhs} plans)")
    t0 = time.perf_counter()
    plans = []
    for i, (_, A) in enumerate(mats):
        plans.append(Plan(A, value_dtype=EHYB_F32, n_rhs=nrhs, lds_bytes=args.lds_bytes,
                          halo_rows=args.halo_rows, rows_per_wave=args.rows_per_wave).upload(dev))
        if i % 16 == 15:
            log(f"  {i + 1} plans built")
    t_pre = time.perf_counter() - t0
    B = Batch(plans, nrhs, dev)
    g = matgen.rng(4999)
    X = [g.uniform(-1.0, 1.0, (A.n_rows, nrhs)) for _, A in mats]
    Xd = [torch.from_numpy(x[p.perm()].astype(np.float32)).to(dev) for x, p in zip(X, plans)]
    Yd = [torch.empty_like(x) for x in Xd]
    flops = 2.0 * sum_nnz * nrhs
    algo = sum(p.stats()["algorithmic_bytes"] + 2 * (nrhs - 1) * p.n * 4 for p in plans)

    log("batched launch, eager")
    wall_e, kern_e = time_launches(torch, lambda: B.spmm(Xd, Yd), args.steps, args.warmup)
    log("batched launch, recorded in a HIP graph")
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        B.spmm(Xd, Yd)
    torch.cuda.current_stream().wait_stream(cs)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=cs):
        B.spmm(Xd, Yd, stream=cs)
    wall_g, kern_g = time_launches(torch, graph.replay, args.steps, args.warmup)
    torch.cuda.synchronize()

    # accuracy: every matrix against the FP64 product of its stored (binary32)
    # values and binary32 X, in plan order; the binary32 accumulation bound
    # gamma_{m+2}(2^-24) * (|A| |X|) per entry must hold
    log("checking all matrices against the FP64 product of the stored values")
    worst = 0.0
    u32 = 2.0 ** -24
    for i, (p, y, xd) in enumerate(zip(plans, Yd, Xd)):
        if i % 16 == 15:
            log(f"  {i + 1} matrices checked")
        rp, ci, v = p.decode()
        ref, sc = fp64_products(rp, ci, v, xd.cpu().numpy().astype(np.float64))
        m = np.diff(rp).astype(np.float64)[:, None] + 2.0
        e = scaled_error(y.cpu().numpy().astype(np.float64), ref, sc)
        if not np.all(e <= m * u32 / (1.0 - m * u32)):
            raise SystemExit("batched result outside the binary32 accumulation bound")
        worst = max(worst, float(e.max()))

    log("separate products: plans for one right-hand side, 8 launches per matrix")
    single = []
    for i, (_, A) in enumerate(mats):
        single.append(Plan(A, value_dtype=EHYB_F32).upload(dev))
        if i % 16 == 15:
            log(f"  {i + 1} single-vector plans built")
    xs = [torch.from_numpy(np.ascontiguousarray(x[p.perm()].T).astype(np.float32)).to(dev)
          for x, p in zip(X, single)]
    ys = [torch.empty_like(x) for x in xs]

    def separate():
        for p, x, y in zip(single, xs, ys):
            for r in range(nrhs):
                p.spmv(x[r], y[r])
    steps_sep = max(5, args.steps // 10)
    wall_s, kern_s = time_launches(torch, separate, steps_sep, max(2, args.warmup // 10))
    gs = torch.cuda.CUDAGraph()
    with torch.cuda.stream(cs):
        separate()
    torch.cuda.synchronize()
    with torch.cuda.graph(gs, stream=cs):
        separate()
    wall_sg, kern_sg = time_launches(torch, gs.replay, steps_sep, max(2, args.warmup // 10))
    # the separate products must agree with the batched one within twice the bound
    for (_, A), p1, pb, y1, yb in zip(mats[:8], single, plans, ys, Yd):
        a = np.empty((A.n_rows, nrhs))
        a[p1.perm()] = y1.cpu().numpy().T
        b = np.empty((A.n_rows, nrhs))
        b[pb.perm()] = yb.cpu().numpy()
        assert np.allclose(a, b, rtol=1e-4, atol=1e-4)

    cpu = None
    if not args.no_cpu:
        import oracle
        log("CPU oracle on the first matrices (bounded sample)")
        t0 = time.perf_counter()
        done_nnz, used = 0, []
        for (_, A), x in zip(mats, X):
            oracle.spmm(A, x)
            done_nnz += A.nnz
            used.append(A.n_rows)
            if time.perf_counter() - t0 > args.cpu_seconds:
                break
        t_cpu = time.perf_counter() - t0
        cpu = {"value": round(2.0 * done_nnz * nrhs / t_cpu / 1e9, 3), "unit": "GFLOP/s",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"FP64 CSR x 8 right-hand sides over the first {len(used)} matrices "
                         f"({done_nnz} nnz), one pass"}
    out = {
        "metric": "batched EHYB SpMM GFLOP/s, 64 uneven matrices x 8 RHS, FP32",
        "value": round(flops / wall_g / 1e9, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall_g * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.count} matrices, n log-uniform in [1e4, 5e5], 2-D Poisson / "
                               f"27-point stencil / kNN-FEM 3 dof (seeds 4000+i), 8 RHS ~ U[-1,1], FP32",
                   "plan": {"lds_bytes": args.lds_bytes or 160 * 1024, "halo_rows": args.halo_rows,
                            "rows_per_wave": args.rows_per_wave,
                            "source": "autotuner (paper_2204_06666_amd/data/batched_tuning.json)"
                            if batched_tuned() else "default"},
                   "sum_n": sum_n, "sum_nnz": sum_nnz, "work_items": sum(p.stats()["nparts"] for p in plans)},
        "roofline": {"bound": "hbm", "achieved": round(algo / kern_g / 1e9, 1), "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": round(algo / kern_g / 1e9 / PEAK_HBM_GBPS, 4),
                     "traffic": load_traffic(kernel_source_hash(), "ehyb_spmm_batched_f32x8_64mat_traffic.json"),
                     "kernel": "ehyb_spmm_batched_kernel<EHYB_F32, L=1, NRHS=8, streaming loads>"
                               + (" + er_pieces_batched_kernel (one product)" if any(p.stats()["n_er_pieces"]
                                                                                   for p in plans) else ""),
                     "algorithmic_bytes": algo, "launch_us": round(kern_g * 1e6, 2)},
        "cpu_baseline": cpu,
        "batched_eager_us": round(wall_e * 1e6, 2),
        "batched_graph_us": round(wall_g * 1e6, 2),
        "separate_eager_us": round(wall_s * 1e6, 2),
        "separate_graph_us": round(wall_sg * 1e6, 2),
        "speedup_vs_separate_graph": round(wall_sg / wall_g, 2),
        "max_row_scaled_error_vs_quantized": worst,
        "preprocess_s": round(t_pre, 1),
    }
    print(json.dumps(out), flush=True)


def run_powerlaw(args):
    """Power-law graphs (Chung-Lu) with hub rows of 10^4-10^5 entries, FP64
    and FP32 values, default plans (hub rows summed over the whole device
    before the product), plus the FP64 plan with a 64-entry ELL cap: EHYB
    against the plain CSR kernel and rocSPARSE on the same GPU, each checked
    against scipy's FP64 product.  The roofline is the FP64 default plan of
    the larger graph (both kernels of one product)."""
    import numpy as np
    import torch

    import matgen
    from paper_2204_06666_amd import EHYB_F32, EHYB_F64, Plan, csr_spmv
    from paper_2204_06666_amd.workloads import POWERLAW

    dev = torch.device("cuda:0")
    cases = [("n=6e4 exponent 2.2 mean degree 30", dict(n=60000, exponent=2.2, mean_deg=30, seed=5), 3),
             ("n=2.5e5 exponent 2.1 mean degree 40", POWERLAW["matgen"], POWERLAW["x_seed"])]
    res = []
    for desc, kw, xs in cases:
        log(f"generating power-law {desc}")
        A = matgen.powerlaw(**kw)
        x = matgen.uniform_vector(A.n_rows, xs)
        y64, s64 = fp64_products(A.row_ptr, A.col, A.val, x)
        rp = torch.from_numpy(A.row_ptr.astype(np.int32)).to(dev)
        ci = torch.from_numpy(A.col).to(dev)
        cv = torch.from_numpy(A.val).to(dev)
        xo = torch.from_numpy(x).to(dev)
        yo = torch.empty_like(xo)
        csr = {lanes: time_launches(torch, lambda: csr_spmv(rp, ci, cv, xo, yo, lanes), args.steps, args.warmup)[0]
               for lanes in (4, 8, 16, 32)}
        _, rs_k, _, rs_err = rocsparse_time(torch, A.row_ptr, A.col, A.val, xo, args.steps, args.warmup)
        row = {"matrix": desc, "n": int(A.n_rows), "nnz": int(A.nnz),
               "max_row": int(np.diff(A.row_ptr).max()),
               "csr_best_us": round(min(csr.values()) * 1e6, 2),
               "rocsparse_us": round(rs_k * 1e6, 2) if rs_k else rs_err}
        for name, dt, cap in (("f64", EHYB_F64, 0), ("f32", EHYB_F32, 0), ("f64_cap64", EHYB_F64, 64)):
            t0 = time.perf_counter()
            plan = Plan(A, value_dtype=dt, ell_width_cap=cap).upload(dev)
            t_pre = time.perf_counter() - t0
            st = plan.stats()
            xp = torch.from_numpy(x[plan.perm()].astype(np.float64 if dt == EHYB_F64 else np.float32)).to(dev)
            yp = torch.empty_like(xp)
            wall, _ = time_launches(torch, lambda: plan.spmv(xp, yp), args.steps, args.warmup)
            y = np.empty(A.n_rows)
            y[plan.perm()] = yp.cpu().numpy()
            row[name] = {"us": round(wall * 1e6, 2), "GFLOPs": round(2.0 * A.nnz / wall / 1e9, 2),
                         "algorithmic_bytes": st["algorithmic_bytes"],
                         "frac_of_8TBps": round(st["algorithmic_bytes"] / wall / 8e12, 4),
                         "nparts": st["nparts"], "nnz_er": st["nnz_er"], "n_er_wide": st["n_er_wide"],
                         "n_er_pieces": st["n_er_pieces"], "max_halo": st["max_halo"],
                         "preprocess_s": round(t_pre, 2),
                         "max_row_scaled_error_vs_fp64": float(scaled_error(y, y64, s64).max())}
            del plan, xp, yp
        row["speedup_f64_vs_csr"] = round(row["csr_best_us"] / row["f64"]["us"], 2)
        log(f"{row}")
        res.append(row)
        last = (A, x)
    big = res[-1]["f64"]
    batched = time_powerlaw_batch(args, torch, dev)
    cpu = None
    if not args.no_cpu:
        import oracle
        log("CPU oracle baseline")
        A, x = last
        cpu = cpu_oracle_baseline(oracle, A, x, 2.0 * A.nnz, "the whole 2.5e5-row power-law graph")
    out = {"metric": "EHYB SpMV on power-law graphs with hub rows, us per product", "value": big["us"],
           "unit": "us", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(big["us"] / 1e3, 5), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": POWERLAW["workload"]},
           "roofline": {"bound": "hbm", "achieved": round(big["algorithmic_bytes"] / big["us"] / 1e3, 1),
                        "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": big["frac_of_8TBps"],
                        "traffic": load_traffic(kernel_source_hash(), "ehyb_spmv_f64_powerlaw250k_traffic.json"),
                        "kernel": "er_pieces_kernel<EHYB_F64> + ehyb_spmv_kernel<EHYB_F64, L=1, plain loads> "
                                  "(one product)",
                        "algorithmic_bytes": big["algorithmic_bytes"], "launch_us": big["us"]},
           "cpu_baseline": cpu, "matrices": res, "batched": batched}
    print(json.dumps(out), flush=True)


def time_powerlaw_batch(args, torch, dev):
    """The batched product over 12 power-law graphs (hub rows summed in pieces
    over the whole device, for all graphs in one launch before the product):
    FP32 x 8 right-hand sides and FP64 x 1, each graph checked against
    scipy's FP64 product of the stored values."""
    import numpy as np

    import matgen
    from paper_2204_06666_amd import EHYB_F32, EHYB_F64, Batch, Plan
    from paper_2204_06666_amd.workloads import POWERLAW_BATCH, POWERLAW_BATCH_F32X8, powerlaw_batch

    log("generating the power-law batch")
    mats = powerlaw_batch()
    out = {"workload": f"{POWERLAW_BATCH['count']} Chung-Lu graphs, n log-uniform in [2e4, 2.5e5], exponent "
                       "U[2.1, 2.5], mean degree U[10, 40]",
           "n": int(sum(A.n_rows for A in mats)), "nnz": int(sum(A.nnz for A in mats))}
    for name, dt, prm in (("f32x8", EHYB_F32, POWERLAW_BATCH_F32X8), ("f64x1", EHYB_F64, dict(n_rhs=1, rows_per_wave=64))):
        n_rhs = prm["n_rhs"]
        plans = [Plan(A, value_dtype=dt, **prm).upload(dev) for A in mats]
        batch = Batch(plans, n_rhs, dev)
        g = matgen.rng(11)
        X = [g.uniform(-1, 1, (A.n_rows, n_rhs)) for A in mats]
        tdt = torch.float64 if dt == EHYB_F64 else torch.float32
        Xd = [torch.from_numpy(x[p.perm()]).to(dev, tdt).contiguous() for x, p in zip(X, plans)]
        Yd = [torch.empty_like(v) for v in Xd]
        wall, _ = time_launches(torch, lambda: batch.spmm(Xd, Yd), args.steps, args.warmup)
        err = 0.0
        for A, p, x, y in zip(mats, plans, X, Yd):
            xq = x if dt == EHYB_F64 else x.astype(np.float32).astype(np.float64)
            val = A.val if dt == EHYB_F64 else A.val.astype(np.float32).astype(np.float64)
            ref, s = fp64_products(A.row_ptr, A.col, val, xq)
            Y = np.empty((A.n_rows, n_rhs))
            Y[p.perm()] = y.cpu().numpy()
            err = max(err, float(scaled_error(Y, ref, s).max()))
        xb = 8 if dt == EHYB_F64 else 4
        algo = sum(p.stats()["algorithmic_bytes"] + 2 * (n_rhs - 1) * p.n * xb for p in plans)
        out[name] = {"us": round(wall * 1e6, 2), "GFLOPs": round(2.0 * out["nnz"] * n_rhs / wall / 1e9, 2),
                     "algorithmic_bytes": algo, "frac_of_8TBps": round(algo / wall / 8e12, 4),
                     "n_er_pieces": int(sum(p.stats()["n_er_pieces"] for p in plans)),
                     "max_scaled_error_vs_fp64": err}
        if name == "f32x8":
            out[name]["traffic"] = load_traffic(kernel_source_hash(), "ehyb_spmm_batched_f32x8_powerlaw12_traffic.json")
        log(f"power-law batch {name}: {out[name]}")
        del batch, plans, Xd, Yd
    return out


def run_predictor(args):
    """Learned preprocessing parameters (NEXT-3).  The network is trained here,
    on the device with the library's own kernels, on the committed sweep of
    the training matrices; the held-out matrices are judged on their recorded
    sweep times, and a sample of them is re-generated and re-timed live
    (predicted point, Eq. 1 default, recorded best)."""
    import numpy as np
    import torch

    import matgen
    from paper_2204_06666_amd import EHYB_F32, Plan, features
    from paper_2204_06666_amd.autotune import plan_for_point, time_spmv
    from paper_2204_06666_amd.train_predictor import Predictor, best, evaluate, load_sweeps, train

    data = os.path.join(ROOT, "paper_2204_06666_amd", "data")
    model = json.load(open(os.path.join(data, "predictor_fp32.json")))
    meta = model["meta"]
    recs = load_sweeps([os.path.join(data, "tuning_sweep.jsonl")])
    tr = [r for r in recs if r["i"] < meta["n_train"]]
    te = [r for r in recs if r["i"] >= meta["n_train"]]
    log(f"{len(tr)} training and {len(te)} held-out matrices; training on the device")
    t0 = time.perf_counter()
    pred, hist = train(tr, meta["epochs"], meta["batch"], meta["lr"], meta["seed"], meta.get("near", 0.0))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    same = bool(np.array_equal(pred.params, np.asarray(model["params"], dtype=np.float32)))
    points = pred.predict([r["features"] for r in te])
    held = evaluate(te, points)
    log(f"held-out (recorded times): {held}")
    live = []
    k = min(args.live, len(te))
    for rec, pt in list(zip(te, points))[:k]:
        desc, A = matgen.tuning_matrix(rec["i"], n_hi=250_000)
        f = features(A)
        if not np.allclose(f, rec["features"], rtol=1e-5, atol=1e-6):
            raise SystemExit(f"features of matrix {rec['i']} differ from the recorded sweep")
        x = torch.from_numpy(matgen.uniform_vector(A.n_rows, 7).astype(np.float32)).to("cuda:0")
        y = torch.empty_like(x)
        tp = time_spmv(torch, plan_for_point(A, pt).upload("cuda:0"), x, y, 50, 5)
        tb = time_spmv(torch, plan_for_point(A, best(rec)[0]).upload("cuda:0"), x, y, 50, 5)
        te1 = time_spmv(torch, Plan(A, value_dtype=EHYB_F32).upload("cuda:0"), x, y, 50, 5)
        live.append({"i": rec["i"], "desc": desc, "pred_us": round(tp * 1e6, 2), "best_us": round(tb * 1e6, 2),
                     "eq1_us": round(te1 * 1e6, 2)})
        log(f"  live {live[-1]}")
    gm = lambda a: float(np.exp(np.mean(np.log(a))))  # noqa: E731
    live_sum = {"n": len(live),
                "geomean_pred_over_best": gm([l["pred_us"] / l["best_us"] for l in live]) if live else None,
                "geomean_eq1_over_pred": gm([l["eq1_us"] / l["pred_us"] for l in live]) if live else None}
    out = {
        "metric": "learned EHYB parameters: held-out geomean SpMV time / exhaustive-grid best",
        "value": round(held["geomean_pred_over_best"], 4), "unit": "x", "n_gpus": 1,
        "steps": len(te), "warmup": 0, "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"tuning set: {len(tr)} training + {len(te)} held-out matrices, n log-uniform "
                               f"in [1e4, 2.5e5], stencil / kNN-FEM / power-law families (seeds 50000+i); grid "
                               f"6 partition sizes x 4 ELL width caps x 4 rows-per-wave, FP32",
                   "network": "32 -> 64 -> 64 -> 3, ReLU, binary32, Adam"},
        "held_out": held, "live": live_sum, "live_matrices": live,
        "train_s": round(t_train, 2), "train_loss": [hist[0], hist[-1]],
        "retrained_params_equal_committed": same,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
