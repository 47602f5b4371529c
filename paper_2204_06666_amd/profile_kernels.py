"""Fixed kernel sequence for hardware-counter runs (rocprofv3 --pmc).

Runs the headline EHYB FP64 product (or, with ``--workload batched``, the
batched product of 64 FP32 matrices x 8 right-hand sides; with ``--workload
powerlaw``, the FP64 product of the 2.5e5-row power-law graph with hub rows,
default plan: the hub-row pre-pass, then the product; with ``--workload
powerlaw-batched``, the batched FP32 product of 12 power-law graphs x 8
right-hand sides, pre-pass and product; with ``--workload
knnfem``, the products of the 3e6-row kNN-FEM matrix with FP64, FP32 and
BF16 values, one after the other) `--reps` times and
the copy probe on a buffer of known size `--reps` times, nothing else on the GPU, so that the
per-dispatch FETCH_SIZE / WRITE_SIZE of each kernel can be read off and the
EHYB counters scaled by what the same counters report for the copy of a known
number of bytes.  One line per product kind is printed:
``ehyb[TAG] algorithmic_bytes=... copy_bytes_read=... copy_bytes_written=...``.

    rocprofv3 --pmc FETCH_SIZE -d OUT -o fetch -- python3 paper_2204_06666_amd/profile_kernels.py

``--cache-dir DIR`` keeps the generated kNN-FEM matrix and its plans between
the counter passes of one session (the matrix takes about a minute to
generate).
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--workload", default="stencil27", choices=["stencil27", "batched", "powerlaw", "powerlaw-batched", "knnfem"])
    ap.add_argument("--cache-dir", default=None, help="knnfem: keep the matrix and plans here between runs")
    args = ap.parse_args()
    import torch

    import matgen
    from paper_2204_06666_amd import Plan, probe_copy
    from paper_2204_06666_amd.workloads import HEADLINE, HEADLINE_PARAMS

    dev = torch.device("cuda:0")
    tags = ["ehyb"]
    if args.workload == "stencil27":
        A = matgen.config_matrix(HEADLINE["config"])
        x = matgen.uniform_vector(A.n_rows, HEADLINE["x_seed"])
        plan = Plan(A, **HEADLINE_PARAMS).upload(dev)
        algo = plan.stats()["algorithmic_bytes"]
        xp = torch.from_numpy(x[plan.perm()]).to(dev)
        yp = torch.empty_like(xp)
        run = lambda: plan.spmv(xp, yp)  # noqa: E731
    elif args.workload == "powerlaw":
        from paper_2204_06666_amd.workloads import POWERLAW
        A = matgen.powerlaw(**POWERLAW["matgen"])
        x = matgen.uniform_vector(A.n_rows, POWERLAW["x_seed"])
        plan = Plan(A).upload(dev)
        algo = plan.stats()["algorithmic_bytes"]
        xp = torch.from_numpy(x[plan.perm()]).to(dev)
        yp = torch.empty_like(xp)
        run = lambda: plan.spmv(xp, yp)  # noqa: E731
    elif args.workload == "powerlaw-batched":
        from paper_2204_06666_amd import EHYB_F32, Batch
        from paper_2204_06666_amd.workloads import POWERLAW_BATCH_F32X8, powerlaw_batch
        mats = powerlaw_batch()
        nrhs = POWERLAW_BATCH_F32X8["n_rhs"]
        plans = [Plan(A, value_dtype=EHYB_F32, **POWERLAW_BATCH_F32X8).upload(dev) for A in mats]
        batch = Batch(plans, nrhs, dev)
        g = matgen.rng(11)
        Xd = [torch.from_numpy(g.uniform(-1, 1, (A.n_rows, nrhs))).to(dev, torch.float32).contiguous() for A in mats]
        Yd = [torch.empty_like(v) for v in Xd]
        algo = sum(p.stats()["algorithmic_bytes"] + 2 * (nrhs - 1) * p.n * 4 for p in plans)
        run = lambda: batch.spmm(Xd, Yd)  # noqa: E731
    elif args.workload == "knnfem":
        import numpy as np

        from paper_2204_06666_amd import EHYB_BF16, EHYB_F32, EHYB_F64
        A = _knn_matrix(args.cache_dir)
        x = matgen.uniform_vector(A.n_rows, matgen.CONFIG_SEEDS[3] + 2)
        tags, algo, runs = [], [], []
        for tag, dt in (("f64", EHYB_F64), ("f32", EHYB_F32), ("bf16", EHYB_BF16)):
            plan = _cached_plan(A, dt, args.cache_dir, tag).upload(dev)
            xt = torch.from_numpy(x[plan.perm()].astype(np.float64 if dt == EHYB_F64 else np.float32)).to(dev)
            runs.append((plan, xt, torch.empty_like(xt)))
            tags.append(f"ehyb[{tag}]")
            algo.append(plan.stats()["algorithmic_bytes"])

        def run():
            for p, xt, yt in runs:
                for _ in range(args.reps):
                    p.spmv(xt, yt)
    else:
        from paper_2204_06666_amd import EHYB_F32, Batch
        from paper_2204_06666_amd.workloads import BATCHED_PARAMS, batched_tuned
        prm = batched_tuned() or BATCHED_PARAMS
        nrhs = prm["n_rhs"]
        mats = [A for _, A in matgen.batch_matrices(64)]
        plans = [Plan(A, value_dtype=EHYB_F32, **prm).upload(dev) for A in mats]
        batch = Batch(plans, nrhs, dev)
        g = matgen.rng(4999)
        Xd = [torch.from_numpy(g.uniform(-1, 1, (A.n_rows, nrhs)).astype("float32")).to(dev) for A in mats]
        Yd = [torch.empty_like(v) for v in Xd]
        algo = sum(p.stats()["algorithmic_bytes"] + 2 * (nrhs - 1) * p.n * 4 for p in plans)
        run = lambda: batch.spmm(Xd, Yd)  # noqa: E731
    src = torch.ones((args.copy_mib << 20) // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    if args.workload == "knnfem":
        run()  # each product kind `reps` times in a row
    else:
        for _ in range(args.reps):
            run()
        algo = [algo]
    torch.cuda.synchronize()
    for _ in range(args.reps):
        probe_copy(src, dst)
    torch.cuda.synchronize()
    for tag, a in zip(tags, algo):
        print(f"{tag} algorithmic_bytes={a} copy_bytes_read={src.numel() * 4} "
              f"copy_bytes_written={dst.numel() * 4} reps={args.reps}", flush=True)


def _knn_matrix(cache_dir):
    """The 3e6-row kNN-FEM matrix, generated or read back from `cache_dir`."""
    import numpy as np

    import matgen
    path = os.path.join(cache_dir, "knnfem.npz") if cache_dir else None
    if path and os.path.exists(path):
        z = np.load(path)
        return matgen.Csr(int(z["n"]), int(z["n"]), z["row_ptr"], z["col"], z["val"])
    A = matgen.config_matrix(3)
    if path:
        os.makedirs(cache_dir, exist_ok=True)
        np.savez(path, n=A.n_rows, row_ptr=A.row_ptr, col=A.col, val=A.val)
    return A


def _cached_plan(A, dt, cache_dir, tag):
    from paper_2204_06666_amd import Plan
    path = os.path.join(cache_dir, f"knnfem_{tag}.plan") if cache_dir else None
    if path and os.path.exists(path):
        return Plan.load(path)
    plan = Plan(A, value_dtype=dt)
    if path:
        plan.save(path)
    return plan


if __name__ == "__main__":
    main()
