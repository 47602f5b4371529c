"""Named workloads and the plan parameters the benchmark times them with.

The headline workload is the randomly relabelled 27-point stencil on a 100^3
grid (1,000,000 rows, 26,463,592 stored entries, FP64).  Its plan parameters
live here so that the benchmark and the full-size parity test launch the same
configuration.
"""

HEADLINE = {
    "name": "stencil27-100^3",
    "workload": "27-point stencil on a 100^3 grid, nodes randomly relabelled (seed 2000), "
                "off-diagonals ~U[-1,1] (seed 2001), dominant diagonal; x ~U[-1,1] (seed 2002); "
                "FP64 values, FP64 x/y/accumulation",
    "config": 2,
    "n": 1_000_000,
    "nnz": 26_463_592,
    "x_seed": 2002,
}

# Plan parameters of the headline run (zero = the Eq. 1-2 / library default).
HEADLINE_PARAMS = {
    "slice_rows": 0,
    "rows_per_wave": 64,
    "ell_width_cap": 0,
    "halo_rows": 0,        # neighbour x entries cached in LDS as far as it allows
    "seed": 0,
}

# The paper's split: every entry outside the partition goes to the residual
# part and reads x from device memory.
PAPER_SPLIT_PARAMS = dict(HEADLINE_PARAMS, halo_rows=-1, ell_width_cap=-1)

# The larger power-law graph (Chung-Lu, hub rows of ~10^5 entries) of the
# power-law benchmark, FP64, default plan.
POWERLAW = {
    "name": "powerlaw-2.5e5",
    "workload": "Chung-Lu power-law graph, n=2.5e5, degree exponent 2.1, mean degree 40 (seed 7), "
                "x ~U[-1,1] (seed 3), FP64, default plan",
    "matgen": dict(n=250000, exponent=2.1, mean_deg=40, seed=7),
    "x_seed": 3,
}

# a batch of power-law graphs with hub rows: graph i draws, from generator
# seed 77, n ~ log-uniform [2e4, 2.5e5], degree exponent ~ U[2.1, 2.5] and
# mean degree ~ U[10, 40], and is generated with seed 900 + i
POWERLAW_BATCH = {"count": 12, "seed": 77, "n_lo": 2e4, "n_hi": 2.5e5, "graph_seed": 900}
# its FP32 plans for 8 right-hand sides (two workgroups per CU, no halo)
POWERLAW_BATCH_F32X8 = dict(n_rhs=8, lds_bytes=80 * 1024, halo_rows=0, rows_per_wave=64)


def powerlaw_batch():
    import numpy as np

    import matgen
    g = matgen.rng(POWERLAW_BATCH["seed"])
    out = []
    for i in range(POWERLAW_BATCH["count"]):
        n = int(np.exp(g.uniform(np.log(POWERLAW_BATCH["n_lo"]), np.log(POWERLAW_BATCH["n_hi"]))))
        out.append(matgen.powerlaw(n, exponent=float(g.uniform(2.1, 2.5)), mean_deg=float(g.uniform(10, 40)),
                                   seed=POWERLAW_BATCH["graph_seed"] + i))
    return out


# the batched product (64 uneven FP32 matrices x 8 right-hand sides): plans
# within half the LDS, so that two workgroups share a CU
BATCHED_PARAMS = dict(n_rhs=8, lds_bytes=80 * 1024, halo_rows=0, rows_per_wave=64)


def batched_tuned():
    """Plan parameters the batch autotuner chose (committed result), or None."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "batched_tuning.json")
    try:
        best = json.load(open(path))["best"]
    except (OSError, ValueError, KeyError):
        return None
    return dict(n_rhs=8, **best)
