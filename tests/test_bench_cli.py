"""bench.py on the CPU: the one-GPU contract, its error helpers against the
oracle, and its reading of the committed traffic evidence."""
import os
import subprocess
import sys

import numpy as np

import bench
import matgen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_error_helpers_match_the_oracle():
    A = matgen.random_small(400, 0.02, 3, empty_rows=40, dense_row=True, explicit_zeros=10, negative_zero=True)
    x = matgen.uniform_vector(400, 8)
    y, s = bench.fp64_products(A.row_ptr, A.col, A.val, x)
    assert np.allclose(y, oracle.spmv(A, x), rtol=0, atol=1e-12 * max(1.0, float(s.max())))
    assert np.allclose(s, oracle.abs_scale(A, x), rtol=1e-14, atol=0)
    X = np.stack([x, 2 * x, -x], axis=1)
    Y, _ = bench.fp64_products(A.row_ptr, A.col, A.val, X)
    assert np.allclose(Y, oracle.spmm(A, X), rtol=0, atol=1e-11)
    e = bench.scaled_error(np.array([0.0, 1.0, 3.0, 1.0]), np.array([0.0, 1.0, 1.0, 0.0]),
                           np.array([0.0, 0.0, 4.0, 0.0]))
    assert e[0] == 0 and e[1] == 0 and e[2] == 0.5 and np.isinf(e[3])


def test_traffic_evidence_is_for_the_current_kernel_source():
    """The committed FETCH_SIZE / WRITE_SIZE figures were taken on the kernel
    source as it stands; bench.py reports them only then."""
    h = bench.kernel_source_hash()
    for name in ("ehyb_spmv_f64_stencil27_traffic.json", "ehyb_spmm_batched_f32x8_64mat_traffic.json",
                 "ehyb_spmm_batched_f32x8_powerlaw12_traffic.json",
                 "ehyb_spmv_f64_powerlaw250k_traffic.json", "ehyb_spmv_f64_knnfem_traffic.json",
                 "ehyb_spmv_f32_knnfem_traffic.json", "ehyb_spmv_bf16_knnfem_traffic.json"):
        t = bench.load_traffic(h, name)
        assert t is not None, f"{name}: taken on another kernel source"
    assert bench.load_traffic("0" * 16) is None
