"""The committed rocprofv3 evidence: HBM traffic counted request by request
(TCC_EA0_RDREQ_32B/64B/128B, TCC_EA0_WRREQ / _64B) against the algorithmic
bytes of the same launch.  The request count must reproduce the copy probe's
known bytes, and FETCH_SIZE / WRITE_SIZE scaled by the same probe must agree
with it."""
import json
import os

import pytest

PROFILES = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles")


@pytest.mark.parametrize("name,limit", [("ehyb_spmv_f64_stencil27_traffic.json", 1.10),
                                        ("ehyb_spmm_batched_f32x8_64mat_traffic.json", 1.10),
                                        ("ehyb_spmm_batched_f32x8_powerlaw12_traffic.json", 2.30),
                                        ("ehyb_spmv_f64_powerlaw250k_traffic.json", 1.35),
                                        ("ehyb_spmv_f64_knnfem_traffic.json", 1.05),
                                        ("ehyb_spmv_f32_knnfem_traffic.json", 1.05),
                                        ("ehyb_spmv_bf16_knnfem_traffic.json", 1.05)])
def test_measured_traffic_close_to_algorithmic(name, limit):
    d = json.load(open(os.path.join(PROFILES, name)))
    ratio = d["bytes_per_launch"] / d["algorithmic_bytes"]
    assert 0.95 <= ratio <= limit, ratio
    assert d["read_bytes"] + d["write_bytes"] == pytest.approx(d["bytes_per_launch"], abs=2)
    rq = d["read_requests"]
    assert d["read_bytes"] == pytest.approx(32 * rq["32"] + 64 * rq["64"] + 128 * rq["128"], rel=1e-6)
    assert rq["32"] + rq["64"] + rq["128"] == pytest.approx(d["read_requests_total"], rel=1e-3)
    # the request count reproduces the copy probe's bytes
    c = d["copy_check"]
    assert c["read_bytes_counted"] == pytest.approx(c["bytes_read"], rel=0.01)
    assert c["write_bytes_counted"] == pytest.approx(c["bytes_written"], rel=0.01)
    # and the copy-scaled FETCH_SIZE / WRITE_SIZE agree with it
    f = d["fetch_size_cross_check"]
    assert f["bytes_per_launch"] == pytest.approx(d["bytes_per_launch"], rel=0.02)


@pytest.mark.parametrize("name", ["ehyb_spmv_f64_stencil27_traffic.json", "ehyb_spmm_batched_f32x8_64mat_traffic.json",
                                  "ehyb_spmm_batched_f32x8_powerlaw12_traffic.json",
                                  "ehyb_spmv_f64_powerlaw250k_traffic.json", "ehyb_spmv_f64_knnfem_traffic.json",
                                  "ehyb_spmv_f32_knnfem_traffic.json", "ehyb_spmv_bf16_knnfem_traffic.json"])
def test_lds_counters_recorded(name):
    d = json.load(open(os.path.join(PROFILES, name)))
    lds = d["lds"]
    assert lds["SQ_WAVES"] > 0 and lds["SQ_INSTS_LDS"] > 0
    assert 0 <= lds["SQ_LDS_BANK_CONFLICT"] <= lds["SQ_LDS_IDX_ACTIVE"]
