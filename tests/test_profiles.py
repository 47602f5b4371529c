"""The committed rocprofv3 evidence: HBM traffic measured by the FETCH_SIZE
and WRITE_SIZE counters against the algorithmic bytes of the same launch
(no wasted re-reads on the headline kernel; the batched kernel's halo
re-reads stay bounded)."""
import json
import os

import pytest

PROFILES = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles")


@pytest.mark.parametrize("name,limit", [("ehyb_spmv_f64_stencil27_traffic.json", 1.10),
                                        ("ehyb_spmm_batched_f32x8_64mat_traffic.json", 1.30)])
def test_measured_traffic_close_to_algorithmic(name, limit):
    d = json.load(open(os.path.join(PROFILES, name)))
    ratio = d["bytes_per_launch"] / d["algorithmic_bytes"]
    assert 0.95 <= ratio <= limit, ratio
    assert d["fetch_bytes"] + d["write_bytes"] == pytest.approx(d["bytes_per_launch"], abs=2)
    # the copy probe that scales the counters moved a known number of bytes
    assert 1.9 <= d["fetch_scale"] <= 2.1 and 0.95 <= d["write_scale"] <= 1.05
