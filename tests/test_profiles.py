"""The committed HBM-traffic summaries (profiles/traffic_<name>.json) against the sources and the arithmetic they
state: each was taken on the kernel's current sources (so the bench reports it), and its byte counts follow from
its counters, its calibration and the workload's node count."""
import json
import os

import pytest

import bench
from paper_1501_05430_amd import workloads as W


@pytest.mark.parametrize("name", sorted(bench.TRAFFIC_SPECS))
def test_traffic_summary_is_current_and_consistent(name):
    spec = bench.TRAFFIC_SPECS[name]
    path = os.path.join(bench.ROOT, "profiles", f"traffic_{name}.json")
    with open(path) as f:
        tr = json.load(f)
    sources = {"adjoint": bench.ADJOINT_SRC, "step": bench.STEP1_SRC}.get(spec.get("sources"), bench.KERNEL_SRC)
    assert tr["kernel_source_sha256"] == bench.kernel_sha(sources), "kernel changed since its counters were taken"
    assert bench.profile_traffic(path, sources)[0] == tr["hbm_bytes_per_launch"]
    kib = tr["kernel_counters_kib_per_launch"]
    cal = tr["calibration"]
    rd = kib["FETCH_SIZE"] * 1024 * cal["fetch_scale"]
    wr = kib["WRITE_SIZE"] * 1024 * cal["write_scale"]
    # the stored counters are rounded to 0.1 KiB
    assert abs(rd - tr["hbm_read_bytes_per_launch"]) <= 0.06 * 1024 * cal["fetch_scale"]
    assert abs(wr - tr["hbm_write_bytes_per_launch"]) <= 0.06 * 1024 * cal["write_scale"]
    # each of the three truncated to whole bytes on its own
    assert abs(tr["hbm_bytes_per_launch"] - tr["hbm_read_bytes_per_launch"] - tr["hbm_write_bytes_per_launch"]) <= 1
    nodes = W.c3_large().fluid_nodes if spec["workload"] == "c3" else sum(c.fluid_nodes for c in W.c4_batch())
    steps = spec.get("steps", 2)
    assert tr["time_steps_per_launch"] == steps
    assert tr["algorithmic_bytes_per_launch"] == steps * spec.get("bytes_per_update", 72) * nodes
    assert tr["traffic_over_algorithmic"] == pytest.approx(
        tr["hbm_bytes_per_launch"] / tr["algorithmic_bytes_per_launch"], abs=1e-4)
    # a copy of known size reads each byte once on FETCH_SIZE x scale and writes it once on WRITE_SIZE x scale
    assert 1.9 < cal["fetch_scale"] < 2.1 and 0.95 < cal["write_scale"] < 1.05
