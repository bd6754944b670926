"""Host logic of bench.py (no GPU needed): the HBM traffic it reports next to
the roofline comes from the committed counter summary only for the workload,
batch and kernel sources it was counted on."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_only_for_the_counted_workload_and_batch():
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    wl, B = d["workload_id"], d["global_batch"]
    for k, v in d["kernels"].items():
        got = bench.traffic_for(k, wl, B)
        if d["source_hash"] == bench.kernel_source_hash():
            assert got == v["bytes_per_launch"]
        else:
            assert got is None
        assert bench.traffic_for(k, wl, B + 1) is None
        assert bench.traffic_for(k, "mlp784-1024x4-10", B) is None
    assert bench.traffic_for("no_such_kernel", wl, B) is None

