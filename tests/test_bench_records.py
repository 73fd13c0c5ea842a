"""The counter records under profiles/ that the bench line's roofline reads:
each parses, names the launch the bench times for its workload, and is
ignored (traffic None) for any other launch or kernel source."""
import json
import os

import pytest

import bench
from paper_1806_07300_amd import presets

PRESETS = {"tabular": presets.TABULAR, "image": presets.IMAGE}


def parse(path):
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    return vals


@pytest.mark.parametrize("workload", sorted(PRESETS))
def test_record_fields(workload):
    vals = parse(bench.traffic_file(workload))
    assert len(vals["kernel_source_sha256"]) == 16
    assert json.loads(vals["launch"]) == PRESETS[workload]["tune"]
    steps = int(vals["launches_per_step"])
    assert steps == max(1, PRESETS[workload]["tune"].get("tree_passes", 1))
    fetch, write = float(vals["fetch_bytes_per_step"]), float(vals["write_bytes_per_step"])
    # FETCH_SIZE x2.0 and WRITE_SIZE x1.0 copy calibration, KiB per dispatch
    assert fetch == pytest.approx(float(vals["fetch_kib_per_dispatch"]) * 1024 * 2.0 * steps, rel=1e-5)
    assert write == pytest.approx(float(vals["write_kib_per_dispatch"]) * 1024 * steps, rel=1e-5)
    assert 0.0 < float(vals["l2_hit_rate"]) < 1.0


@pytest.mark.parametrize("workload", sorted(PRESETS))
def test_record_applies_only_to_its_launch(workload):
    tune = PRESETS[workload]["tune"]
    vals = parse(bench.traffic_file(workload))
    current = vals["kernel_source_sha256"] == bench.kernel_source_hash()
    got = bench.read_traffic(workload, tune)
    if current:
        assert got == pytest.approx(float(vals["fetch_bytes_per_step"]) + float(vals["write_bytes_per_step"]))
    else:  # taken on another kernel source: the bench reports no traffic
        assert got is None
    other = dict(tune, rows_per_block=tune["rows_per_block"] + 1)
    assert bench.read_traffic(workload, other) is None
