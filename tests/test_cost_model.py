"""The EU run-time estimate of Sec. III-A (Eqs. 1-2) as bench.py --ladder uses it.

Pins from the paper's text: a line is used at least once (EU = 1 with no
bias), at most four times (two nodes per line plus the prefetched adjacent
line: EU = 4 at bias 1), and the DF layout's bias of one half gives 1.875
(printed as 1.85 in the paper; reading Q17).  The estimate reproduces the
BF time for BF itself, and removing fetches or raising EU lowers it.
"""
import pytest

import bench


def test_eu_closed_forms():
    assert bench.eu_stat(0.0) == 1.0
    assert bench.eu_stat(0.5) == 1.875
    assert bench.eu_stat(1.0) == 4.0
    xs = [0.5 + 0.05 * i for i in range(11)]
    assert all(bench.eu_stat(a) < bench.eu_stat(b) for a, b in zip(xs, xs[1:]))


def test_eu_model_rungs():
    info = {"expected_fetches": 11.0, "expected_depth": 10.0, "mean_bias": 0.75}
    assert bench.eu_model("BF", info, 0) == (11.0, 0.0, 1.0)
    assert bench.eu_model("DF", info, 0) == (11.0, 0.0, 1.875)
    f, wun, eu = bench.eu_model("Stat", dict(info, expected_fetches=10.0), 0)
    assert (f, wun) == (10.0, 0.0) and eu == pytest.approx(1 + 0.75 * (1 + 0.75 * 1.75))
    assert bench.eu_model("Bin", dict(info, expected_fetches=10.0), 3)[1] == 4.0  # levels 0..3 stay near
    assert bench.eu_model("Bin", dict(info, expected_fetches=2.0, expected_depth=2.0), 3)[1] == 2.0
    assert bench.eu_model("CLUSTERED", dict(info, expected_fetches=2.4), 3) == (2.4, 0.0, 1.0)
