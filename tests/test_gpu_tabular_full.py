"""The full-size tabular workload (28 features, 1,024 trees grown on 1,000,000
rows, 10,000,000 rows predicted, bins of 16 trees, PACKED, BLOCKED and CLUSTERED layouts)
on the GPU, checked against the CPU checker on sampled rows and against the
naive layout on every row.  Training the forest takes minutes of host CPU, so the test runs only
with FP_FULL_TABULAR=1 (it prints training progress)."""
import os
import time

import numpy as np
import pytest
import torch

import oracle
import paper_1806_07300_amd as fp
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


class Progress:
    chunk = 64

    def __call__(self, done, total):
        print(f"[tabular] trained {done}/{total} trees", flush=True)


@pytest.mark.skipif(os.environ.get("FP_FULL_TABULAR") != "1", reason="set FP_FULL_TABULAR=1 (trains 1,024 trees on 1M rows)")
def test_tabular_full_size():
    w = synth.tabular()
    t0 = time.time()
    f = w.forest(progress=Progress())
    print(f"[tabular] forest: {f.n_internal() / f.n_trees:.0f} internal nodes/tree, max depth {int(f.depth.max())}, "
          f"{time.time() - t0:.0f} s", flush=True)
    X, _ = w.predict_rows()
    Xd = torch.from_numpy(X).cuda()
    n = len(X)
    out = {}
    runs = (("packed", {"bin_size": 16, "interleave_depth": 3},
             {"rows_per_block": 32, "cursors": 4, "block_threads": 1024}),
            ("blocked", {"layout": fp.FP_LAYOUT_BLOCKED, "bin_size": 16, "interleave_depth": 3},
             {"rows_per_block": 256, "cursors": 1, "block_threads": 1024, "refill_lanes": 32}),
            ("clustered", {"layout": fp.FP_LAYOUT_CLUSTERED, "bin_size": 16, "interleave_depth": 3},
             {"rows_per_block": 512, "cursors": 1, "block_threads": 1024, "refill_lanes": 32}),
            ("naive", {"layout": fp.FP_LAYOUT_NAIVE}, {"block_threads": 256}))
    for name, kw, tune in runs:
        p = fp.fp_pack_forest(f, **kw)
        fp.fp_packed_upload(p)
        votes = torch.empty((n, 2), dtype=torch.int32, device="cuda")
        cls = torch.empty((n,), dtype=torch.int32, device="cuda")
        fp.fp_predict_tuned(p, tune, Xd, votes, cls)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        fp.fp_predict_tuned(p, tune, Xd, votes, cls)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e)
        print(f"[tabular] {name}: {ms:.1f} ms per 10M rows = {n / ms / 1e3:.2f} M obs/s "
              f"({fp.fp_packed_info_get(p)['bytes'] / 2**30:.2f} GiB)", flush=True)
        out[name] = (votes.cpu().numpy(), cls.cpu().numpy())
        del p
    v, c = out["packed"]
    assert (v.sum(1) == f.n_trees).all()
    for name in ("packed", "blocked", "clustered"):
        assert np.array_equal(out[name][0], out["naive"][0]) and np.array_equal(out[name][1], out["naive"][1]), name
    rows = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(11).integers(0, n, 10_000)]))
    wv, wc = oracle.predict(f, X[rows])
    assert np.array_equal(v[rows], wv) and np.array_equal(c[rows], wc)
    print(f"[tabular] {len(rows)} sampled rows equal the checker", flush=True)
