"""The full-size tabular workload on the GPU: 28 features, 1,024 trees grown
to pure leaves on 1,000,000 rows, 10,000,000 rows predicted, bins of 16 trees.

The CLUSTERED layout runs in the launch configuration the benchmark times
(presets.TABULAR); PACKED and BLOCKED run beside it.  Every layout must equal
the naive layout on all 10,000,000 rows, and the first 1,000,000 rows plus a
spread sample must equal the CPU checker bit for bit.  Training the forest
takes minutes of host CPU (progress is printed every 64 trees); the forest is
cached under FP_TEST_CACHE for later runs in the same machine session."""
import os
import time

import numpy as np
import pytest
import torch

import oracle
import paper_1806_07300_amd as fp
from paper_1806_07300_amd import presets
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

CACHE = os.environ.get("FP_TEST_CACHE", "/tmp/forestpack_cache")
ORACLE_ROWS = 1_000_000


class Progress:
    chunk = 64

    def __init__(self, say):
        self.say = say

    def __call__(self, done, total):
        self.say(f"[tabular] trained {done}/{total} trees")


def oracle_by_tree_chunks(forest, X, say, trees_per_chunk=8):
    """The checker's votes for a large forest, computed on consecutive groups
    of trees and added up: a forest's votes are the sum over its trees of one
    vote each, so splitting the trees into groups and summing the groups'
    integer votes is the same definition (each group's forest fits the host's
    caches, which keeps the checker's walks fast).  Classes: argmax, lowest
    index on ties (numpy's argmax returns the first maximum)."""
    votes = np.zeros((len(X), forest.n_classes), np.int32)
    for t0 in range(0, forest.n_trees, trees_per_chunk):
        sub = forest.subset(range(t0, min(forest.n_trees, t0 + trees_per_chunk)))
        v, _ = oracle.predict(sub, X)
        votes += v
        if (t0 // trees_per_chunk) % 16 == 15:
            say(f"[tabular] checker: {t0 + trees_per_chunk}/{forest.n_trees} trees")
    return votes, np.argmax(votes, axis=1).astype(np.int32)


@pytest.mark.timeout(900)
def test_tabular_full_size(say):
    w = synth.tabular()
    t0 = time.time()
    f = w.forest(cache_dir=CACHE, progress=Progress(say))
    say(f"[tabular] forest: {f.n_internal() / f.n_trees:.0f} internal nodes/tree, max depth {int(f.depth.max())}, "
          f"{time.time() - t0:.0f} s")
    X, _ = w.predict_rows()
    Xd = torch.from_numpy(X).cuda()
    n = len(X)
    out = {}
    runs = (("clustered", presets.TABULAR["pack"], presets.TABULAR["tune"]),
            ("packed", {"bin_size": 16, "interleave_depth": 3},
             {"rows_per_block": 256, "cursors": 1, "block_threads": 1024, "tree_passes": 64}),
            ("blocked", {"layout": fp.FP_LAYOUT_BLOCKED, "bin_size": 16, "interleave_depth": 3},
             {"rows_per_block": 256, "cursors": 1, "block_threads": 1024, "refill_lanes": 32}),
            ("naive", {"layout": fp.FP_LAYOUT_NAIVE}, presets.TABULAR["naive_tune"]))
    for name, kw, tune in runs:
        t0 = time.time()
        p = fp.fp_pack_forest(f, **kw)
        pack_s = time.time() - t0
        fp.fp_packed_upload(p)
        votes = torch.full((n, 2), -1, dtype=torch.int32, device="cuda")
        cls = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        say(f"[tabular] {name}: packed in {pack_s:.1f} s, launching {tune}")
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        fp.fp_predict_tuned(p, tune, Xd, votes, cls)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e)
        say(f"[tabular] {name}: {ms:.1f} ms per 10M rows = {n / ms / 1e3:.2f} M obs/s "
            f"({fp.fp_packed_info_get(p)['bytes'] / 2**30:.2f} GiB)")
        out[name] = (votes.cpu().numpy(), cls.cpu().numpy())
        del p
    v, c = out["clustered"]
    assert (v.sum(1) == f.n_trees).all()
    for name in ("clustered", "packed", "blocked"):
        assert np.array_equal(out[name][0], out["naive"][0]) and np.array_equal(out[name][1], out["naive"][1]), name
    # the checker: the first 1,000,000 rows, and 4,096 rows spread over the rest
    t0 = time.time()
    wv, wc = oracle_by_tree_chunks(f, X[:ORACLE_ROWS], say)
    assert np.array_equal(v[:ORACLE_ROWS], wv) and np.array_equal(c[:ORACLE_ROWS], wc)
    rows = np.unique(np.concatenate([[n - 1], np.random.default_rng(11).integers(ORACLE_ROWS, n, 4096)]))
    wv, wc = oracle.predict(f, X[rows])
    assert np.array_equal(v[rows], wv) and np.array_equal(c[rows], wc)
    say(f"[tabular] {ORACLE_ROWS + len(rows)} rows equal the checker ({time.time() - t0:.0f} s)")
