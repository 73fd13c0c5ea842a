"""GPU parity of the batched path (many forests, one persistent launch in a
hipGraph) and of the autotuner: every forest's votes equal the CPU checker's
and its own single-forest prediction, bit for bit, on every graph replay."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1806_07300_amd as fp
import synth
from packed_format import decode

pytestmark = pytest.mark.gpu

CACHE = os.environ.get("FP_TEST_CACHE", "/tmp/forestpack_cache")

SMALL_SPECS = [  # (trees, features, classes, rows, max_depth, bin, depth, tune)
    (16, 4, 2, 1, 12, 16, 3, {}),
    (40, 30, 3, 17, 6, 8, 2, {"rows_per_block": 8}),
    (64, 100, 5, 1000, 12, 64, 4, {"rows_per_block": 32, "tree_groups": 1}),
    (33, 7, 2, 5000, -1, 16, 1, {"rows_per_block": 16, "tree_groups": 3}),
    (20, 12, 6, 0, 12, 20, 3, {}),
    (48, 60, 4, 2049, 10, 4, 5, {"rows_per_block": 64, "feature_lds": -1}),
    (1, 5, 2, 300, 8, 1, 0, {"rows_per_block": 1}),
    (57, 9, 10, 3000, 12, 19, 3, {"rows_per_block": 32, "tree_groups": 2, "lds_top_nodes": 40}),
    (70, 20, 3, 4000, -1, 70, 4, {"rows_per_block": 32, "layout": "compact"}),
    (30, 50, 7, 777, 12, 8, 2, {"rows_per_block": 16, "tree_groups": 2, "layout": "compact"}),
    (45, 16, 4, 2500, -1, 45, 0, {"rows_per_block": 32, "layout": "blocked"}),
    (26, 33, 9, 999, 14, 5, 3, {"rows_per_block": 8, "tree_groups": 3, "layout": "blocked"}),
    (37, 25, 6, 1800, -1, 37, 3, {"rows_per_block": 24, "layout": "clustered"}),
    (50, 18, 3, 2600, -1, 5, 3, {"rows_per_block": 32, "tree_passes": 4, "layout": "clustered"}),
    (29, 11, 4, 1500, 12, 4, 2, {"rows_per_block": 16, "tree_passes": 3, "tree_groups": 2}),
]


def make_job(i, spec):
    T, F, C, N, depth, B, D, tune = spec
    Xt, yt = synth.gaussian_mixture(3000, F, C, seed=500 + i)
    f = synth.train_forest(Xt, yt, n_trees=T, n_classes=C, mtry=max(1, int(np.sqrt(F))), max_depth=depth, seed=600 + i)
    X, _ = synth.gaussian_mixture(N, F, C, seed=700 + i)
    tune = dict(tune)
    layout = {"compact": fp.FP_LAYOUT_COMPACT, "blocked": fp.FP_LAYOUT_BLOCKED,
              "clustered": fp.FP_LAYOUT_CLUSTERED}.get(tune.pop("layout", None),
                                                                                fp.FP_LAYOUT_PACKED)
    p = fp.fp_pack_forest(f, layout=layout, bin_size=B, interleave_depth=D)
    fp.fp_packed_upload(p)
    if tune:
        fp.fp_packed_set_tune(p, tune)
    Xd = torch.from_numpy(X).cuda()
    votes = torch.full((N, C), -7, dtype=torch.int32, device="cuda")
    cls = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    return {"forest": f, "X": X, "packed": p, "Xd": Xd, "votes": votes, "cls": cls, "tune": tune}


@pytest.fixture(scope="module")
def small_jobs():
    jobs = [make_job(i, s) for i, s in enumerate(SMALL_SPECS)]
    for j in jobs:
        j["want"] = oracle.predict(j["forest"], j["X"])
    return jobs


def check_jobs(jobs, what):
    torch.cuda.synchronize()
    for i, j in enumerate(jobs):
        wv, wc = j["want"]
        gv, gc = j["votes"].cpu().numpy(), j["cls"].cpu().numpy()
        assert np.array_equal(gv, wv), f"{what}: job {i} votes differ"
        assert np.array_equal(gc, wc), f"{what}: job {i} classes differ"


@pytest.mark.parametrize("use_graph", [True, False])
@pytest.mark.parametrize("threads,cursors", [(512, 4), (256, 2), (1024, 1)])
def test_batched_small(small_jobs, use_graph, threads, cursors):
    plan = fp.fp_plan_create([(j["packed"], j["Xd"], j["votes"], j["cls"]) for j in small_jobs],
                             block_threads=threads, cursors=cursors, use_graph=use_graph)
    info = fp.fp_plan_info_get(plan)
    assert info["graph"] == int(use_graph) and info["n_jobs"] == len(small_jobs)
    for replay in range(3):
        # eager work between replays: scribble over every output
        for j in small_jobs:
            j["votes"].fill_(-1)
            j["cls"].fill_(-1)
        fp.fp_predict_batched(plan)
        check_jobs(small_jobs, f"graph={use_graph} replay {replay}")
        torch.cuda.synchronize()


def test_batched_equals_solo(small_jobs):
    for j in small_jobs:
        if j["X"].shape[0] == 0:
            continue
        v, c = fp.fp_predict(j["packed"], j["Xd"])
        torch.cuda.synchronize()
        assert np.array_equal(v.cpu().numpy(), j["want"][0])
        assert np.array_equal(c.cpu().numpy(), j["want"][1])


def test_autotune_small(small_jobs):
    j = small_jobs[2]
    res = fp.fp_autotune(j["forest"], j["Xd"], block_threads=512, cursors=4, sample_rows=1000)
    assert res["n_tried"] > 5 and res["best_ms"] > 0 and not res["cache_hit"]
    assert res["tune"]["block_threads"] == 512 and res["tune"]["cursors"] == 4
    again = fp.fp_autotune(j["forest"], j["Xd"], block_threads=512, cursors=4, sample_rows=1000)
    assert again["cache_hit"] and again["pack"] == res["pack"]
    p = fp.fp_pack_forest(j["forest"], **res["pack"])
    fp.fp_packed_upload(p)
    v, c = fp.fp_predict_tuned(p, res["tune"], j["Xd"])
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy(), j["want"][0]) and np.array_equal(c.cpu().numpy(), j["want"][1])


@pytest.mark.parametrize("threads,cursors", [(1024, 2), (512, 4)])
def test_batched_fp16_tile(threads, cursors):
    """Batched launches that walk the CLUSTERED 48-byte form over an fp16 row
    tile (rounded toward +infinity) beside the same forest on an fp32 tile
    and a 64-byte clustered forest: every job equals the checker, with rows
    on thresholds, halfway to their fp16 neighbours and non-finite values."""
    w = synth.image(n_train=6000, n_trees=16)
    f = w.forest()
    X, _ = w.predict_rows(3001)
    X = X.copy()
    rng = np.random.default_rng(31)
    thr = f.threshold[f.feature >= 0].astype(np.float16)
    m = rng.random(X.shape)
    sel = m < 0.2
    t = rng.choice(thr, size=sel.sum())
    with np.errstate(over="ignore"):
        up = np.nextafter(t, np.float16(np.inf)).astype(np.float64)
    X[sel] = ((t.astype(np.float64) + up) / 2).astype(np.float32)  # nearest-even would land on t or up
    X[(m >= 0.2) & (m < 0.22)] = np.nan
    X[(m >= 0.22) & (m < 0.24)] = np.float32(1e-40)
    X[(m >= 0.24) & (m < 0.26)] = np.float32(7e4)
    want = oracle.predict(f, X)
    Xg, yg = synth.gaussian_mixture(4000, 12, 3, seed=77)
    g = synth.train_forest(Xg, yg, n_trees=20, n_classes=3, mtry=3, max_depth=12, seed=78)
    Xq, _ = synth.gaussian_mixture(2500, 12, 3, seed=79)
    jobs = []
    for forest, rows, tune in ((f, X, {"rows_per_block": 40}), (f, X, {"rows_per_block": 16, "feature_lds": 2}),
                               (g, Xq, {"rows_per_block": 32})):
        p = fp.fp_pack_forest(forest, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=8, interleave_depth=3)
        fp.fp_packed_upload(p)
        fp.fp_packed_set_tune(p, tune)
        C = forest.n_classes
        jobs.append({"packed": p, "Xd": torch.from_numpy(rows).cuda(),
                     "votes": torch.full((len(rows), C), -7, dtype=torch.int32, device="cuda"),
                     "cls": torch.full((len(rows),), -7, dtype=torch.int32, device="cuda"),
                     "want": want if forest is f else oracle.predict(g, Xq)})
    assert decode(fp.fp_packed_host_bytes(jobs[0]["packed"]))["h"]["block_bytes"] == 48
    assert decode(fp.fp_packed_host_bytes(jobs[2]["packed"]))["h"]["block_bytes"] == 64
    plan = fp.fp_plan_create([(j["packed"], j["Xd"], j["votes"], j["cls"]) for j in jobs],
                             block_threads=threads, cursors=cursors)
    for replay in range(2):
        for j in jobs:
            j["votes"].fill_(-1)
            j["cls"].fill_(-1)
        fp.fp_predict_batched(plan)
        check_jobs(jobs, f"fp16 tile, {threads} x {cursors}, replay {replay}")


@pytest.mark.timeout(900)  # trains 64 forests on the host first (about a minute on 16 threads)
def test_batched_workload_64_forests(say):
    """The 64-forest workload (16-2048 trees, 4-784 features, 2-10 classes,
    1-200,000 rows each), every forest autotuned, one persistent graph launch.
    Every row of every forest equals the checker on two graph replays, and
    its single-forest prediction and the naive layout exactly."""
    threads, cursors = 1024, 2
    jobs = []
    for i in range(64):
        w = synth.batched_workload(i)
        f = w.forest(cache_dir=CACHE)
        X, _ = w.predict_rows()
        Xd = torch.from_numpy(X).cuda()
        res = fp.fp_autotune(f, Xd, block_threads=threads, cursors=cursors, sample_rows=16384)
        if i % 4 == 3:
            say(f"[batched] {i + 1} forests trained and tuned")
        p = fp.fp_pack_forest(f, **res["pack"])
        fp.fp_packed_upload(p)
        fp.fp_packed_set_tune(p, res["tune"])
        votes = torch.full((len(X), f.n_classes), -7, dtype=torch.int32, device="cuda")
        cls = torch.full((len(X),), -7, dtype=torch.int32, device="cuda")
        jobs.append({"forest": f, "X": X, "Xd": Xd, "packed": p, "votes": votes, "cls": cls})
    plan = fp.fp_plan_create([(j["packed"], j["Xd"], j["votes"], j["cls"]) for j in jobs],
                             block_threads=threads, cursors=cursors)
    # timing for the record: the graph replay vs every forest's naive-layout launch in turn
    rows = sum(len(j["X"]) for j in jobs)
    fp.fp_predict_batched(plan)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(5):
        fp.fp_predict_batched(plan)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / 5
    naive = [fp.fp_pack_forest(j["forest"], layout=fp.FP_LAYOUT_NAIVE) for j in jobs]
    for q in naive:
        fp.fp_packed_upload(q)
    nv = [torch.empty_like(j["votes"]) for j in jobs]
    nc = [torch.empty_like(j["cls"]) for j in jobs]
    run_naive = lambda: [fp.fp_predict_tuned(q, {"block_threads": 256}, j["Xd"], v, c)
                         for q, j, v, c in zip(naive, jobs, nv, nc)]
    run_naive()
    torch.cuda.synchronize()
    t0.record()
    run_naive()
    t1.record()
    torch.cuda.synchronize()
    ms_naive = t0.elapsed_time(t1)
    layouts = [fp.fp_packed_info_get(j["packed"])["layout"] for j in jobs]
    say(f"\n[batched] 64 forests, {rows} rows: one graph launch {ms:.3f} ms = {rows / ms / 1e3:.2f} M obs/s; "
          f"naive layout, 64 launches {ms_naive:.3f} ms = {rows / ms_naive / 1e3:.2f} M obs/s "
        f"({ms_naive / ms:.2f}x); layouts chosen {np.bincount(layouts, minlength=5).tolist()}")
    for i, j in enumerate(jobs):
        if len(j["X"]):
            assert torch.equal(nv[i], j["votes"]), f"forest {i}: naive votes differ"
    want = [oracle.predict(j["forest"], j["X"]) for j in jobs]  # every row of every forest
    say(f"[batched] checker done for {rows} rows")
    for replay in range(2):
        for j in jobs:
            j["votes"].fill_(-1)
            j["cls"].fill_(-1)
        fp.fp_predict_batched(plan)
        torch.cuda.synchronize()
        for i, j in enumerate(jobs):
            f = j["forest"]
            gv, gc = j["votes"].cpu().numpy(), j["cls"].cpu().numpy()
            assert (gv.sum(1) == f.n_trees).all(), f"forest {i}: votes do not sum to T"
            wv, wc = want[i]
            assert np.array_equal(gv, wv) and np.array_equal(gc, wc), f"forest {i} vs checker, replay {replay}"
            if replay == 0:
                sv, sc = fp.fp_predict(j["packed"], j["Xd"])
                torch.cuda.synchronize()
                assert np.array_equal(sv.cpu().numpy(), gv) and np.array_equal(sc.cpu().numpy(), gc), f"forest {i} solo"
