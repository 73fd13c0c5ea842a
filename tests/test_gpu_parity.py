"""GPU parity: every layout and launch configuration returns exactly the CPU
checker's int32 votes and classes (bit-exact), through the C ABI.

Sizes: the checker finishes each case in well under a second; cases span many
row tiles and bins with ragged tails.  The full image-shaped workload (1M rows,
128 trees) is checked on sampled rows in the launch configuration the
benchmark times.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1806_07300_amd as fp
from paper_1806_07300_amd import presets
import synth
from packed_format import decode

pytestmark = pytest.mark.gpu


def run(p, X, tune=None, ld_pad=0):
    n, F = X.shape
    if ld_pad:
        Xp = np.full((n, F + ld_pad), np.nan, np.float32)
        Xp[:, :F] = X
        Xd = torch.from_numpy(Xp).cuda()
    else:
        Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    if tune is None:
        v, c = fp.fp_predict(p, Xd)
    else:
        v, c = fp.fp_predict_tuned(p, tune, Xd)
    torch.cuda.synchronize()
    return v.cpu().numpy(), c.cpu().numpy()


def upload(forest, **kw):
    p = fp.fp_pack_forest(forest, **kw)
    fp.fp_packed_upload(p)
    return p


def assert_same(got, want, what=""):
    gv, gc = got
    wv, wc = want
    if not np.array_equal(gv, wv):
        bad = np.nonzero((gv != wv).any(1))[0]
        raise AssertionError(f"{what}: {len(bad)} rows differ, first {bad[:5]}: {gv[bad[0]]} vs {wv[bad[0]]}")
    assert np.array_equal(gc, wc), f"{what}: classes differ"


@pytest.fixture(scope="module")
def small():
    w = synth.small()
    f = w.forest()
    X, _ = w.predict_rows()
    return f, X, oracle.predict(f, X)


def test_naive_small(small):
    f, X, want = small
    p = upload(f, layout=fp.FP_LAYOUT_NAIVE)
    for threads in (64, 256, 1024):
        assert_same(run(p, X, {"block_threads": threads}), want, f"naive threads={threads}")


@pytest.mark.parametrize("B", [1, 2, 16, 32])
@pytest.mark.parametrize("D", [0, 1, 3, 6])
def test_packed_layout_grid(small, B, D):
    f, X, want = small
    p = upload(f, bin_size=B, interleave_depth=D, line_align=int(B % 2 == 0))
    assert_same(run(p, X), want, f"B={B} D={D}")


TUNES = [
    {"rows_per_block": 1, "cursors": 1, "block_threads": 64},
    {"rows_per_block": 4, "cursors": 8, "block_threads": 256},
    {"rows_per_block": 16, "cursors": 2, "tree_groups": 2},
    {"rows_per_block": 64, "cursors": 4, "tree_groups": 4, "block_threads": 1024},
    {"rows_per_block": 16, "cursors": 4, "feature_lds": -1},
    {"rows_per_block": 32, "cursors": 2, "lds_top_nodes": -1},
    {"rows_per_block": 8, "cursors": 1, "lds_top_nodes": 5, "tree_groups": 3},
    {"rows_per_block": 16, "cursors": 8, "feature_lds": 1, "block_threads": 512},
    {"rows_per_block": 128, "cursors": 2, "block_threads": 1024},
    {"rows_per_block": 3, "cursors": 4, "tree_groups": 8, "block_threads": 64},
    {"rows_per_block": 33, "cursors": 1, "lds_top_nodes": 100, "block_threads": 128},
    {"rows_per_block": 16, "cursors": 2, "tree_passes": 3},
    {"rows_per_block": 40, "cursors": 1, "tree_passes": 4, "block_threads": 1024},
    {"rows_per_block": 8, "cursors": 4, "tree_passes": 2, "tree_groups": 2},
    {"rows_per_block": 24, "cursors": 1, "tree_passes": 9, "lds_top_nodes": -1},
    # one workgroup per CU with the CU's whole LDS (the large-forest launch shape)
    {"rows_per_block": 768, "cursors": 1, "block_threads": 1024, "refill_lanes": 24, "feature_lds": 1,
     "tree_passes": 3, "lds_bytes": 163840},
    {"rows_per_block": 200, "cursors": 2, "block_threads": 1024, "lds_bytes": 163840, "tree_groups": 2},
]


@pytest.mark.parametrize("layout", [fp.FP_LAYOUT_PACKED, fp.FP_LAYOUT_COMPACT, fp.FP_LAYOUT_BLOCKED,
                                    fp.FP_LAYOUT_CLUSTERED])
@pytest.mark.parametrize("tune", TUNES, ids=lambda t: "-".join(f"{k[:4]}{v}" for k, v in t.items()))
def test_packed_launch_grid(small, tune, layout):
    f, X, want = small
    p = upload(f, layout=layout, bin_size=8, interleave_depth=3)
    assert_same(run(p, X, tune), want, f"layout {layout} {tune}")


@pytest.mark.parametrize("layout", [fp.FP_LAYOUT_COMPACT, fp.FP_LAYOUT_BLOCKED, fp.FP_LAYOUT_CLUSTERED])
@pytest.mark.parametrize("B", [1, 7, 32])
@pytest.mark.parametrize("D", [0, 2, 5])
def test_compact_layout_grid(small, B, D, layout):
    f, X, want = small
    p = upload(f, layout=layout, bin_size=B, interleave_depth=D)
    for K in (1, 2, 4, 8):
        assert_same(run(p, X, {"cursors": K, "rows_per_block": 16, "block_threads": 512}), want,
                    f"layout={layout} B={B} D={D} K={K}")


def test_ablation_orders(small):
    """The DF layout (NAIVE, depth-first, leaves stored) on the naive kernel and
    DF- (PACKED without Stat) on the packed kernel, one and four walks per
    lane, against the checker."""
    f, X, want = small
    p = upload(f, layout=fp.FP_LAYOUT_NAIVE, node_order=fp.FP_ORDER_DF)
    assert_same(run(p, X, {"block_threads": 256}), want, "DF")
    for B, D in ((1, 0), (16, 3)):
        p = upload(f, bin_size=B, interleave_depth=D, node_order=fp.FP_ORDER_DF)
        for K in (1, 4):
            assert_same(run(p, X, {"cursors": K, "rows_per_block": 32, "block_threads": 1024}), want,
                        f"DF- B={B} D={D} K={K}")


def test_infer_cardinality_matches_training_counts():
    """Trees grown without bootstrap: walking the training rows on the GPU
    gives back exactly the training cardinality of every node, and packing
    with the inferred statistics gives the same bytes."""
    X, y = synth.gaussian_mixture(6000, 10, 3, seed=41)
    f = synth.train_forest(X, y, n_trees=7, n_classes=3, mtry=3, max_depth=14, bootstrap=False, seed=42)
    card = fp.fp_infer_cardinality(f, torch.from_numpy(X).cuda())
    for t in range(f.n_trees):
        assert card[f.tree_node_offset[t]] == len(X)
    assert np.array_equal(card, f.cardinality)
    g = f.subset(range(f.n_trees))
    g.cardinality = card
    for kw in ({"bin_size": 3, "interleave_depth": 2}, {"layout": fp.FP_LAYOUT_CLUSTERED, "bin_size": 3}):
        assert np.array_equal(fp.fp_packed_host_bytes(fp.fp_pack_forest(f, **kw)),
                              fp.fp_packed_host_bytes(fp.fp_pack_forest(g, **kw)))


def test_infer_cardinality_invariants(small):
    """Bootstrap forest, unseen rows (padded leading dimension): each tree's
    root count is the row count, internal counts are sums of their children,
    internal counts add up to the checker's node visits, and the leaf counts
    per class add up to the checker's votes."""
    f, X, want = small
    n = 5000
    Xp = np.full((n, X.shape[1] + 3), np.nan, np.float32)
    Xp[:, :X.shape[1]] = X[:n]
    card = fp.fp_infer_cardinality(f, torch.from_numpy(Xp).cuda())
    votes, _, visits = oracle.predict(f, X[:n], return_visits=True)
    internal = f.feature >= 0
    assert card[internal].sum() == visits
    per_class = np.bincount(f.leaf_class[~internal], weights=card[~internal], minlength=f.n_classes)
    assert np.array_equal(per_class.astype(np.int64), votes.sum(0))
    for t in range(f.n_trees):
        o, e = f.tree_node_offset[t], f.tree_node_offset[t + 1]
        assert card[o] == n
        for i in np.nonzero(f.feature[o:e] >= 0)[0]:
            assert card[o + i] == card[o + f.left[o + i]] + card[o + f.right[o + i]]
    assert not fp.fp_infer_cardinality(f, torch.empty((0, X.shape[1]), dtype=torch.float32, device="cuda")).any()


@pytest.mark.parametrize("n", [0, 1, 15, 17, 257, 4099])
def test_ragged_and_empty(small, n):
    f, X, _ = small
    Xn = X[:n]
    want = oracle.predict(f, Xn)
    for kw in ({"layout": fp.FP_LAYOUT_NAIVE}, {"bin_size": 16, "interleave_depth": 2}):
        p = upload(f, **kw)
        got = run(p, Xn, {"rows_per_block": 16, "cursors": 2})
        assert got[0].shape == (n, 2)
        assert_same(got, want, f"n={n} {kw}")


def test_strided_rows_and_special_values(small):
    f, X, _ = small
    X = X[:3000].copy()
    rng = np.random.default_rng(0)
    thr = f.threshold[f.feature >= 0]
    m = rng.random(X.shape)
    X[m < 0.05] = np.nan
    X[(m >= 0.05) & (m < 0.08)] = np.inf
    X[(m >= 0.08) & (m < 0.11)] = -np.inf
    X[(m >= 0.11) & (m < 0.13)] = np.float32(1e-44)   # denormal
    X[(m >= 0.13) & (m < 0.15)] = np.float32(-1e-44)
    X[(m >= 0.15) & (m < 0.17)] = -0.0
    # values exactly on thresholds and one ulp either side
    sel = (m >= 0.17) & (m < 0.40)
    pick = rng.choice(thr, size=sel.sum())
    bump = rng.integers(-1, 2, size=sel.sum())
    pick = np.where(bump > 0, np.nextafter(pick, np.float32(np.inf)),
                    np.where(bump < 0, np.nextafter(pick, np.float32(-np.inf)), pick))
    X[sel] = pick
    want = oracle.predict(f, X)
    for kw in ({"layout": fp.FP_LAYOUT_NAIVE}, {"bin_size": 4, "interleave_depth": 5},
               {"layout": fp.FP_LAYOUT_COMPACT, "bin_size": 4, "interleave_depth": 2},
               {"layout": fp.FP_LAYOUT_BLOCKED, "bin_size": 4, "interleave_depth": 1},
               {"layout": fp.FP_LAYOUT_CLUSTERED, "bin_size": 4, "interleave_depth": 3}):
        p = upload(f, **kw)
        assert_same(run(p, X, ld_pad=13), want, f"padded ld {kw}")
        assert_same(run(p, X, {"feature_lds": -1, "rows_per_block": 16}), want, f"global features {kw}")


def test_fp16_threshold_blocks_special_values():
    """CLUSTERED 48-byte blocks (fp16 thresholds): a forest whose thresholds
    are fp16 subnormals and an image forest, with rows on the thresholds, one
    fp32 ulp either side, and non-finite values; the default launch walks an
    fp16 tile, features from memory meet the thresholds widened to fp32."""
    rng = np.random.default_rng(5)
    Xi = rng.integers(0, 120, size=(4000, 6))
    y = ((Xi[:, 0] + Xi[:, 1] * 2 + rng.integers(0, 40, 4000)) // 70).astype(np.int32)
    tiny = synth.train_forest((Xi * 2.0 ** -23).astype(np.float32), y, n_trees=8, n_classes=int(y.max()) + 1,
                              mtry=3, max_depth=12, seed=3)
    w = synth.image(n_train=6000, n_trees=8)
    for f, X in ((tiny, (rng.integers(0, 120, size=(5000, 6)) * 2.0 ** -23).astype(np.float32)),
                 (w.forest(), w.predict_rows(5000)[0])):
        X = X.copy()
        thr = f.threshold[f.feature >= 0]
        m = rng.random(X.shape)
        sel = m < 0.3
        pick = rng.choice(thr, size=sel.sum())
        bump = rng.integers(-1, 2, size=sel.sum())
        X[sel] = np.where(bump > 0, np.nextafter(pick, np.float32(np.inf)),
                          np.where(bump < 0, np.nextafter(pick, np.float32(-np.inf)), pick))
        X[(m >= 0.3) & (m < 0.33)] = np.nan
        X[(m >= 0.33) & (m < 0.35)] = -np.inf
        X[(m >= 0.35) & (m < 0.37)] = np.float32(1e-44)
        X[(m >= 0.37) & (m < 0.39)] = -0.0
        want = oracle.predict(f, X)
        p = upload(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=4, interleave_depth=3)
        assert decode(fp.fp_packed_host_bytes(p))["h"]["block_bytes"] == 48
        assert_same(run(p, X), want, f"F={X.shape[1]} staged rows")
        assert_same(run(p, X, ld_pad=3), want, f"F={X.shape[1]} padded ld")
        assert_same(run(p, X, {"feature_lds": -1, "rows_per_block": 16}), want, f"F={X.shape[1]} global features")


def test_degenerate_forests():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((5000, 3)).astype(np.float32)
    y = (X[:, 0] > 0).astype(np.int32)
    y[:50] = 2
    f = synth.train_forest(X, y, n_trees=9, n_classes=3, mtry=1, max_depth=3, seed=2)
    g = f.subset(range(9))
    g.feature[g.tree_node_offset[4]] = -1  # tree 4: the root is a leaf
    g.leaf_class[g.tree_node_offset[4]] = 2
    for forest in (g, g.subset([4]), g.subset([0])):
        want = oracle.predict(forest, X)
        for kw in ({"layout": fp.FP_LAYOUT_NAIVE}, {"bin_size": 4, "interleave_depth": 0},
                   {"bin_size": 1, "interleave_depth": 3},
                   {"layout": fp.FP_LAYOUT_COMPACT, "bin_size": 4, "interleave_depth": 0},
                   {"layout": fp.FP_LAYOUT_BLOCKED, "bin_size": 4, "interleave_depth": 0},
                   {"layout": fp.FP_LAYOUT_BLOCKED, "bin_size": 2, "interleave_depth": 2},
                   {"layout": fp.FP_LAYOUT_CLUSTERED, "bin_size": 4, "interleave_depth": 0}):
            assert_same(run(upload(forest, **kw), X, {"rows_per_block": 8, "cursors": 4}), want,
                        f"T={forest.n_trees} {kw}")


def test_image_lite():
    w = synth.image(n_train=6000, n_trees=16)
    f = w.forest()
    X, _ = w.predict_rows(20_000)
    want = oracle.predict(f, X)
    assert_same(run(upload(f, layout=fp.FP_LAYOUT_NAIVE), X), want, "naive")
    for B, D, tune in ((16, 4, None), (4, 6, {"rows_per_block": 8, "cursors": 4, "tree_groups": 4}),
                       (8, 2, {"feature_lds": -1, "rows_per_block": 32})):
        assert_same(run(upload(f, bin_size=B, interleave_depth=D, line_align=1), X, tune), want, f"B={B} D={D}")
        assert_same(run(upload(f, layout=fp.FP_LAYOUT_COMPACT, bin_size=B, interleave_depth=D), X, tune), want,
                    f"compact B={B} D={D}")
        assert_same(run(upload(f, layout=fp.FP_LAYOUT_BLOCKED, bin_size=B, interleave_depth=D), X, tune), want,
                    f"blocked B={B} D={D}")
        assert_same(run(upload(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=B, interleave_depth=D), X, tune), want,
                    f"clustered B={B} D={D}")


def test_tabular_lite():
    w = synth.tabular(n_train=30_000, n_trees=32)
    f = w.forest()
    X, _ = w.predict_rows(50_000)
    want = oracle.predict(f, X)
    assert_same(run(upload(f, layout=fp.FP_LAYOUT_NAIVE), X), want, "naive")
    for B, D in ((16, 3), (32, 6)):
        assert_same(run(upload(f, bin_size=B, interleave_depth=D), X), want, f"B={B} D={D}")
        assert_same(run(upload(f, layout=fp.FP_LAYOUT_COMPACT, bin_size=B, interleave_depth=D), X), want,
                    f"compact B={B} D={D}")
        assert_same(run(upload(f, layout=fp.FP_LAYOUT_BLOCKED, bin_size=B, interleave_depth=D), X), want,
                    f"blocked B={B} D={D}")
        assert_same(run(upload(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=B, interleave_depth=D), X), want,
                    f"clustered B={B} D={D}")


def test_image_full_size():
    """1M rows x 128 trees in the benchmark's launch configuration: every row
    equals the CPU checker and the naive layout; every row's votes sum to T."""
    w = synth.image()
    f = w.forest()
    X, _ = w.predict_rows()
    cfg = presets.IMAGE
    p = upload(f, **cfg["pack"])
    Xd = torch.from_numpy(X).cuda()
    v, c = fp.fp_predict_tuned(p, cfg["tune"], Xd)
    pn = upload(f, layout=fp.FP_LAYOUT_NAIVE)
    vn, cn = fp.fp_predict_tuned(pn, cfg["naive_tune"], Xd)
    torch.cuda.synchronize()
    v, c, vn, cn = v.cpu().numpy(), c.cpu().numpy(), vn.cpu().numpy(), cn.cpu().numpy()
    assert (v.sum(1) == f.n_trees).all()
    want_v, want_c = oracle.predict(f, X)
    assert_same((v, c), (want_v, want_c), "clustered, all rows")
    assert_same((vn, cn), (want_v, want_c), "naive, all rows")


@pytest.mark.parametrize("F,pad", [(30, 2), (31, 1), (29, 7), (13, 3), (30, 0)])
def test_row_staging_ragged_columns(F, pad):
    """Whole-row tile staging (16-byte row loads, rows 16-byte aligned) with a
    column count that is not a multiple of 4, padded leading dimensions, and
    the unaligned fallback (pad 0 with F % 4 != 0)."""
    X, y = synth.gaussian_mixture(4000, F, 3, seed=900 + F)
    f = synth.train_forest(X, y, n_trees=12, n_classes=3, mtry=max(1, F // 3), max_depth=10, seed=901 + F)
    Xq, _ = synth.gaussian_mixture(3001, F, 3, seed=902 + F)
    want = oracle.predict(f, Xq)
    for layout in (fp.FP_LAYOUT_PACKED, fp.FP_LAYOUT_BLOCKED, fp.FP_LAYOUT_CLUSTERED):
        p = upload(f, layout=layout, bin_size=12, interleave_depth=3)
        assert_same(run(p, Xq, {"rows_per_block": 32, "cursors": 1, "block_threads": 512}, ld_pad=pad), want,
                    f"F={F} pad={pad} layout={layout}")


def test_many_classes_and_features():
    """Wide forests at the layouts' field limits through the kernels: 4,096
    classes (the packed kernel's vote-counter limit) in the node layouts, 32
    classes over 4,096 used features in the clustered 64-byte form, and 512
    features with fp16 thresholds in the clustered 48-byte form."""
    from handmade import depth3_forest
    rng = np.random.default_rng(12)
    feats = lambda n_used, T: [[(7 * t + k) % n_used for k in range(7)] for t in range(T)]
    cases = [(depth3_forest(600, feats(700, 600), 4096), [{"layout": fp.FP_LAYOUT_NAIVE},
                                                          {"bin_size": 16, "interleave_depth": 2},
                                                          {"layout": fp.FP_LAYOUT_COMPACT, "bin_size": 16}]),
             (depth3_forest(586, feats(4096, 586), 32), [{"layout": fp.FP_LAYOUT_CLUSTERED, "bin_size": 64}]),
             (depth3_forest(74, feats(512, 74), 32), [{"layout": fp.FP_LAYOUT_CLUSTERED, "bin_size": 74}])]
    for f, layouts in cases:
        X = rng.random((3000, f.n_features), dtype=np.float32)
        want = oracle.predict(f, X)
        for kw in layouts:
            try:
                p = upload(f, **kw)
            except fp.FPError as e:  # a layout whose fields cannot hold this forest says so
                assert e.code == fp.FP_E2BIG, kw
                continue
            r = 2 if f.n_classes > 1000 else 8  # explicit tiles must fit 4,096 vote counters per row
            for tune in (None, {"rows_per_block": r, "cursors": 1, "block_threads": 256}):
                assert_same(run(p, X, tune), want, f"C={f.n_classes} F={f.n_features} {kw} {tune}")


def test_fp16_tile_rounding_edges():
    """The fp16 observation tile of the CLUSTERED 48-byte form (features
    rounded toward +infinity): thresholds across the fp16 range (subnormals,
    +-65504, integers where the fp16 step is 2) and features on them, one
    fp32 ulp beside them, halfway to their fp16 neighbours (where nearest-even
    rounding would land on the threshold) and beyond the fp16 range.  The
    fp16 tile, the fp32 tile (feature_lds 2) and features from memory all
    equal the checker; a tile that fits LDS only in fp16 is refused in fp32."""
    from handmade import depth3_forest
    rng = np.random.default_rng(21)
    n_used, T = 512, 74
    f = depth3_forest(T, [[(7 * t + k) % n_used for k in range(7)] for t in range(T)], 5)
    bits = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16).view(np.float16)
    fin = bits[np.isfinite(bits)]
    special = np.array([0.0, -0.0, 65504, -65504, 2.0 ** -24, -(2.0 ** -24), 2.0 ** -14, 1.0, 2048, 2050, 0.5,
                        1000.5, -3.25], np.float16)
    thr = np.concatenate([special, fin[rng.integers(0, fin.size, f.n_trees * 15)]])[:f.n_trees * 15]
    f.threshold[:] = rng.permutation(thr).astype(np.float32)
    internal = f.feature >= 0
    n = 6000
    X = np.empty((n, f.n_features), np.float32)
    col_thr = [f.threshold[internal & (f.feature == c)] for c in range(f.n_features)]
    for c in range(f.n_features):
        t = rng.choice(col_thr[c], n).astype(np.float16)
        t32 = t.astype(np.float32).astype(np.float64)
        with np.errstate(over="ignore"):
            up = np.nextafter(t, np.float16(np.inf)).astype(np.float64)
            dn = np.nextafter(t, np.float16(-np.inf)).astype(np.float64)
        up = np.where(np.isinf(up), 65520.0, up)
        dn = np.where(np.isinf(dn), -65520.0, dn)
        cand = np.stack([t32, (t32 + up) / 2, (t32 + dn) / 2, up, dn]).astype(np.float32)
        x = cand[rng.integers(0, 5, n), np.arange(n)]
        step = rng.integers(-1, 2, n)
        x = np.where(step > 0, np.nextafter(x, np.float32(np.inf)),
                     np.where(step < 0, np.nextafter(x, np.float32(-np.inf)), x))
        m = rng.random(n)
        x[m < 0.02] = np.nan
        x[(m >= 0.02) & (m < 0.03)] = np.float32(1e-40)
        x[(m >= 0.03) & (m < 0.04)] = np.float32(-1e-40)
        x[(m >= 0.04) & (m < 0.05)] = np.float32(65519.99)
        x[(m >= 0.05) & (m < 0.06)] = np.float32(-7e4)
        x[(m >= 0.06) & (m < 0.07)] = -np.inf
        x[(m >= 0.07) & (m < 0.08)] = np.inf
        X[:, c] = x
    want = oracle.predict(f, X)
    p = upload(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=T, interleave_depth=3)
    assert decode(fp.fp_packed_host_bytes(p))["h"]["block_bytes"] == 48
    # 64 rows of 513 fp16 columns fit a workgroup's LDS; in fp32 they do not
    for tune in (None, {"rows_per_block": 64, "feature_lds": 1}, {"rows_per_block": 16, "feature_lds": 2},
                 {"rows_per_block": 16, "feature_lds": -1}, {"rows_per_block": 7, "block_threads": 256}):
        assert_same(run(p, X, tune), want, f"{tune}")
        assert_same(run(p, X, tune, ld_pad=3), want, f"{tune} padded ld")
    with pytest.raises(fp.FPError) as e:
        run(p, X, {"rows_per_block": 64, "feature_lds": 2})
    assert e.value.code == fp.FP_E2BIG
    with pytest.raises(fp.FPError) as e:
        run(p, X, {"feature_lds": 3})
    assert e.value.code == fp.FP_EINVAL
