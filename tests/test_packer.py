"""Host packer (no GPU): layout invariants of Sec. III-A and packed == unpacked.

Invariants checked on the decoded bytes:
  * DF-  : no leaf is stored; leaves are class references; every internal node
           of the forest is stored exactly once;
  * Bin  : bins hold consecutive trees (last one short); the top region holds
           exactly the internal nodes of depth <= D, level-major and tree-minor,
           so depth 0 (the roots) is contiguous (Fig. 2 caption);
  * Stat : below depth D, the child with more training samples (left on ties,
           an internal child over a leaf) sits right after its parent;
  * every reference points forward inside its bin (walks terminate);
  * walking the packed bytes gives exactly the checker's votes, for a grid of
    bin sizes and interleave depths (layout never changes predictions).
"""
import os

import numpy as np
import pytest

import oracle
import paper_1806_07300_amd as fp
import synth

from packed_format import decode, walk


@pytest.fixture(scope="module")
def small_forest():
    return synth.small().forest()


@pytest.fixture(scope="module")
def small_rows():
    X, _ = synth.small().predict_rows(2000)
    return X


def node_map(forest, dec, be, j):
    """Map packed node index -> (original local id, depth) for tree j of bin be."""
    t = be["first_tree"] + j
    off = forest.tree_node_offset[t]
    bn = dec["nodes"][be["node_base"]:be["node_base"] + be["top_len"] + be["deep_len"]]
    root = dec["roots"][be["root_base"] + j]
    out = {}
    stack = [(root, 0, 0)]
    while stack:
        ref, orig, d = stack.pop()
        if ref < 0:
            assert forest.feature[off + orig] < 0
            assert -ref - 1 == forest.leaf_class[off + orig]
            continue
        assert forest.feature[off + orig] >= 0
        assert ref not in out
        out[ref] = (orig, d)
        nd = bn[ref]
        assert dec["fmap"][nd["feat"]] == forest.feature[off + orig]
        assert nd["thr"] == forest.threshold[off + orig]
        stack.append((nd["left"], forest.left[off + orig], d + 1))
        stack.append((nd["right"], forest.right[off + orig], d + 1))
    return out


@pytest.mark.parametrize("B", [1, 2, 7, 16, 32])
@pytest.mark.parametrize("D", [0, 1, 3, 6])
def test_packed_equals_unpacked(small_forest, small_rows, B, D):
    p = fp.fp_pack_forest(small_forest, bin_size=B, interleave_depth=D)
    dec = decode(fp.fp_packed_host_bytes(p))
    votes, _ = oracle.predict(small_forest, small_rows)
    assert (walk(dec, small_rows) == votes).all()


@pytest.mark.parametrize("B,D,align", [(16, 3, 0), (5, 2, 1), (32, 0, 0), (1, 4, 1)])
def test_layout_invariants(small_forest, B, D, align):
    f = small_forest
    p = fp.fp_pack_forest(f, bin_size=B, interleave_depth=D, line_align=align)
    info = fp.fp_packed_info_get(p)
    dec = decode(fp.fp_packed_host_bytes(p))
    h = dec["h"]
    assert info["n_internal"] == f.n_internal() and info["n_leaves"] == f.n_nodes - f.n_internal()
    bins = dec["bins"]
    assert len(bins) == -(-f.n_trees // B)
    assert [int(b["first_tree"]) for b in bins] == list(range(0, f.n_trees, B))
    assert all(b["n_trees"] == B for b in bins[:-1]) and 1 <= bins[-1]["n_trees"] <= B
    stored = 0
    for be in bins:
        assert be["node_base"] % 8 == 0  # every bin starts on a 128-byte line
        bn = dec["nodes"][be["node_base"]:be["node_base"] + be["top_len"] + be["deep_len"]]
        real = ~((bn["feat"] == 0) & (bn["left"] == 0) & (bn["right"] == 0))
        assert (bn["feat"][real] < h["n_used_features"]).all()
        stored += int(real.sum())
        seen = {}
        tree_of = {}
        for j in range(be["n_trees"]):
            m = node_map(f, dec, be, j)
            for ref, (orig, d) in m.items():
                seen[ref] = (orig, d, j)
        assert set(seen) == set(np.nonzero(real)[0].tolist())
        top = [seen[i] for i in range(be["top_len"])]
        # top region = exactly the internal nodes of depth <= D, level-major, tree-minor
        assert all(d <= D for _, d, _ in top)
        assert all(d > D for i, (_, d, _) in seen.items() if i >= be["top_len"])
        keys = [(d, j) for _, d, j in top]
        assert keys == sorted(keys)
        # roots contiguous at the start
        n_int_roots = sum(1 for _, d, _ in top if d == 0)
        roots = dec["roots"][be["root_base"]:be["root_base"] + be["n_trees"]]
        assert sorted(int(r) for r in roots if r >= 0) == list(range(n_int_roots))
        # references point forward
        for i in np.nonzero(real)[0]:
            for c in (bn[i]["left"], bn[i]["right"]):
                assert c < 0 or c > i
        # Stat: hot child adjacent below depth D
        for i, (orig, d, j) in seen.items():
            if i < be["top_len"]:
                continue
            t = be["first_tree"] + j
            off = f.tree_node_offset[t]
            l, r = f.left[off + orig], f.right[off + orig]
            li, ri = f.feature[off + l] >= 0, f.feature[off + r] >= 0
            if li and ri:
                hot = l if f.cardinality[off + l] >= f.cardinality[off + r] else r
            elif li:
                hot = l
            elif ri:
                hot = r
            else:
                continue
            nxt = seen.get(i + 1)
            assert nxt is not None and nxt[0] == hot and nxt[2] == j, (i, orig, hot)
    assert stored == f.n_internal()
    assert h["max_top_len"] == max(int(b["top_len"]) for b in bins)
    used = np.unique(f.feature[f.feature >= 0])
    assert np.array_equal(dec["fmap"], used) and info["n_used_features"] == len(used)


def test_naive_depth_first_order(small_forest, small_rows):
    """NAIVE with node_order DF (the DF layout of Sec. III-A): every tree's
    nodes, leaves included, in depth-first pre-order, left child first; the
    walk still gives the checker's votes."""
    f = small_forest
    dec = decode(fp.fp_packed_host_bytes(fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_NAIVE,
                                                           node_order=fp.FP_ORDER_DF)))
    off = dec["tree_off"]
    for t in range(f.n_trees):
        tn = dec["nodes"][off[t]:off[t + 1]]
        o = f.tree_node_offset[t]
        assert len(tn) == f.tree_node_offset[t + 1] - o
        # packed index i must be the i-th node of a pre-order walk of the original tree
        order, stack = [], [0]
        while stack:
            n = stack.pop()
            order.append(n)
            if f.feature[o + n] >= 0:
                stack += [f.right[o + n], f.left[o + n]]
        pos = {n: i for i, n in enumerate(order)}
        for i, n in enumerate(order):
            nd = tn[i]
            if f.feature[o + n] >= 0:
                assert (nd["feat"], nd["thr"]) == (f.feature[o + n], f.threshold[o + n])
                assert (nd["left"], nd["right"]) == (pos[f.left[o + n]], pos[f.right[o + n]])
                assert nd["left"] == i + 1  # the left child always follows its parent
            else:
                assert nd["feat"] < 0 and nd["left"] == f.leaf_class[o + n]
    assert (walk(dec, small_rows) == oracle.predict(f, small_rows)[0]).all()


@pytest.mark.parametrize("B,D", [(1, 0), (16, 3), (5, 1)])
def test_packed_without_stat(small_forest, small_rows, B, D):
    """PACKED with node_order DF (DF-: class references, no Stat): below the
    interleaved levels the left internal child follows its parent whatever
    the cardinalities; predictions unchanged."""
    f = small_forest
    dec = decode(fp.fp_packed_host_bytes(fp.fp_pack_forest(f, bin_size=B, interleave_depth=D,
                                                           node_order=fp.FP_ORDER_DF)))
    assert (walk(dec, small_rows) == oracle.predict(f, small_rows)[0]).all()
    n_right_hot = 0
    for be in dec["bins"]:
        seen = {}
        for j in range(be["n_trees"]):
            for ref, (orig, d) in node_map(f, dec, be, j).items():
                seen[ref] = (orig, d, j)
        for i, (orig, d, j) in seen.items():
            if i < be["top_len"]:
                continue
            off = f.tree_node_offset[be["first_tree"] + j]
            l, r = f.left[off + orig], f.right[off + orig]
            li, ri = f.feature[off + l] >= 0, f.feature[off + r] >= 0
            if not (li or ri):
                continue
            nxt = seen.get(i + 1)
            assert nxt is not None and nxt[0] == (l if li else r) and nxt[2] == j
            n_right_hot += li and ri and f.cardinality[off + r] > f.cardinality[off + l]
    assert n_right_hot > 0  # Stat would have placed these right children first


def test_node_order_rejected_where_undefined(small_forest):
    for layout in (fp.FP_LAYOUT_COMPACT, fp.FP_LAYOUT_BLOCKED, fp.FP_LAYOUT_CLUSTERED):
        with pytest.raises(fp.FPError) as e:
            fp.fp_pack_forest(small_forest, layout=layout, node_order=fp.FP_ORDER_DF)
        assert e.value.code == fp.FP_EINVAL
    with pytest.raises(fp.FPError) as e:
        fp.fp_pack_forest(small_forest, node_order=2)
    assert e.value.code == fp.FP_EINVAL


def test_cost_model_statistics():
    """expected_depth, expected_fetches and mean_bias mean what they claim.
    Trees grown without bootstrap give every node the number of training rows
    that reach it as its cardinality, so walking the training rows themselves
    must visit expected_depth internal nodes and load expected_fetches fetch
    units per tree on average, exactly; mean_bias is max(LC, RC) / PN averaged
    over internal nodes, recounted here from the trees."""
    from packed_format import walk_blocked, walk_clustered
    X, y = synth.gaussian_mixture(3000, 12, 3, seed=31)
    f = synth.train_forest(X, y, n_trees=5, n_classes=3, mtry=4, max_depth=10, bootstrap=False, seed=32)
    n_walks = len(X) * f.n_trees
    _, _, visits = oracle.predict(f, X, return_visits=True)
    depth = visits / n_walks
    ratios = []
    for t in range(f.n_trees):
        o = f.tree_node_offset[t]
        for n in range(f.tree_node_offset[t + 1] - o):
            if f.feature[o + n] >= 0:
                lc, rc = f.cardinality[o + f.left[o + n]], f.cardinality[o + f.right[o + n]]
                assert lc + rc == f.cardinality[o + n]
                ratios.append(max(lc, rc) / (lc + rc))
    bias = float(np.mean(ratios))
    assert 0.5 < bias < 1.0
    for layout in (fp.FP_LAYOUT_NAIVE, fp.FP_LAYOUT_PACKED, fp.FP_LAYOUT_COMPACT, fp.FP_LAYOUT_BLOCKED,
                   fp.FP_LAYOUT_CLUSTERED):
        p = fp.fp_pack_forest(f, layout=layout, bin_size=2, interleave_depth=3)
        info = fp.fp_packed_info_get(p)
        assert info["expected_depth"] == pytest.approx(depth, rel=1e-12), layout
        assert info["mean_bias"] == pytest.approx(bias, rel=1e-12), layout
        if layout == fp.FP_LAYOUT_NAIVE:
            want = depth + 1  # the stored leaf is fetched too
        elif layout in (fp.FP_LAYOUT_PACKED, fp.FP_LAYOUT_COMPACT):
            want = depth
        else:
            stats = {}
            dec = decode(fp.fp_packed_host_bytes(p))
            walk_fn = walk_blocked if layout == fp.FP_LAYOUT_BLOCKED else walk_clustered
            assert (walk_fn(dec, X, stats) == oracle.predict(f, X)[0]).all()
            want = stats["fetches"] / n_walks
            assert want < depth / 2  # a block serves more than two visits here
        assert info["expected_fetches"] == pytest.approx(want, rel=1e-12), layout


def test_deterministic_bytes_and_roundtrip(small_forest, tmp_path):
    a = fp.fp_packed_host_bytes(fp.fp_pack_forest(small_forest, bin_size=8, interleave_depth=2))
    b = fp.fp_packed_host_bytes(fp.fp_pack_forest(small_forest, bin_size=8, interleave_depth=2))
    assert np.array_equal(a, b)
    p = fp.fp_packed_from_bytes(a)
    assert np.array_equal(fp.fp_packed_host_bytes(p), a)
    path = str(tmp_path / "f.fpk")
    fp.fp_packed_save(p, path)
    q = fp.fp_packed_load(path)
    assert np.array_equal(fp.fp_packed_host_bytes(q), a)
    # one flipped byte in the node section, a truncation, a bad magic
    bad = a.copy()
    bad[len(bad) // 2] ^= 0x40
    for corrupt in (bad, a[:-256], np.concatenate([np.zeros(8, np.uint8), a[8:]])):
        with pytest.raises(fp.FPError) as e:
            fp.fp_packed_from_bytes(corrupt)
        assert e.value.code == fp.FP_ECORRUPT
    with open(path, "r+b") as fh:
        fh.truncate(1000)
    with pytest.raises(fp.FPError) as e:
        fp.fp_packed_load(path)
    assert e.value.code == fp.FP_ECORRUPT


def test_naive_layout(small_forest, small_rows):
    p = fp.fp_pack_forest(small_forest, layout=fp.FP_LAYOUT_NAIVE)
    info = fp.fp_packed_info_get(p)
    assert info["n_nodes"] == small_forest.n_nodes  # leaves are stored
    dec = decode(fp.fp_packed_host_bytes(p))
    votes, _ = oracle.predict(small_forest, small_rows)
    assert (walk(dec, small_rows) == votes).all()
    assert np.array_equal(fp.fp_packed_host_bytes(fp.fp_packed_from_bytes(fp.fp_packed_host_bytes(p))),
                          fp.fp_packed_host_bytes(p))


def test_no_cardinality_and_single_node_trees():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((300, 3)).astype(np.float32)
    y = (X[:, 0] > 0).astype(np.int32)
    y[:5] = 2
    f = synth.train_forest(X, y, n_trees=9, n_classes=3, mtry=1, max_depth=3, seed=2)
    # make tree 4 a lone leaf (root is a leaf)
    g = f.subset(range(9))
    off = g.tree_node_offset
    g.feature[off[4]] = -1
    g.leaf_class[off[4]] = 2
    for use_card in (True, False):
        for B, D in ((4, 0), (9, 2), (1, 1)):
            p = fp.fp_pack_forest(g, bin_size=B, interleave_depth=D, use_cardinality=use_card)
            votes, _ = oracle.predict(g, X)
            assert (walk(decode(fp.fp_packed_host_bytes(p)), X) == votes).all()


def _forest_copy(f):
    return f.subset(range(f.n_trees))


@pytest.mark.parametrize("mutation", ["feature", "child_range", "cycle", "shared", "class", "offsets"])
def test_malformed_forest_rejected(small_forest, mutation):
    g = _forest_copy(small_forest)
    off = g.tree_node_offset
    t0 = off[3]
    internal = np.nonzero(g.feature[off[3]:off[4]] >= 0)[0]
    leaf = np.nonzero(g.feature[off[3]:off[4]] < 0)[0]
    i = int(internal[2])
    if mutation == "feature":
        g.feature[t0 + i] = g.n_features
    elif mutation == "child_range":
        g.right[t0 + i] = int(off[4] - off[3])
    elif mutation == "cycle":
        g.left[t0 + i] = 0
    elif mutation == "shared":
        g.right[t0 + i] = g.left[t0 + i]
    elif mutation == "class":
        g.leaf_class[t0 + int(leaf[0])] = g.n_classes
    elif mutation == "offsets":
        g.tree_node_offset = off.copy()
        g.tree_node_offset[5] = g.tree_node_offset[4] - 1
    with pytest.raises(fp.FPError) as e:
        fp.fp_pack_forest(g, bin_size=4, interleave_depth=2)
    assert e.value.code == fp.FP_ECORRUPT


def test_bad_options(small_forest):
    with pytest.raises(fp.FPError) as e:
        fp.fp_pack_forest(small_forest, layout=7)
    assert e.value.code == fp.FP_EINVAL
    with pytest.raises(fp.FPError) as e:
        fp.fp_pack_forest(small_forest, interleave_depth=-1)
    assert e.value.code == fp.FP_EINVAL


def test_image_forest_packs(tmp_path):
    w = synth.image(n_train=6000, n_trees=8)
    f = w.forest()
    X, _ = w.predict_rows(500)
    votes, _ = oracle.predict(f, X)
    for B, D in ((8, 4), (3, 6)):
        p = fp.fp_pack_forest(f, bin_size=B, interleave_depth=D, line_align=1)
        assert (walk(decode(fp.fp_packed_host_bytes(p)), X) == votes).all()



@pytest.mark.parametrize("B", [1, 5, 16, 32])
@pytest.mark.parametrize("D", [0, 2, 4])
def test_compact_equals_unpacked(small_forest, small_rows, B, D):
    p = fp.fp_pack_forest(small_forest, layout=fp.FP_LAYOUT_COMPACT, bin_size=B, interleave_depth=D)
    dec = decode(fp.fp_packed_host_bytes(p))
    assert dec["h"]["layout"] == 2
    votes, _ = oracle.predict(small_forest, small_rows)
    assert (walk(dec, small_rows) == votes).all()
    # round trip through the verifier
    q = fp.fp_packed_from_bytes(fp.fp_packed_host_bytes(p))
    assert np.array_equal(fp.fp_packed_host_bytes(q), fp.fp_packed_host_bytes(p))


def test_compact_layout_invariants():
    """Every compact deep node's adjacent child is the Stat hot child; the two
    layouts place every internal node at the same reference."""
    from packed_format import compact_bin, decode_node8
    w = synth.image(n_train=6000, n_trees=8)
    f = w.forest()
    a = decode(fp.fp_packed_host_bytes(fp.fp_pack_forest(f, bin_size=4, interleave_depth=3)))
    c = decode(fp.fp_packed_host_bytes(fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_COMPACT, bin_size=4,
                                                          interleave_depth=3)))
    assert np.array_equal(a["roots"], c["roots"]) and np.array_equal(a["fmap"], c["fmap"])
    n_deep = 0
    for ba, bc in zip(a["bins"], c["bins"]):
        assert ba["top_len"] == bc["top_len"] and ba["deep_len"] == bc["deep_len"]
        bn = a["nodes"][ba["node_base"]:ba["node_base"] + ba["top_len"] + ba["deep_len"]]
        top, deep = compact_bin(c, bc)
        tl = int(ba["top_len"])
        assert np.array_equal(top["thr"], bn["thr"][:tl]) and np.array_equal(top["left"], bn["left"][:tl])
        fl = decode_node8(c["h"], deep["w"])
        for i in range(len(deep)):
            nd = bn[tl + i]
            self = tl + i
            assert deep["thr"][i] == nd["thr"] and fl["feat"][i] == nd["feat"]
            l, r = int(nd["left"]), int(nd["right"])
            if l < 0 and r < 0:
                assert fl["adj"][i] == 0 and fl["lclass"][i] == -l - 1 and fl["rclass"][i] == -r - 1
                continue
            assert fl["adj"][i] == 1
            adj, other = (l, r) if fl["adj_left"][i] else (r, l)
            assert adj == self + 1
            if other < 0:
                assert fl["cold_class"][i] == 1 and fl["payload"][i] == -other - 1
            else:
                assert fl["cold_class"][i] == 0 and self + fl["payload"][i] == other
            n_deep += 1
    assert n_deep > 1000


def test_compact_rejects_bad_bytes(small_forest):
    a = fp.fp_packed_host_bytes(fp.fp_pack_forest(small_forest, layout=fp.FP_LAYOUT_COMPACT, bin_size=8,
                                                  interleave_depth=2))
    bad = a.copy()
    bad[len(bad) - 300] ^= 0x10
    with pytest.raises(fp.FPError) as e:
        fp.fp_packed_from_bytes(bad)
    assert e.value.code == fp.FP_ECORRUPT


@pytest.mark.parametrize("B", [1, 5, 16, 32])
@pytest.mark.parametrize("D", [0, 2, 4])
def test_blocked_equals_unpacked(small_forest, small_rows, B, D):
    p = fp.fp_pack_forest(small_forest, layout=fp.FP_LAYOUT_BLOCKED, bin_size=B, interleave_depth=D)
    dec = decode(fp.fp_packed_host_bytes(p))
    assert dec["h"]["layout"] == 3
    votes, _ = oracle.predict(small_forest, small_rows)
    assert (walk(dec, small_rows) == votes).all()
    q = fp.fp_packed_from_bytes(fp.fp_packed_host_bytes(p))
    assert np.array_equal(fp.fp_packed_host_bytes(q), fp.fp_packed_host_bytes(p))


def wide_forest():
    """A forest whose node words need the 64-byte block form (11 feature bits,
    12 classes)."""
    X, y = synth.gaussian_mixture(3000, 1100, 12, seed=77)
    return synth.train_forest(X, y, n_trees=6, n_classes=12, mtry=300, max_depth=14, seed=78), X


@pytest.mark.parametrize("which", ["image48", "wide64"])
def test_blocked_layout_invariants(which):
    """Each block holds a complete three-level subtree of one tree (slot s has
    its children at 2s+1 and 2s+2); every internal node is stored exactly once;
    a block's child blocks are contiguous, after it, and in descending order of
    training cardinality; blocks whose root has depth <= D come first,
    level-major and tree-minor (Bin at block granularity)."""
    from packed_format import blocked_bin, block_fields
    if which == "image48":
        f = synth.image(n_train=6000, n_trees=8).forest()
    else:
        f, _ = wide_forest()
    for B, D in ((4, 3), (8, 0), (3, 7)):
        c = decode(fp.fp_packed_host_bytes(fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_BLOCKED, bin_size=B,
                                                              interleave_depth=D)))
        h = c["h"]
        assert h["block_bytes"] == (48 if which == "image48" else 64)
        n_block_nodes = 0
        for bc in c["bins"]:
            assert bc["top_len"] == 0 and bc["node_base"] % 16 == 0
            _, blocks = blocked_bin(c, bc)
            bf = block_fields(h, blocks)
            owner = {}  # block -> (tree j, block level)
            for j in range(int(bc["n_trees"])):
                t = int(bc["first_tree"]) + j
                off = f.tree_node_offset[t]
                root = int(c["roots"][bc["root_base"] + j])
                if root < 0:
                    assert f.feature[off] < 0 and -root - 1 == f.leaf_class[off]
                    continue
                stack = [(root, 0, 0)]
                while stack:
                    k, orig, level = stack.pop()
                    assert k not in owner
                    owner[k] = (j, level)
                    assert f.depth[off + orig] == 3 * level
                    slot_orig = {0: orig}
                    exits = []
                    for sl in range(7):
                        if sl not in slot_orig:
                            assert bf["word"][k, sl] == 0 and bf["thr"][k, sl] == 0
                            continue
                        o = slot_orig[sl]
                        assert c["fmap"][bf["feat"][k, sl]] == f.feature[off + o]
                        assert bf["thr"][k, sl] == f.threshold[off + o]
                        n_block_nodes += 1
                        for side, ch in enumerate((f.left[off + o], f.right[off + o])):
                            kind, pay = bf["kind"][k, sl, side], bf["pay"][k, sl, side]
                            if f.feature[off + ch] < 0:
                                assert kind == 1 and pay == f.leaf_class[off + ch]
                            elif sl < 3:
                                assert kind == 0 and pay == 0
                                slot_orig[2 * sl + 1 + side] = ch
                            else:
                                assert kind == 0
                                exits.append((int(pay), ch))
                    exits.sort()
                    assert [r for r, _ in exits] == list(range(len(exits)))
                    cards = [f.cardinality[off + ch] for _, ch in exits]
                    assert cards == sorted(cards, reverse=True)
                    for r, ch in exits:
                        child = int(bf["child_base"][k]) + r
                        assert child > k
                        stack.append((child, ch, level + 1))
            assert set(owner) == set(range(int(bc["deep_len"])))
            # interleaved prefix: level-major, tree-minor; then tree by tree
            order = [owner[k] for k in range(int(bc["deep_len"]))]
            n_front = sum(1 for _, lv in order if lv <= D // 3)
            front, rest = order[:n_front], order[n_front:]
            assert all(lv <= D // 3 for _, lv in front) and front == sorted(front, key=lambda x: (x[1], x[0]))
            assert all(lv > D // 3 for _, lv in rest) and [j for j, _ in rest] == sorted(j for j, _ in rest)
        assert n_block_nodes == int((f.feature >= 0).sum())


def test_blocked_wide_equals_unpacked():
    f, X = wide_forest()
    votes, _ = oracle.predict(f, X[:500])
    for B, D in ((6, 3), (2, 0)):
        p = fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_BLOCKED, bin_size=B, interleave_depth=D)
        dec = decode(fp.fp_packed_host_bytes(p))
        assert dec["h"]["block_bytes"] == 64
        assert (walk(dec, X[:500]) == votes).all()


def test_blocked_rejects_bad_bytes(small_forest):
    a = fp.fp_packed_host_bytes(fp.fp_pack_forest(small_forest, layout=fp.FP_LAYOUT_BLOCKED, bin_size=8,
                                                  interleave_depth=2))
    bad = a.copy()
    bad[len(bad) - 300] ^= 0x10
    with pytest.raises(fp.FPError) as e:
        fp.fp_packed_from_bytes(bad)
    assert e.value.code == fp.FP_ECORRUPT


def test_blocked_verifier_catches_structural_faults(small_forest):
    """Faults planted behind a valid checksum, in both block forms: a backward
    exit, a stray slot, a class out of range, a missing exit rank / child base."""
    from packed_format import BLOCK, BLOCK48, reseal
    wide, _ = wide_forest()
    for f in (small_forest, wide):
        p = fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_BLOCKED, bin_size=4, interleave_depth=1)
        good = fp.fp_packed_host_bytes(p)
        assert np.array_equal(fp.fp_packed_host_bytes(fp.fp_packed_from_bytes(reseal(good))), good)
        dec = decode(good)
        h, be = dec["h"], dec["bins"][0]
        base = h["nodes_offset"] + 8 * int(be["node_base"])
        faults = []

        def planted(offset, value):
            bad = good.copy()
            bad[offset:offset + 4] = np.frombuffer(np.array([value], "<u4").tobytes(), np.uint8)
            return reseal(bad)

        if h["block_bytes"] == 48:
            blocks = np.frombuffer(good.tobytes(), BLOCK48, count=int(be["deep_len"]), offset=base)
            cb = blocks["words"][:, 4] >> 8
            k = int(np.nonzero(cb > 8)[0][8])  # a block with exits, 8 blocks in
            faults.append(planted(base + 48 * k + 16, int(blocks["words"][k, 4]) & 0xFF))  # child base 0
            kl = int(np.nonzero(blocks["thr"][:, 6] == 0)[0][0])  # last slot empty
            faults.append(planted(base + 48 * kl + 20 + 24, 0x3F800000))  # a threshold in an absent slot
            faults.append(planted(base + 48 * k, int(blocks["words"][k, 0]) | (((h["n_classes"] << 1) | 1)
                                                                                << h["compact_fbits"])))
        else:
            blocks = np.frombuffer(good.tobytes(), BLOCK, count=int(be["deep_len"]), offset=base)
            k = int(np.nonzero(blocks["ranks"])[0][8])
            kl = int(np.nonzero(blocks["slot"]["w"][:, 6] == 0)[0][0])
            faults.append(planted(base + 64 * k, 0))  # child_base 0: exit points backward
            faults.append(planted(base + 64 * kl + 8 + 6 * 8 + 4, 1))  # word in an absent slot
            faults.append(planted(base + 64 * k + 8 + 4, int(blocks["slot"]["w"][k, 0]) |
                                  (((h["n_classes"] << 1) | 1) << h["compact_fbits"])))
            faults.append(planted(base + 64 * k + 4, 0))  # exits lose their ranks
        for i, bad in enumerate(faults):
            with pytest.raises(fp.FPError) as e:
                fp.fp_packed_from_bytes(bad)
            assert e.value.code == fp.FP_ECORRUPT, (h["block_bytes"], i)


@pytest.mark.parametrize("B", [1, 5, 32])
@pytest.mark.parametrize("D", [0, 3, 6])
def test_clustered_equals_unpacked(small_forest, small_rows, B, D):
    p = fp.fp_pack_forest(small_forest, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=B, interleave_depth=D)
    dec = decode(fp.fp_packed_host_bytes(p))
    assert dec["h"]["layout"] == 4
    votes, _ = oracle.predict(small_forest, small_rows)
    assert (walk(dec, small_rows) == votes).all()
    q = fp.fp_packed_from_bytes(fp.fp_packed_host_bytes(p))
    assert np.array_equal(fp.fp_packed_host_bytes(q), fp.fp_packed_host_bytes(p))


def test_clustered_layout_invariants():
    """A block holds a connected group of at most 7 internal nodes grown from
    its root by always taking the frontier node with the most training samples
    (ties: lower node id); every internal node is in exactly one block; exits
    partition the outcomes of the block's slots; child blocks are contiguous,
    after their parent, in descending order of cardinality."""
    import heapq
    from packed_format import blocked_bin, cluster_fields
    f = synth.image(n_train=6000, n_trees=6).forest()
    X, _ = synth.image(n_train=6000, n_trees=6).predict_rows(300)
    c = decode(fp.fp_packed_host_bytes(fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=3,
                                                          interleave_depth=3)))
    assert c["h"]["block_bytes"] == 48  # 353 used pixel columns, half-integer thresholds
    assert (walk(c, X) == oracle.predict(f, X)[0]).all()
    seen_nodes = 0
    for bc in c["bins"]:
        _, blocks = blocked_bin(c, bc)
        cf = cluster_fields(blocks)
        assert all(v == 0 for v in cf["stray"])
        owner = set()
        for j in range(int(bc["n_trees"])):
            t = int(bc["first_tree"]) + j
            off = f.tree_node_offset[t]
            feat, left, right, card = (f.feature[off:], f.left[off:], f.right[off:], f.cardinality[off:])
            root = int(c["roots"][bc["root_base"] + j])
            stack = [(root, 0)] if root >= 0 else []
            while stack:
                k, orig = stack.pop()
                assert k not in owner
                owner.add(k)
                # greedy reconstruction of the group from the forest
                members, front = [], [(-card[orig], orig)]
                while front and len(members) < 7:
                    _, nd = heapq.heappop(front)
                    members.append(nd)
                    for ch in (left[nd], right[nd]):
                        if feat[ch] >= 0:
                            heapq.heappush(front, (-card[ch], ch))
                m = len(members)
                assert cf["n_exits"][k] == m + 1
                for sl, nd in enumerate(members):
                    assert c["fmap"][cf["feat"][k, sl]] == feat[nd] and cf["thr"][k, sl] == f.threshold[off + nd]
                assert (cf["feat"][k, m:] == 0).all() and (cf["thr"][k, m:] == 0).all()
                seen_nodes += m
                # the exits partition the 2^m outcomes
                hits = np.zeros(1 << m, np.int64)
                g = np.arange(1 << m)
                for e in range(m + 1):
                    hits += ((g ^ cf["val"][k, e]) & cf["care"][k, e]) == 0
                assert (hits == 1).all()
                # child blocks: the internal children outside the group, in exit
                # order (slot, then side), then hottest first (stable)
                outside = [ch for nd in members for ch in (left[nd], right[nd]) if feat[ch] >= 0 and ch not in members]
                assert sorted(outside) == sorted(nd for _, nd in front)
                kids = sorted(outside, key=lambda nd: -card[nd])
                ranks = sorted(int(tg & 7) for tg in cf["target"][k, :m + 1] if tg & 32)
                assert ranks == list(range(len(kids))) and cf["n_children"][k] == len(kids)
                cards = [card[nd] for nd in kids]
                assert cards == sorted(cards, reverse=True)
                for r, nd in enumerate(kids):
                    child = int(cf["child_base"][k]) + r
                    assert child > k
                    stack.append((child, nd))
        assert owner == set(range(int(bc["deep_len"])))
    assert seen_nodes == int((f.feature >= 0).sum())


@pytest.fixture(scope="module")
def image_forest():
    return synth.image(n_train=6000, n_trees=6).forest(), synth.image(n_train=6000, n_trees=6).predict_rows(500)[0]


def test_clustered_block_form_choice(small_forest, image_forest):
    """The 48-byte form (fp16 thresholds, 9-bit features) is taken only when
    every threshold converts to fp16 exactly and the used features fit 9 bits,
    so both forms compare the same fp32 values."""
    f, X = image_forest
    pack = lambda f: decode(fp.fp_packed_host_bytes(fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=2,
                                                                      interleave_depth=3)))
    assert pack(small_forest)["h"]["block_bytes"] == 64  # thresholds are not fp16 values
    c48 = pack(f)
    assert c48["h"]["block_bytes"] == 48 and c48["h"]["compact_fbits"] <= 9
    votes = oracle.predict(f, X)[0]
    assert (walk(c48, X) == votes).all()
    # one threshold with fp32-only precision sends the whole forest to 64 bytes
    g = f.subset(range(f.n_trees))  # copies every array
    i = int(np.nonzero(g.feature >= 0)[0][3])
    g.threshold[i] = np.float32(g.threshold[i] + np.float32(1e-3))
    c64 = pack(g)
    assert c64["h"]["block_bytes"] == 64
    assert (walk(c64, X) == oracle.predict(g, X)[0]).all()


def test_clustered_fp16_denormal_thresholds():
    """Thresholds that are fp16 subnormals (multiples of 2^-24 below 2^-14)
    still take the 48-byte form and widen back to the same fp32 values."""
    rng = np.random.default_rng(5)
    Xi = rng.integers(0, 120, size=(4000, 6))
    y = ((Xi[:, 0] + Xi[:, 1] * 2 + rng.integers(0, 40, 4000)) // 70).astype(np.int32)
    X = (Xi * 2.0 ** -23).astype(np.float32)
    f = synth.train_forest(X, y, n_trees=8, n_classes=int(y.max()) + 1, mtry=3, max_depth=12, seed=3)
    th = f.threshold[f.feature >= 0]
    assert ((np.abs(th) < 2.0 ** -14) & (th != 0)).all()
    c = decode(fp.fp_packed_host_bytes(fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=4,
                                                          interleave_depth=3)))
    assert c["h"]["block_bytes"] == 48
    Xq = (rng.integers(0, 120, size=(3000, 6)) * 2.0 ** -23).astype(np.float32)
    Xq[::7] = np.nextafter(Xq[::7], np.float32(1))  # one fp32 ulp above grid points
    assert (walk(c, Xq) == oracle.predict(f, Xq)[0]).all()


@pytest.mark.parametrize("form", [64, 48])
def test_clustered_verifier_catches_overlapping_exits(small_forest, image_forest, form):
    from packed_format import reseal
    f = small_forest if form == 64 else image_forest[0]
    good = fp.fp_packed_host_bytes(fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=4,
                                                     interleave_depth=0))
    dec = decode(good)
    assert dec["h"]["block_bytes"] == form
    be = dec["bins"][0]
    base = dec["h"]["nodes_offset"] + 8 * int(be["node_base"])
    care = 28 if form == 64 else 16  # byte offset of the care bytes in a block
    faults = []
    bad = good.copy()
    bad[base + care] = 0x01  # exit 0 tests only slot 0: it now overlaps another exit
    faults.append(bad)
    bad = good.copy()
    bad[base + care + 7] = 0x00  # an unused exit (care 0x80) that would match everything
    faults.append(bad)
    if form == 48:
        bad = good.copy()
        bad[base + 32 + 7] |= 0x40  # bit 62: a spare bit between the fields
        faults.append(bad)
        bad = good.copy()
        bad[base + 32 + 11] |= 0x10  # bit 92: another spare bit
        faults.append(bad)
        bad = good.copy()
        bad[base:base + 2] = [0x00, 0x7E]  # a NaN threshold
        faults.append(bad)
    for i, bad in enumerate(faults):
        with pytest.raises(fp.FPError) as e:
            fp.fp_packed_from_bytes(reseal(bad))
        assert e.value.code == fp.FP_ECORRUPT, i


def test_clustered_limits():
    from handmade import depth3_forest
    """CLUSTERED holds at most 32 classes and 4,096 used features (12-bit
    fields), and takes the 48-byte form up to 512 used features when every
    threshold is an fp16 value; past each limit it reports FP_E2BIG or falls
    back to the 64-byte form, and packs at the limit walk like the checker."""
    rng = np.random.default_rng(8)
    def check(f, want_bytes):
        dec = decode(fp.fp_packed_host_bytes(fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=64,
                                                               interleave_depth=3)))
        assert dec["h"]["block_bytes"] == want_bytes
        X = rng.random((200, f.n_features), dtype=np.float32)
        assert (walk(dec, X) == oracle.predict(f, X)[0]).all()
    feats = lambda n_used, T: [[(7 * t + k) % n_used for k in range(7)] for t in range(T)]
    check(depth3_forest(74, feats(512, 74), 32), 48)           # 518 splits over exactly 512 features
    check(depth3_forest(74, feats(513, 74), 32), 64)           # 513 features: 9 bits no longer suffice
    check(depth3_forest(74, feats(512, 74), 32, thr=0.1), 64)  # 0.1 is not an fp16 value
    check(depth3_forest(586, feats(4096, 586), 32), 64)        # 4,102 splits over exactly 4,096 features
    for f in (depth3_forest(586, feats(4097, 586), 32), depth3_forest(8, feats(56, 8), 33)):
        with pytest.raises(fp.FPError) as e:
            fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_CLUSTERED)
        assert e.value.code == fp.FP_E2BIG
