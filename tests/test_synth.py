"""Pins of the seeded input generators (rows and the CART trainer).

The trainer only manufactures inputs, but a forest it gets wrong would make
every parity claim rest on odd forests, so it is pinned independently:
exhaustive split search with exact rational Gini on tiny data, structural
invariants (cardinality conservation, depth cap, threshold separation,
thread-count independence) and a partition cross-check against scikit-learn's
CART on tie-free data.
"""
from fractions import Fraction
import os
import itertools

import numpy as np
import pytest

import synth


def gini_score(y_left, y_right, C):
    """sum_c L_c^2/n_L + sum_c R_c^2/n_R as an exact rational (higher is better)."""
    s = Fraction(0)
    for part in (y_left, y_right):
        n = len(part)
        cnt = np.bincount(part, minlength=C)
        s += Fraction(int((cnt.astype(np.int64) ** 2).sum()), n)
    return s


def brute_force_candidates(X, y, C):
    """All (feature, threshold, score) candidates at boundaries of distinct values."""
    out = []
    for f in range(X.shape[1]):
        vals = np.unique(X[:, f])
        for a, b in zip(vals[:-1], vals[1:]):
            left = X[:, f] <= a
            out.append((f, a, b, gini_score(y[left], y[~left], C)))
    return out


def root_split(forest):
    return int(forest.feature[0]), np.float32(forest.threshold[0])


@pytest.mark.parametrize("seed", range(12))
def test_root_split_is_exhaustive_best(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 13))
    F = int(rng.integers(1, 4))
    C = int(rng.integers(2, 4))
    # small integer grid -> many ties, exercising the tie rules
    X = rng.integers(-3, 4, size=(n, F)).astype(np.float32)
    y = rng.integers(0, C, size=n).astype(np.int32)
    cands = brute_force_candidates(X, y, C)
    f = synth.train_forest(X, y, n_trees=1, n_classes=C, mtry=F, max_depth=1,
                           bootstrap=False, seed=seed)
    if not cands or len(np.unique(y)) == 1:
        assert f.feature[0] == -1
        return
    best = max(c[3] for c in cands)
    feat, thr = root_split(f)
    assert feat >= 0
    chosen = [c for c in cands if c[0] == feat and c[1] <= thr < c[2]]
    assert len(chosen) == 1, "threshold must fall strictly between two consecutive values"
    assert chosen[0][3] == best
    # tie rule inside the chosen feature: lowest threshold among equal best scores
    same_feature_best = [c for c in cands if c[0] == feat and c[3] == best]
    assert chosen[0][1] == min(c[1] for c in same_feature_best)
    # midpoint rule
    a, b = chosen[0][1], chosen[0][2]
    mid = np.float32((np.float64(a) + np.float64(b)) / 2)
    assert thr == (a if mid >= b else mid)


def test_root_split_tie_free_exact():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((11, 3)).astype(np.float32)
    y = np.array([0, 1, 1, 0, 1, 0, 0, 1, 1, 1, 0], np.int32)
    cands = brute_force_candidates(X, y, 2)
    best = max(cands, key=lambda c: c[3])
    assert sum(c[3] == best[3] for c in cands) == 1
    f = synth.train_forest(X, y, n_trees=1, n_classes=2, mtry=3, max_depth=1, bootstrap=False, seed=0)
    feat, thr = root_split(f)
    assert feat == best[0] and best[1] <= thr < best[2]


def test_threshold_between_adjacent_floats():
    a = np.float32(1.0)
    b = np.nextafter(a, np.float32(2.0))
    X = np.array([[a], [b]], np.float32)
    y = np.array([0, 1], np.int32)
    f = synth.train_forest(X, y, n_trees=1, n_classes=2, mtry=1, bootstrap=False, seed=0)
    assert f.threshold[0] == a  # the rounded midpoint would equal b: pulled down to a


def check_tree_invariants(f, n_train, max_depth):
    off = f.tree_node_offset
    for t in range(f.n_trees):
        lo, hi = off[t], off[t + 1]
        feat, left, right = f.feature[lo:hi], f.left[lo:hi], f.right[lo:hi]
        card, depth = f.cardinality[lo:hi], f.depth[lo:hi]
        internal = feat >= 0
        assert card[0] == n_train and depth[0] == 0
        assert (card[internal] == card[left[internal]] + card[right[internal]]).all()
        assert (card >= 1).all()
        assert (depth[left[internal]] == depth[internal] + 1).all()
        if max_depth >= 0:
            assert depth.max() <= max_depth
        # breadth-first creation order: children ids increase with parent ids, left before right
        assert (left[internal] == right[internal] - 1).all()
        assert (np.diff(left[internal]) > 0).all()
        assert (left[internal] > np.nonzero(internal)[0]).all()
        assert ((left[~internal] == -1) & (right[~internal] == -1)).all()
        assert (np.diff(depth) >= 0).all()


def test_small_forest_invariants_and_determinism():
    w = synth.small()
    X, y = w.train_rows()
    kw = dict(n_trees=6, n_classes=2, mtry=4, max_depth=12, seed=3)
    f1 = synth.train_forest(X, y, n_threads=1, **kw)
    f8 = synth.train_forest(X, y, n_threads=8, **kw)
    for k in ("tree_node_offset", "feature", "threshold", "left", "right", "leaf_class", "cardinality"):
        assert np.array_equal(getattr(f1, k), getattr(f8, k)), k
    check_tree_invariants(f1, len(X), 12)
    # a different seed gives a different forest
    f2 = synth.train_forest(X, y, n_threads=8, **{**kw, "seed": 4})
    assert not np.array_equal(f1.feature, f2.feature)


def test_thresholds_separate_training_values():
    """Every split threshold lies in [a, b) for consecutive distinct values of its node."""
    rng = np.random.default_rng(9)
    X = rng.standard_normal((300, 4)).astype(np.float32)
    y = (X[:, 0] + 0.3 * rng.standard_normal(300) > 0).astype(np.int32)
    f = synth.train_forest(X, y, n_trees=1, n_classes=2, mtry=4, bootstrap=False, seed=1)
    # route rows and check each internal node's threshold against its own rows
    members = {0: np.arange(300)}
    for node in range(f.n_nodes):
        rows = members.pop(node, None)
        if rows is None or f.feature[node] < 0:
            continue
        v = X[rows, f.feature[node]]
        go_left = v <= f.threshold[node]
        assert go_left.any() and (~go_left).any()
        assert v[go_left].max() <= f.threshold[node] < v[~go_left].min()
        members[int(f.left[node])] = rows[go_left]
        members[int(f.right[node])] = rows[~go_left]


def test_partition_matches_sklearn():
    """CART with mtry = F, no bootstrap, depth 3 on tie-free data reproduces
    scikit-learn's training-set partition (same '<=' and midpoint conventions)."""
    sk = pytest.importorskip("sklearn.tree")
    rng = np.random.default_rng(21)
    X = rng.standard_normal((2000, 4)).astype(np.float32)
    y = ((X[:, 0] * X[:, 1] + 0.5 * X[:, 2] + 0.4 * rng.standard_normal(2000)) > 0).astype(np.int32)
    f = synth.train_forest(X, y, n_trees=1, n_classes=2, mtry=4, max_depth=3, bootstrap=False, seed=2)
    clf = sk.DecisionTreeClassifier(max_depth=3, random_state=0).fit(X, y)

    def leaf_of(x):
        node = 0
        while f.feature[node] >= 0:
            node = f.left[node] if x[f.feature[node]] <= f.threshold[node] else f.right[node]
        return node
    ours = np.array([leaf_of(x) for x in X])
    theirs = clf.apply(X)
    part = lambda a: sorted(tuple(np.nonzero(a == v)[0]) for v in np.unique(a))
    assert part(ours) == part(theirs)


def test_row_chunks_are_independent():
    for gen in (lambda n, s, st: synth.gaussian_mixture(n, 5, 3, s, st),
                lambda n, s, st: synth.tabular_data(n, s, st),
                lambda n, s, st: synth.image_data(n, s, st)):
        Xa, ya = gen(70_000, 7, 0)
        Xb, yb = gen(1_000, 7, 65_000)
        assert np.array_equal(Xa[65_000:66_000], Xb) and np.array_equal(ya[65_000:66_000], yb)
        Xc, _ = gen(100, 7, 0)
        assert np.array_equal(Xa[:100], Xc)


def test_image_rows_statistics():
    X, y = synth.image_data(20_000, 102)
    assert X.shape == (20_000, 784) and X.dtype == np.float32
    assert abs((X == 0).mean() - 0.80) <= 0.01
    assert X.min() >= 0 and X.max() <= 255 and np.array_equal(X, np.rint(X))
    assert set(np.unique(y)) == set(range(10))


def test_tabular_rows_statistics():
    X, y = synth.tabular_data(50_000, 202)
    assert X.shape == (50_000, 28)
    assert abs(y.mean() - 0.5) < 0.02
    m = synth.tabular_model()
    z = X[:, :21].astype(np.float64)
    prod = z[:, m.pairs[:, 0]] * z[:, m.pairs[:, 1]]
    assert np.allclose(prod, X[:, 21:], rtol=1e-5, atol=1e-6)


def test_batched_specs():
    s = [synth.batched_spec(i) for i in range(64)]
    assert (s[0].n_trees, s[0].n_features, s[0].n_classes, s[0].n_rows) == (16, 4, 2, 1)
    assert (s[63].n_trees, s[63].n_features, s[63].n_classes, s[63].n_rows) == (2048, 784, 10, 200_000)
    for b in s:
        assert 16 <= b.n_trees <= 2048 and 4 <= b.n_features <= 784
        assert 2 <= b.n_classes <= 10 and 1 <= b.n_rows <= 200_000


def test_chunked_training_is_identical():
    w = synth.small()
    X, y = w.train_rows()
    a = synth.train_forest(X, y, n_trees=10, n_classes=2, mtry=4, max_depth=12, seed=3)
    seen = []

    class Progress:
        chunk = 3

        def __call__(self, done, total):
            seen.append((done, total))

    b = synth.train_forest(X, y, n_trees=10, n_classes=2, mtry=4, max_depth=12, seed=3, progress=Progress())
    assert seen == [(3, 10), (6, 10), (9, 10), (10, 10)]
    for k in ("tree_node_offset", "feature", "threshold", "left", "right", "leaf_class", "cardinality"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k


# --- the node's feature order, restated from the published generators -----
# SplitMix64 (Steele, Lea, Flood) seeds xoshiro256** (Blackman, Vigna); the
# tree's stream starts from (forest seed, tree index) and, without bootstrap,
# its first draws are the root's Fisher-Yates shuffle of the feature indices.
M64 = (1 << 64) - 1


def _splitmix(x):
    x = (x + 0x9E3779B97F4A7C15) & M64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return x, z ^ (z >> 31)


def _rotl(v, k):
    return ((v << k) | (v >> (64 - k))) & M64


def _root_feature_order(seed, tree, F):
    x = (seed ^ ((0xD1B54A32D192ED03 * (tree + 1)) & M64)) & M64
    s = []
    for _ in range(4):
        x, z = _splitmix(x)
        s.append(z)

    def nxt():
        r = (_rotl((s[1] * 5) & M64, 7) * 9) & M64
        t = (s[1] << 17) & M64
        s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3]
        s[2] ^= t
        s[3] = _rotl(s[3], 45)
        return r

    def bounded(n):  # rejection of the biased low range
        lim = (1 << 64) % n
        while True:
            v = nxt()
            if v >= lim:
                return v % n

    perm = list(range(F))
    for i in range(F - 1, 0, -1):
        j = bounded(i + 1)
        perm[i], perm[j] = perm[j], perm[i]
    return perm


@pytest.mark.parametrize("seed", range(16))
def test_cross_feature_tie_keeps_first_in_shuffled_order(seed):
    """Features 0, 1 and 2 split the rows identically (1 is 0 scaled, 2 is 0
    negated and so splits the same rows from the other side): three
    candidates with the same exact Gini score.  The root must split on the
    tied feature that comes first in the node's shuffled order, whichever
    that is for this seed; feature 3 is noise with a worse score."""
    rng = np.random.default_rng(100 + seed)
    x0 = rng.permutation(np.arange(40, dtype=np.float32))
    y = (x0 >= 17).astype(np.int32)
    noise = rng.standard_normal(40).astype(np.float32)
    X = np.stack([x0, 4.0 * x0, -x0, noise], axis=1).astype(np.float32)
    f = synth.train_forest(X, y, n_trees=1, n_classes=2, mtry=4, max_depth=1, bootstrap=False, seed=seed)
    order = _root_feature_order(seed, 0, 4)
    first_tied = next(k for k in order if k in (0, 1, 2))
    assert f.feature[0] == first_tied, (order, int(f.feature[0]))
    # a later tied feature would have been kept by a rule that prefers the last
    assert f.feature[0] != [k for k in order if k in (0, 1, 2)][-1]


@pytest.mark.parametrize("seed", range(12))
def test_mtry_fallback_searches_past_constant_features(seed):
    """Three of four features are constant: with mtry = 1 the shuffled list's
    first feature is usually one of them, and the search must continue down
    the list until the one separating feature is found (a leaf would be the
    mistake)."""
    rng = np.random.default_rng(seed)
    X = np.zeros((30, 4), np.float32)
    X[:, 0], X[:, 1], X[:, 2] = 1.0, -2.0, 5.0
    X[:, 3] = rng.standard_normal(30).astype(np.float32)
    y = (X[:, 3] > 0).astype(np.int32)
    f = synth.train_forest(X, y, n_trees=1, n_classes=2, mtry=1, max_depth=1, bootstrap=False, seed=seed)
    assert f.feature[0] == 3
    assert X[y == 0, 3].max() <= f.threshold[0] < X[y == 1, 3].min()


def test_shuffle_restatement_matches_the_trainer():
    """The restated shuffle above is the trainer's: with mtry = 1 and every
    feature separating the rows, the root splits on the order's first entry."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((50, 6)).astype(np.float32)
    y = (X.sum(1) > 0).astype(np.int32)
    for seed in range(20):
        f = synth.train_forest(X, y, n_trees=1, n_classes=2, mtry=1, max_depth=1, bootstrap=False, seed=seed)
        assert f.feature[0] == _root_feature_order(seed, 0, 6)[0], seed


def test_training_rejects_nan():
    X = np.zeros((10, 2), np.float32)
    X[3, 1] = np.nan
    y = np.arange(10, dtype=np.int32) % 2
    with pytest.raises(RuntimeError):
        synth.train_forest(X, y, n_trees=1, n_classes=2, mtry=2, bootstrap=False, seed=0)


class _StopAfter:
    """A progress callback that interrupts training after `n` chunks."""
    chunk = 8

    def __init__(self, n):
        self.n, self.calls = n, []

    def __call__(self, done, total):
        self.calls.append(done)
        if len(self.calls) == self.n:
            raise KeyboardInterrupt


def test_interrupted_training_resumes_to_the_same_forest(tmp_path):
    """Chunks of finished trees are kept while a forest trains; a second call
    after an interruption loads them, trains only the rest, and the forest is
    the one an uninterrupted training gives (tree t depends on (seed, t) only)."""
    w = synth.small()
    X, y = w.train_rows()
    kw = dict(n_trees=w.n_trees, n_classes=w.n_classes, mtry=w.mtry, max_depth=w.max_depth, seed=w.forest_seed)
    whole = synth.train_forest(X, y, **kw)
    prefix = str(tmp_path / "f")
    stop = _StopAfter(2)
    with pytest.raises(KeyboardInterrupt):
        synth.train_forest(X, y, progress=stop, checkpoint=prefix, **kw)
    assert sorted(os.listdir(tmp_path)) == ["f.trees0-8.npz", "f.trees8-16.npz"]
    seen = []

    class Count:
        chunk = 8

        def __call__(self, done, total):
            seen.append(done)

    # a chunk file that cannot be read is trained again
    with open(tmp_path / "f.trees8-16.npz", "wb") as fh:
        fh.write(b"not a forest")
    resumed = synth.train_forest(X, y, progress=Count(), checkpoint=prefix, **kw)
    assert seen == [8, 16, 24, 32]
    assert sorted(os.listdir(tmp_path)) == ["f.trees0-8.npz", "f.trees16-24.npz", "f.trees24-32.npz",
                                            "f.trees8-16.npz"]
    for k in ("tree_node_offset", "feature", "threshold", "left", "right", "leaf_class", "cardinality", "depth"):
        assert np.array_equal(getattr(resumed, k), getattr(whole, k)), k


def test_workload_cache_removes_its_chunks(tmp_path):
    w = synth.small()
    f = w.forest(cache_dir=str(tmp_path))
    assert os.listdir(tmp_path) == ["forest_small.npz"]
    g = w.forest(cache_dir=str(tmp_path))
    assert np.array_equal(f.threshold, g.threshold) and np.array_equal(f.tree_node_offset, g.tree_node_offset)
