"""Pins of the CPU checker against facts fixed outside it.

* Brute force over hand-built trees: every tree in tests/golden/box_trees.json
  also lists, written out by hand, the axis-aligned region each leaf covers.
  Every point of the grid {each threshold, its float32 neighbours, -inf, +inf,
  NaN}^F is classified by the checker and by box containment; they must agree.
  A dropped branch, a swapped child, '<' for '<=', denormal flushing or an
  off-by-one node base all fail here.
* Forest votes are one vote per tree for its leaf's class (Sec. III: a leaf
  holds a single class label), so they equal the sum of the box answers, sum
  to T for every row, are invariant under tree permutation, and a forest of T
  copies of one tree gives T times that tree's one-hot answer.
* Trees grown to purity without bootstrap classify every (distinct) training
  row as its own label: votes on training rows are T * onehot(y).
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "box_trees.json")


def f32(s):
    return np.float32(float(s))


def load_golden():
    with open(GOLDEN) as fh:
        return json.load(fh)["trees"]


def tree_forest(trees, n_features, n_classes):
    """Concatenate hand-built trees into the checker's forest arrays."""
    feat, thr, left, right, cls, off = [], [], [], [], [], [0]
    for t in trees:
        for f, th, l, r, c in t["nodes"]:
            feat.append(f); thr.append(f32(th)); left.append(l); right.append(r)
            cls.append(c if f < 0 else 0)
        off.append(off[-1] + len(t["nodes"]))
    n = off[-1]
    return synth.Forest(len(trees), n_features, n_classes, np.array(off, np.int64),
                        np.array(feat, np.int32), np.array(thr, np.float32),
                        np.array(left, np.int32), np.array(right, np.int32),
                        np.array(cls, np.int32), np.ones(n, np.int64), np.zeros(n, np.int32))


def box_class(tree, x):
    """Class of the unique box containing x (NaN lands where +inf does)."""
    hits = []
    for b in tree["boxes"]:
        ok = True
        for j in range(tree["n_features"]):
            v = np.float32(np.inf) if np.isnan(x[j]) else x[j]
            lo, hi = f32(b["lo"][j]), f32(b["hi"][j])
            lo_ok = (v > lo) or (lo == -np.inf)
            if not (lo_ok and v <= hi):
                ok = False
                break
        if ok:
            hits.append(b["class"])
    assert len(hits) == 1, f"fixture boxes must partition space: {tree['name']} {x} {hits}"
    return hits[0]


def grid(tree, n_features):
    vals = []
    for j in range(n_features):
        ts = {f32(th) for f, th, *_ in tree["nodes"] if f == j}
        s = {np.float32(-np.inf), np.float32(np.inf), np.float32(np.nan), np.float32(0.0)}
        for t in ts:
            s |= {t, np.nextafter(t, np.float32(np.inf)), np.nextafter(t, np.float32(-np.inf))}
        vals.append(sorted(s, key=lambda v: (np.isnan(v), v)))
    pts = np.array(list(itertools.product(*vals)), np.float32).reshape(-1, n_features)
    return pts


@pytest.mark.parametrize("tree", load_golden(), ids=lambda t: t["name"])
def test_single_tree_matches_boxes(tree):
    F, C = tree["n_features"], tree["n_classes"]
    forest = tree_forest([tree], F, C)
    X = grid(tree, F)
    votes, pred = oracle.predict(forest, X)
    expect = np.array([box_class(tree, x) for x in X])
    assert (votes.sum(1) == 1).all()
    assert (pred == expect).all(), X[pred != expect][:5]
    onehot = np.eye(C, dtype=np.int32)[expect]
    assert (votes == onehot).all()


def test_visit_counts():
    trees = {t["name"]: t for t in load_golden()}
    t = trees["one_feature_depth2"]
    X = grid(t, 1)
    _, _, visits = oracle.predict(tree_forest([t], 1, 2), X, return_visits=True)
    assert visits == 2 * len(X)  # complete depth-2 tree: two internal nodes per walk
    t = trees["root_is_leaf"]
    _, _, visits = oracle.predict(tree_forest([t], 2, 3), grid(t, 2), return_visits=True)
    assert visits == 0


def test_forest_votes_are_sum_of_boxes():
    trees = load_golden()
    F, C = 3, 4
    rng = np.random.default_rng(0)
    # points: mix of grid values of all trees, padded to 3 features
    specials = [np.float32(v) for v in (-np.inf, np.inf, np.nan, 0.0, -3.0, 3.0, 1.5, -0.25, 7.5, 1e-42)]
    base = rng.standard_normal((400, F)).astype(np.float32) * 4
    pick = rng.integers(0, len(specials), size=(400, F))
    mask = rng.random((400, F)) < 0.4
    X = np.where(mask, np.array(specials, np.float32)[pick], base).astype(np.float32)
    forest = tree_forest(trees, F, C)
    votes, pred = oracle.predict(forest, X)
    expect = np.zeros((len(X), C), np.int32)
    for t in trees:
        for i, x in enumerate(X):
            expect[i, box_class(t, x[:t["n_features"]])] += 1
    assert (votes == expect).all()
    assert (votes.sum(1) == len(trees)).all()
    assert (pred == np.argmax(expect, axis=1)).all()  # first maximum = lowest class on ties


def test_identical_trees_and_permutation():
    trees = load_golden()
    t = trees[3]
    X = grid(t, 3)
    one, _ = oracle.predict(tree_forest([t], 3, 4), X)
    many, _ = oracle.predict(tree_forest([t] * 9, 3, 4), X)
    assert (many == 9 * one).all()
    perm = [trees[i] for i in (5, 0, 3, 2, 1, 4)]
    a, _ = oracle.predict(tree_forest(trees, 3, 4), X)
    b, _ = oracle.predict(tree_forest(perm, 3, 4), X)
    assert (a == b).all()


def test_argmax_ties_lowest_class():
    trees = {t["name"]: t for t in load_golden()}
    # one tree answering 1 and one answering 0 at x=-5 (feature 0): a 1-1 tie -> class 0
    a = trees["one_feature_depth2"]  # x=-5 -> class 0
    b = trees["denormal_threshold"]  # x=-5 -> class 1
    votes, pred = oracle.predict(tree_forest([b, a], 1, 2), np.array([[-5.0]], np.float32))
    assert votes.tolist() == [[1, 1]] and pred.tolist() == [0]


def test_pure_trees_reproduce_training_labels():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((600, 5)).astype(np.float32)  # continuous: no duplicate rows
    y = rng.integers(0, 3, 600).astype(np.int32)           # labels carry no signal: deep trees
    f = synth.train_forest(X, y, n_trees=4, n_classes=3, mtry=2, bootstrap=False, seed=11)
    votes, pred, visits = oracle.predict(f, X, return_visits=True)
    assert (votes == 4 * np.eye(3, dtype=np.int32)[y]).all()
    assert (pred == y).all()
    assert visits > 600 * 4 * 3


def test_trained_forest_invariants():
    w = synth.small()
    f = w.forest()
    X, _ = w.predict_rows(3000)
    votes, pred = oracle.predict(f, X)
    assert (votes.sum(1) == f.n_trees).all()
    order = np.random.default_rng(1).permutation(f.n_trees)
    v2, _ = oracle.predict(f.subset(order), X)
    assert (v2 == votes).all()
    v3, _ = oracle.predict(f.subset([7]), X)
    assert (v3.sum(1) == 1).all()
    # thread count does not change the result
    v4, _ = oracle.predict(f, X, n_threads=1)
    assert (v4 == votes).all()


def test_strided_rows_and_empty():
    w = synth.small()
    f = w.forest()
    X, _ = w.predict_rows(257)
    wide = np.zeros((257, 40), np.float32)
    wide[:, :16] = X
    wide[:, 16:] = np.nan  # padding beyond n_features is never read
    a, _ = oracle.predict(f, X)
    b, _ = oracle.predict(f, wide)
    assert (a == b).all()
    v, p = oracle.predict(f, np.zeros((0, 16), np.float32))
    assert v.shape == (0, 2) and p.shape == (0,)
