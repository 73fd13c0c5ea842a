"""CPU checker for forest classification -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1806_07300_amd``) and never imports it.

``predict`` is the plain definition of forest classification that a packed
forest has to reproduce exactly: forest packing changes layout and evaluation
order, not the prediction (Sec. III-A).  Every observation walks each tree from
the root, going left when ``x[feature] <= threshold`` (fp32), until a leaf; the
leaf's single class label (Sec. III) gets one vote; votes are summed over the
trees; the predicted class is the argmax, ties to the lowest class index.

The forest arrives as concatenated per-tree arrays in node-creation order (the
breadth-first layout of Sec. III-A), exactly as the trainer in ``synth`` emits
them; the arithmetic lives in ``oracle.c`` (plain C, OpenMP over rows only).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the checker: plain -O2, OpenMP, no fast-math."""
    src = os.path.join(HERE, "oracle.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
           "-o", LIB_PATH + ".tmp", src]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.oracle_predict.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, i64, i64,
                                       vp, vp, vp, i32]
        lib.oracle_predict.restype = ctypes.c_int
        _lib = lib
    return _lib


def predict(forest, X: np.ndarray, n_threads: int = 0, return_visits: bool = False):
    """Votes int32 [n, C], predicted class int32 [n] (and total internal-node visits).

    ``forest`` is any object with ``n_trees, n_features, n_classes,
    tree_node_offset, feature, threshold, left, right, leaf_class`` arrays.
    """
    lib = _load()
    X = np.asarray(X)
    if X.dtype != np.float32:
        raise TypeError("X must be float32")
    if X.ndim != 2 or X.shape[1] < forest.n_features:
        raise ValueError("X must be [n, >= n_features]")
    if X.strides[1] != 4:
        X = np.ascontiguousarray(X)
    n = X.shape[0]
    ld = X.strides[0] // 4 if n > 0 else X.shape[1]
    C = forest.n_classes
    votes = np.zeros((n, C), np.int32)
    pred = np.zeros(n, np.int32)
    visits = ctypes.c_int64(0)
    arrs = [np.ascontiguousarray(getattr(forest, k), dtype=dt) for k, dt in
            (("tree_node_offset", np.int64), ("feature", np.int32), ("threshold", np.float32),
             ("left", np.int32), ("right", np.int32), ("leaf_class", np.int32))]
    rc = lib.oracle_predict(forest.n_trees, forest.n_features, C, *(a.ctypes.data for a in arrs),
                            X.ctypes.data if n else None, n, ld, votes.ctypes.data,
                            pred.ctypes.data, ctypes.byref(visits), n_threads)
    if rc != 0:
        raise ValueError("malformed forest: a walk left its tree or hit a bad class")
    if return_visits:
        return votes, pred, int(visits.value)
    return votes, pred
