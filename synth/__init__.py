"""Seeded synthetic inputs shared by the CPU checker and the GPU library.

This module manufactures the *inputs* of the packing method: observation
matrices shaped like the paper's benchmark datasets (Table I: an MNIST-like
image set and Higgs/Allstate-like tabular sets) and trained random forests
(the method's input is a trained forest of T trees, Sec. III).  It holds none
of the method's arithmetic: no layout, no traversal, no vote counting.

Rows are generated in fixed chunks of ``CHUNK`` rows, each chunk from its own
``numpy.random.Generator(PCG64(SeedSequence([seed, chunk])))`` stream, so any
row range can be regenerated on its own (a sampled check of a large batch only
needs the chunks that hold the sampled rows).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcart.so")
CHUNK = 1 << 16


# --------------------------------------------------------------------------
# native trainer
# --------------------------------------------------------------------------
def build(verbose: bool = False) -> str:
    """Compile the CART trainer (plain C, OpenMP, no fast-math)."""
    src = os.path.join(HERE, "cart.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
           "-o", LIB_PATH + ".tmp", src]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [("n_trees", ctypes.c_int32), ("n_features", ctypes.c_int32),
                ("n_classes", ctypes.c_int32), ("mtry", ctypes.c_int32),
                ("max_depth", ctypes.c_int32), ("min_samples_split", ctypes.c_int32),
                ("bootstrap", ctypes.c_int32), ("n_threads", ctypes.c_int32),
                ("tree_offset", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        lib.cart_train.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, vp,
                                   ctypes.POINTER(_Params), ctypes.POINTER(vp)]
        lib.cart_train.restype = ctypes.c_int
        lib.cart_data_create.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, vp, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.POINTER(vp)]
        lib.cart_data_create.restype = ctypes.c_int
        lib.cart_train_prepared.argtypes = [vp, ctypes.POINTER(_Params), ctypes.POINTER(vp)]
        lib.cart_train_prepared.restype = ctypes.c_int
        lib.cart_data_free.argtypes = [vp]
        lib.cart_data_free.restype = None
        lib.cart_total_nodes.argtypes = [vp]
        lib.cart_total_nodes.restype = ctypes.c_int64
        lib.cart_export.argtypes = [vp] * 9
        lib.cart_export.restype = None
        lib.cart_free.argtypes = [vp]
        lib.cart_free.restype = None
        _lib = lib
    return _lib


@dataclass
class Forest:
    """A trained forest as concatenated per-tree arrays in node-creation order.

    Node ids inside ``left``/``right`` are tree-local; node 0 of every tree is
    its root; ``feature < 0`` marks a leaf whose label is ``leaf_class``.
    ``cardinality`` is the in-bag training count reaching the node.
    """
    n_trees: int
    n_features: int
    n_classes: int
    tree_node_offset: np.ndarray  # int64 [T+1]
    feature: np.ndarray           # int32 [nodes]
    threshold: np.ndarray         # float32 [nodes]
    left: np.ndarray              # int32 [nodes]
    right: np.ndarray             # int32 [nodes]
    leaf_class: np.ndarray        # int32 [nodes]
    cardinality: np.ndarray       # int64 [nodes]
    depth: np.ndarray             # int32 [nodes]

    @property
    def n_nodes(self) -> int:
        return int(self.tree_node_offset[-1])

    def n_internal(self) -> int:
        return int((self.feature >= 0).sum())

    def save(self, path: str) -> None:
        np.savez(path, meta=np.array([self.n_trees, self.n_features, self.n_classes], np.int64),
                 tree_node_offset=self.tree_node_offset, feature=self.feature,
                 threshold=self.threshold, left=self.left, right=self.right,
                 leaf_class=self.leaf_class, cardinality=self.cardinality, depth=self.depth)

    @staticmethod
    def load(path: str) -> "Forest":
        z = np.load(path)  # allow_pickle stays False
        t, f, c = (int(v) for v in z["meta"])
        return Forest(t, f, c, *(z[k] for k in ("tree_node_offset", "feature", "threshold", "left",
                                                  "right", "leaf_class", "cardinality", "depth")))

    def subset(self, trees) -> "Forest":
        """Forest made of the listed trees, in the listed order."""
        off = self.tree_node_offset
        parts = [np.arange(off[t], off[t + 1]) for t in trees]
        idx = np.concatenate(parts) if parts else np.zeros(0, np.int64)
        sizes = np.array([off[t + 1] - off[t] for t in trees], np.int64)
        new_off = np.zeros(len(trees) + 1, np.int64)
        new_off[1:] = np.cumsum(sizes)
        return Forest(len(trees), self.n_features, self.n_classes, new_off,
                      *(getattr(self, k)[idx].copy() for k in
                        ("feature", "threshold", "left", "right", "leaf_class", "cardinality", "depth")))


def train_forest(X: np.ndarray, y: np.ndarray, *, n_trees: int, n_classes: int, mtry: int,
                 max_depth: int = -1, bootstrap: bool = True, seed: int = 0,
                 min_samples_split: int = 2, n_threads: int = 0, tree_offset: int = 0,
                 progress=None, checkpoint: str | None = None) -> Forest:
    """Train a seeded CART random forest (see the header of cart.c).

    Tree t depends only on (seed, tree_offset + t), so a forest can be trained
    in chunks; with ``progress`` set, trees are trained in chunks of that many
    (default 64) and ``progress(done, total)`` is called after each chunk.
    With ``checkpoint`` (a path prefix) set, each finished chunk is saved as
    ``<prefix>.trees<first>-<end>.npz`` and a later call with the same
    prefix loads the chunks it finds instead of training them again, so an
    interrupted training resumes where it stopped and yields the same forest.
    The prefix must name one (data, parameters) pair; the caller removes the
    chunk files once the forest is kept elsewhere."""
    chunk = max(1, int(getattr(progress, "chunk", 64))) if progress is not None else n_trees
    if checkpoint is not None and progress is None:
        chunk = 64
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.int32)
    n, F = X.shape
    data = ctypes.c_void_p()
    rc = lib.cart_data_create(X.ctypes.data, n, F, F, y.ctypes.data, n_classes, n_threads, ctypes.byref(data))
    if rc != 0:
        raise RuntimeError(f"cart_data_create failed with code {rc}")
    try:
        parts = []
        for t0 in range(0, n_trees, chunk):
            k = min(chunk, n_trees - t0)
            part = f"{checkpoint}.trees{tree_offset + t0}-{tree_offset + t0 + k}.npz" if checkpoint else None
            if part and os.path.exists(part):
                try:
                    f = Forest.load(part)
                except Exception:  # an unreadable chunk file is trained again
                    f = None
                if f is not None and f.n_trees == k and f.n_features == F and f.n_classes == n_classes:
                    parts.append(f)
                    if progress is not None:
                        progress(t0 + k, n_trees)
                    continue
            p = _Params(k, F, n_classes, mtry, max_depth, min_samples_split, int(bool(bootstrap)),
                        n_threads, tree_offset + t0, 0, seed & 0xFFFFFFFFFFFFFFFF)
            h = ctypes.c_void_p()
            rc = lib.cart_train_prepared(data, ctypes.byref(p), ctypes.byref(h))
            if rc != 0:
                raise RuntimeError(f"cart_train_prepared failed with code {rc}")
            try:
                parts.append(_export(lib, h, k, F, n_classes))
            finally:
                lib.cart_free(h)
            if part:
                _save_atomic(parts[-1], part)
            if progress is not None:
                progress(t0 + k, n_trees)
    finally:
        lib.cart_data_free(data)
    return parts[0] if len(parts) == 1 else concat_forests(parts)


def _export(lib, h, n_trees, F, n_classes) -> Forest:
    total = lib.cart_total_nodes(h)
    off = np.zeros(n_trees + 1, np.int64)
    arrs = dict(feature=np.empty(total, np.int32), threshold=np.empty(total, np.float32),
                left=np.empty(total, np.int32), right=np.empty(total, np.int32),
                leaf_class=np.empty(total, np.int32), cardinality=np.empty(total, np.int64),
                depth=np.empty(total, np.int32))
    lib.cart_export(h, off.ctypes.data, *(arrs[k].ctypes.data for k in
                                            ("feature", "threshold", "left", "right",
                                             "leaf_class", "cardinality", "depth")))
    return Forest(n_trees, F, n_classes, off, **arrs)


def concat_forests(parts) -> Forest:
    """Forest made of the trees of several forests, in order."""
    sizes = np.concatenate([np.diff(f.tree_node_offset) for f in parts])
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    f0 = parts[0]
    return Forest(int(len(sizes)), f0.n_features, f0.n_classes, off,
                  *(np.concatenate([getattr(f, k) for f in parts]) for k in
                    ("feature", "threshold", "left", "right", "leaf_class", "cardinality", "depth")))


# --------------------------------------------------------------------------
# row generators
# --------------------------------------------------------------------------
def _chunk_rng(seed: int, chunk: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, chunk])))


def _rows(gen_chunk, n: int, start: int, F: int, seed: int):
    """Assemble rows [start, start+n) from independently seeded chunks
    (chunks are generated on a thread pool; each has its own stream, so the
    result does not depend on scheduling)."""
    X = np.empty((n, F), np.float32)
    y = np.empty(n, np.int32)
    if n == 0:
        return X, y
    c0, c1 = start // CHUNK, (start + n - 1) // CHUNK

    def one(c):
        Xc, yc = gen_chunk(_chunk_rng(seed, c), CHUNK)
        lo = max(start, c * CHUNK)
        hi = min(start + n, (c + 1) * CHUNK)
        X[lo - start:hi - start] = Xc[lo - c * CHUNK:hi - c * CHUNK]
        y[lo - start:hi - start] = yc[lo - c * CHUNK:hi - c * CHUNK]

    chunks = range(c0, c1 + 1)
    if len(chunks) == 1:
        one(c0)
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=min(len(chunks), os.cpu_count() or 1, 16)) as ex:
            list(ex.map(one, chunks))
    return X, y


def gaussian_mixture(n: int, n_features: int, n_classes: int, seed: int, start: int = 0):
    """Isotropic Gaussian classes: y uniform over C classes, x ~ N(mu_y * 1, I),
    mu_c = c/(C-1).  With C = 2 this is the two-Gaussian recipe (means 0 and 1, sd 1)."""
    F, C = n_features, n_classes

    def chunk(rng, m):
        y = rng.integers(0, C, size=m).astype(np.int32)
        mu = (y.astype(np.float64) / max(C - 1, 1))[:, None]
        X = (rng.standard_normal((m, F)) + mu).astype(np.float32)
        return X, y
    return _rows(chunk, n, start, F, seed)


@dataclass
class ImageModel:
    """Per-class mean images for the 784-pixel, 10-class image-shaped recipe."""
    active: np.ndarray  # int64 [C, K] pixel indices of each class's active set
    mean: np.ndarray    # float64 [C, K] mean value per active pixel
    keep: float
    noise_sd: float
    label_noise: float


IMAGE_F, IMAGE_C = 784, 10


def image_model(model_seed: int = 100, keep: float = 0.72, noise_sd: float = 48.0,
                label_noise: float = 0.08) -> ImageModel:
    """Class means on 30% of the pixels, drawn inside a shared 45% pool so the
    classes overlap.  ``keep`` (0.72) is tuned for an 80% zero rate and
    ``label_noise`` (8% of labels redrawn uniformly) for trees of about 5,000
    internal nodes and maximum depth near 50, the MNIST forest of Table I."""
    rng = np.random.Generator(np.random.PCG64(model_seed))
    pool = rng.choice(IMAGE_F, size=int(round(0.45 * IMAGE_F)), replace=False)
    K = int(round(0.30 * IMAGE_F))
    active = np.stack([np.sort(rng.choice(pool, size=K, replace=False)) for _ in range(IMAGE_C)])
    mean = rng.uniform(0.0, 255.0, size=(IMAGE_C, K))
    return ImageModel(active.astype(np.int64), mean, keep, noise_sd, label_noise)


def image_data(n: int, seed: int, start: int = 0, model: ImageModel | None = None):
    """MNIST-shaped rows: 784 integer-valued fp32 pixels in 0..255, 10 classes,
    about 80% zeros.  A row's image comes from mixture component k (uniform);
    an active pixel of k is kept with probability ``keep`` and set to
    clip(round(mean + N(0, sd^2)), 0, 255); all others are 0.  The label is k,
    except for a ``label_noise`` fraction of rows whose label is redrawn
    uniformly."""
    mdl = model or image_model()
    K = mdl.active.shape[1]

    def chunk(rng, m):
        k = rng.integers(0, IMAGE_C, size=m)
        noise = rng.standard_normal((m, K))
        kept = rng.random((m, K)) < mdl.keep
        vals = np.clip(np.rint(mdl.mean[k] + mdl.noise_sd * noise), 0.0, 255.0)
        vals = np.where(kept, vals, 0.0).astype(np.float32)
        X = np.zeros((m, IMAGE_F), np.float32)
        np.put_along_axis(X, mdl.active[k], vals, axis=1)
        redraw = rng.random(m) < mdl.label_noise
        y = np.where(redraw, rng.integers(0, IMAGE_C, size=m), k).astype(np.int32)
        return X, y
    return _rows(chunk, n, start, IMAGE_F, seed)


@dataclass
class TabularModel:
    pairs: np.ndarray  # int64 [7, 2]
    A: np.ndarray      # float64 [21, 21] symmetric
    w: np.ndarray      # float64 [21]


TAB_Z, TAB_P = 21, 7


def tabular_model(model_seed: int = 200) -> TabularModel:
    rng = np.random.Generator(np.random.PCG64(model_seed))
    iu = np.array([(a, b) for a in range(TAB_Z) for b in range(a + 1, TAB_Z)], np.int64)
    pairs = iu[np.sort(rng.choice(len(iu), size=TAB_P, replace=False))]
    s = 1.0 / math.sqrt(TAB_Z)
    U = rng.normal(0.0, s, size=(TAB_Z, TAB_Z))
    A = np.triu(U) + np.triu(U, 1).T
    w = rng.normal(0.0, s, size=TAB_Z)
    return TabularModel(pairs, A, w)


def tabular_data(n: int, seed: int, start: int = 0, model: TabularModel | None = None, shift: float = 0.0):
    """Higgs-shaped rows: 21 standard normals plus 7 pairwise products (28 fp32
    features); label ~ Bernoulli(sigmoid(2 q - shift)) for the standardised
    quadratic form q = z'Az + w'z (mean tr A, sd sqrt(2 tr A^2 + |w|^2)).
    shift 0 gives about half positives; shift 3.35 about 10% (class imbalance)."""
    mdl = model or tabular_model()
    mean_q = float(np.trace(mdl.A))
    sd_q = math.sqrt(2.0 * float(np.trace(mdl.A @ mdl.A)) + float(mdl.w @ mdl.w))

    def chunk(rng, m):
        z = rng.standard_normal((m, TAB_Z))
        prods = z[:, mdl.pairs[:, 0]] * z[:, mdl.pairs[:, 1]]
        q = np.einsum("ij,jk,ik->i", z, mdl.A, z) + z @ mdl.w
        qt = (q - mean_q) / sd_q
        p1 = 1.0 / (1.0 + np.exp(-(2.0 * qt - shift)))
        y = (rng.random(m) < p1).astype(np.int32)
        X = np.concatenate([z, prods], axis=1).astype(np.float32)
        return X, y
    return _rows(chunk, n, start, TAB_Z + TAB_P, seed)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    n_features: int
    n_classes: int
    n_trees: int
    mtry: int
    max_depth: int
    n_train: int
    n_predict: int
    train_seed: int
    predict_seed: int
    forest_seed: int
    kind: str  # "mixture" | "image" | "tabular"
    shift: float = 0.0  # tabular: label logit offset (class imbalance)

    def rows(self, n: int, seed: int, start: int = 0):
        if self.kind == "image":
            return image_data(n, seed, start)
        if self.kind == "tabular":
            return tabular_data(n, seed, start, shift=self.shift)
        return gaussian_mixture(n, self.n_features, self.n_classes, seed, start)

    def train_rows(self):
        return self.rows(self.n_train, self.train_seed)

    def predict_rows(self, n: int | None = None, start: int = 0):
        return self.rows(self.n_predict if n is None else n, self.predict_seed, start)

    def forest(self, cache_dir: str | None = None, n_threads: int = 0, progress=None) -> Forest:
        path = None
        if cache_dir:
            os.makedirs(cache_dir, exist_ok=True)
            path = os.path.join(cache_dir, f"forest_{self.name}.npz")
            if os.path.exists(path):
                return Forest.load(path)
        X, y = self.train_rows()
        f = train_forest(X, y, n_trees=self.n_trees, n_classes=self.n_classes, mtry=self.mtry,
                         max_depth=self.max_depth, bootstrap=True, seed=self.forest_seed,
                         n_threads=n_threads, progress=progress,
                         checkpoint=path[:-len(".npz")] if path else None)
        if path and _save_atomic(f, path):
            for name in os.listdir(cache_dir):  # the chunk files of this forest
                if name.startswith(f"forest_{self.name}.trees") and name.endswith(".npz"):
                    try:
                        os.remove(os.path.join(cache_dir, name))
                    except OSError:
                        pass
        return f


def _save_atomic(f: Forest, path: str) -> bool:
    """Save to a temporary name, then rename (np.savez appends .npz only when
    missing), so a reader never sees half a file.  A failure (a full disk)
    only costs the cache: it is reported and False returned."""
    try:
        f.save(path + ".tmp.npz")
        os.replace(path + ".tmp.npz", path)
        return True
    except OSError as e:
        print(f"[synth] forest cache not written ({e})", flush=True)
        if os.path.exists(path + ".tmp.npz"):
            os.remove(path + ".tmp.npz")
        return False


def small() -> Workload:
    """2-class Gaussian rows, 16 features; 32 trees, mtry 4, depth 12; 10k/10k rows."""
    return Workload("small", 16, 2, 32, 4, 12, 10_000, 10_000, 1, 2, 3, "mixture")


def image(n_train: int = 60_000, n_trees: int = 128, n_predict: int = 1_000_000) -> Workload:
    """784-pixel 10-class image rows; 128 trees, mtry 28, pure leaves; 60k train, 1M predict."""
    name = "image" if (n_train, n_trees) == (60_000, 128) else f"image_{n_train}_{n_trees}"
    return Workload(name, IMAGE_F, IMAGE_C, n_trees, 28, -1, n_train, n_predict, 101, 102, 103, "image")


def tabular(n_train: int = 1_000_000, n_trees: int = 1024, n_predict: int = 10_000_000,
            imbalanced: bool = False) -> Workload:
    """28-feature binary tabular rows; 1024 trees, mtry 5, min leaf 1; 1M train, 10M predict.
    imbalanced: about 10% positives (label logit shifted by 3.35), where the
    splits are more lopsided and Stat has more to gain (Sec. IV-C)."""
    name = "tabular" if (n_train, n_trees) == (1_000_000, 1024) else f"tabular_{n_train}_{n_trees}"
    if imbalanced:
        name += "_imb"
    return Workload(name, TAB_Z + TAB_P, 2, n_trees, 5, -1, n_train, n_predict, 201, 202, 203, "tabular",
                    shift=3.35 if imbalanced else 0.0)


@dataclass
class BatchedSpec:
    index: int
    n_trees: int
    n_features: int
    n_classes: int
    n_rows: int


def batched_spec(i: int) -> BatchedSpec:
    """Shape of forest i (0..63) of the 64-forest batched workload: trees, features
    and rows log-uniform in [16, 2048], [4, 784], [1, 200000]; classes uniform 2..10."""
    if i == 0:
        return BatchedSpec(0, 16, 4, 2, 1)
    if i == 63:
        return BatchedSpec(63, 2048, 784, 10, 200_000)
    rng = np.random.Generator(np.random.PCG64(10_000 + i))

    def logu(lo, hi):
        return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    T = logu(16, 2048)
    F = logu(4, 784)
    C = int(rng.integers(2, 11))
    N = logu(1, 200_000)
    return BatchedSpec(i, T, F, C, N)


def batched_workload(i: int) -> Workload:
    s = batched_spec(i)
    return Workload(f"batched_{i}", s.n_features, s.n_classes, s.n_trees,
                    max(1, int(math.isqrt(s.n_features))), 12, 10_000, s.n_rows,
                    30_000 + 2 * i, 30_001 + 2 * i, 20_000 + i, "mixture")
