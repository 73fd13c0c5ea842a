"""forestpack: packed decision-forest classification on MI355X (gfx950).

Thin ctypes binding over ``libforestpack.so`` (C ABI in include/forestpack.h).
Every function here has the name of the C entry point it calls and only
marshals arguments: packing runs in the library's C++ packer and every
prediction runs in the library's HIP kernels.  PyTorch is used for device
memory (tensors' ``data_ptr()``) and streams (``torch.cuda.current_stream()``).
If the library is missing, importing works but every call raises: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libforestpack.so")

FP_OK, FP_EINVAL, FP_ENOMEM, FP_EHIP, FP_ECORRUPT, FP_E2BIG, FP_EAGAIN, FP_ENOTREADY, FP_ENODEV = range(9)
FP_LAYOUT_NAIVE, FP_LAYOUT_PACKED, FP_LAYOUT_COMPACT, FP_LAYOUT_BLOCKED, FP_LAYOUT_CLUSTERED = 0, 1, 2, 3, 4
FP_ORDER_DEFAULT, FP_ORDER_DF = 0, 1
ERROR_NAMES = {0: "FP_OK", 1: "FP_EINVAL", 2: "FP_ENOMEM", 3: "FP_EHIP", 4: "FP_ECORRUPT",
               5: "FP_E2BIG", 6: "FP_EAGAIN", 7: "FP_ENOTREADY", 8: "FP_ENODEV"}


class FPError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# C structures (mirror include/forestpack.h)
# ---------------------------------------------------------------------------
_vp = ctypes.c_void_p
_i32, _i64 = ctypes.c_int32, ctypes.c_int64


class fp_forest_view(ctypes.Structure):
    _fields_ = [("n_trees", _i32), ("n_features", _i32), ("n_classes", _i32), ("reserved", _i32),
                ("tree_node_offset", _vp), ("feature", _vp), ("threshold", _vp), ("left", _vp),
                ("right", _vp), ("leaf_class", _vp), ("cardinality", _vp)]


class fp_pack_opts(ctypes.Structure):
    _fields_ = [("layout", _i32), ("bin_size", _i32), ("interleave_depth", _i32), ("line_align", _i32),
                ("node_order", _i32)]


class fp_packed_info(ctypes.Structure):
    _fields_ = [("layout", _i32), ("n_trees", _i32), ("n_features", _i32), ("n_classes", _i32),
                ("bin_size", _i32), ("interleave_depth", _i32), ("n_bins", _i32), ("max_top_nodes", _i32),
                ("n_nodes", _i64), ("n_internal", _i64), ("n_leaves", _i64), ("bytes", _i64),
                ("uploaded", _i32), ("max_depth", _i32), ("n_used_features", _i32), ("reserved", _i32),
                ("expected_depth", ctypes.c_double), ("mean_bias", ctypes.c_double),
                ("expected_fetches", ctypes.c_double)]


class fp_tune(ctypes.Structure):
    _fields_ = [("rows_per_block", _i32), ("cursors", _i32), ("tree_groups", _i32),
                ("block_threads", _i32), ("lds_top_nodes", _i32), ("feature_lds", _i32),
                ("refill_lanes", _i32), ("lds_bytes", _i32), ("tree_passes", _i32), ("reserved", _i32)]


TUNE_FIELDS = [f for f, _ in fp_tune._fields_ if f != "reserved"]


class fp_autotune_trial(ctypes.Structure):
    _fields_ = [("pack", fp_pack_opts), ("model_cost", ctypes.c_double), ("ms", ctypes.c_double)]


class fp_autotune_opts(ctypes.Structure):
    _fields_ = [("block_threads", _i32), ("cursors", _i32), ("reps", _i32), ("top_k", _i32),
                ("sample_rows", _i64), ("trials", ctypes.POINTER(fp_autotune_trial)), ("max_trials", _i32),
                ("reserved", _i32)]


class fp_autotune_result(ctypes.Structure):
    _fields_ = [("pack", fp_pack_opts), ("tune", fp_tune), ("best_ms", ctypes.c_double),
                ("default_ms", ctypes.c_double), ("n_tried", _i32), ("cache_hit", _i32),
                ("n_candidates", _i32), ("n_trials", _i32)]


class fp_job(ctypes.Structure):
    _fields_ = [("forest", _vp), ("X", _vp), ("n_rows", _i64), ("ld", _i64), ("votes", _vp), ("cls", _vp)]


class fp_plan_opts(ctypes.Structure):
    _fields_ = [("block_threads", _i32), ("cursors", _i32), ("use_graph", _i32), ("items_per_block", _i32),
                ("lds_budget", _i64), ("autotune", _i32), ("reserved", _i32)]


FP_EXECUTOR_HIP, FP_EXECUTOR_CPU_FAKE = 0, 1


class fp_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", _i64), ("max_rows_per_launch", _i64), ("max_inflight", _i32),
                ("max_queue", _i32), ("block_threads", _i32), ("cursors", _i32), ("max_retries", _i32),
                ("executor", _i32), ("fake_delay_us", _i32), ("fake_fail_every", _i32)]


class fp_serve_stats(ctypes.Structure):
    _fields_ = [("submitted", _i64), ("completed", _i64), ("rejected", _i64), ("launches", _i64), ("rows", _i64),
                ("pending", _i64), ("inflight", _i64), ("mean_ms", ctypes.c_double), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("mean_rows_per_launch", ctypes.c_double), ("elapsed_s", ctypes.c_double),
                ("failed_launches", _i64), ("retried", _i64), ("failed", _i64)]


class fp_plan_info(ctypes.Structure):
    _fields_ = [("n_jobs", _i32), ("n_items", _i32), ("blocks", _i32), ("block_threads", _i32),
                ("cursors", _i32), ("graph", _i32), ("lds_bytes", _i32), ("jobs_tuned", _i32),
                ("total_cost", ctypes.c_double), ("jobs_cached", _i32), ("reserved", _i32)]

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FPError(FP_ENODEV, "load", f"{LIB_PATH} is missing: run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "fp_last_error": ([], ctypes.c_char_p),
            "fp_version": ([], ctypes.c_char_p),
            "fp_pack_forest": ([ctypes.POINTER(fp_forest_view), ctypes.POINTER(fp_pack_opts), ctypes.POINTER(_vp)], ctypes.c_int),
            "fp_packed_info_get": ([_vp, ctypes.POINTER(fp_packed_info)], ctypes.c_int),
            "fp_packed_host_bytes": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
            "fp_packed_from_bytes": ([_vp, ctypes.c_size_t, ctypes.POINTER(_vp)], ctypes.c_int),
            "fp_packed_save": ([_vp, ctypes.c_char_p], ctypes.c_int),
            "fp_packed_load": ([ctypes.c_char_p, ctypes.POINTER(_vp)], ctypes.c_int),
            "fp_packed_upload": ([_vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
            "fp_infer_cardinality": ([ctypes.POINTER(fp_forest_view), _vp, _i64, _i64, _vp, _vp], ctypes.c_int),
            "fp_probe_stream": ([_vp, _vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double), _vp], ctypes.c_int),
            "fp_probe_gather": ([_vp, ctypes.c_uint64, _i32, _i32, _i32, ctypes.POINTER(ctypes.c_double), _vp],
                                ctypes.c_int),
            "fp_packed_free": ([_vp], None),
            "fp_packed_set_tune": ([_vp, ctypes.POINTER(fp_tune)], ctypes.c_int),
            "fp_packed_get_tune": ([_vp, ctypes.POINTER(fp_tune)], ctypes.c_int),
            "fp_predict": ([_vp, _vp, _i64, _i64, _vp, _vp, _vp], ctypes.c_int),
            "fp_predict_tuned": ([_vp, ctypes.POINTER(fp_tune), _vp, _i64, _i64, _vp, _vp, _vp], ctypes.c_int),
            "fp_tune_launch": ([_vp, _vp, _i64, _i64, _i32, _i32, ctypes.POINTER(fp_tune), _vp], ctypes.c_int),
            "fp_predict_tune_get": ([_vp, _i64, ctypes.POINTER(fp_tune), ctypes.POINTER(_i32)], ctypes.c_int),
            "fp_autotune": ([ctypes.POINTER(fp_forest_view), _vp, _i64, _i64, ctypes.POINTER(fp_autotune_opts),
                             ctypes.POINTER(fp_autotune_result), _vp], ctypes.c_int),
            "fp_plan_create": ([ctypes.POINTER(fp_job), _i32, ctypes.POINTER(fp_plan_opts), ctypes.POINTER(_vp)],
                               ctypes.c_int),
            "fp_predict_batched": ([_vp, _vp], ctypes.c_int),
            "fp_predict_batched_noalloc": ([ctypes.POINTER(fp_job), _i32, ctypes.POINTER(fp_plan_opts), _vp],
                                           ctypes.c_int),
            "fp_plan_info_get": ([_vp, ctypes.POINTER(fp_plan_info)], ctypes.c_int),
            "fp_plan_free": ([_vp], None),
            "fp_server_create": ([ctypes.POINTER(fp_server_opts), ctypes.POINTER(_vp)], ctypes.c_int),
            "fp_server_add_forest": ([_vp, _vp, ctypes.POINTER(_i32)], ctypes.c_int),
            "fp_serve_submit": ([_vp, _i32, _vp, _i64, _i64, _vp, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
            "fp_serve_poll": ([_vp, ctypes.c_uint64, _i64], ctypes.c_int),
            "fp_server_stats": ([_vp, ctypes.POINTER(fp_serve_stats)], ctypes.c_int),
            "fp_server_reset_stats": ([_vp], ctypes.c_int),
            "fp_server_destroy": ([_vp], None),
            "fp_serve_replay": ([_vp, _vp, _i64, _i32, _vp, _vp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != FP_OK:
        msg = lib().fp_last_error().decode(errors="replace")
        raise FPError(rc, where, msg)


def fp_last_error() -> str:
    return lib().fp_last_error().decode()


def fp_version() -> str:
    return lib().fp_version().decode()


# ---------------------------------------------------------------------------
# packed forest handle
# ---------------------------------------------------------------------------
class Packed:
    """Owns an ``fp_packed*`` and (after upload) the device tensor holding its bytes."""

    def __init__(self, handle: int):
        self.handle = _vp(handle)
        self.device_buffer = None  # torch uint8 tensor, kept alive while uploaded

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.fp_packed_free(h)
            self.handle = None

    @property
    def info(self) -> dict:
        return fp_packed_info_get(self)


def _view_from(forest):
    arrs = {}
    for k, dt in (("tree_node_offset", np.int64), ("feature", np.int32), ("threshold", np.float32),
                  ("left", np.int32), ("right", np.int32), ("leaf_class", np.int32)):
        arrs[k] = np.ascontiguousarray(getattr(forest, k), dtype=dt)
    card = getattr(forest, "cardinality", None)
    if card is not None:
        arrs["cardinality"] = np.ascontiguousarray(card, dtype=np.int64)
    v = fp_forest_view(int(forest.n_trees), int(forest.n_features), int(forest.n_classes), 0,
                       *(arrs[k].ctypes.data for k in ("tree_node_offset", "feature", "threshold",
                                                        "left", "right", "leaf_class")),
                       arrs["cardinality"].ctypes.data if card is not None else None)
    return v, arrs


def fp_pack_forest(forest, layout: int = FP_LAYOUT_PACKED, bin_size: int = 16,
                   interleave_depth: int = 3, line_align: int = 0, use_cardinality: bool = True,
                   node_order: int = FP_ORDER_DEFAULT) -> Packed:
    """Pack a trained forest (any object with the fp_forest_view arrays as attributes)."""
    if not use_cardinality:
        class _NoCard:
            pass
        f2 = _NoCard()
        for k in ("n_trees", "n_features", "n_classes", "tree_node_offset", "feature", "threshold",
                  "left", "right", "leaf_class"):
            setattr(f2, k, getattr(forest, k))
        f2.cardinality = None
        forest = f2
    view, keep = _view_from(forest)
    opts = fp_pack_opts(layout, bin_size, interleave_depth, line_align, node_order)
    out = _vp()
    _check(lib().fp_pack_forest(ctypes.byref(view), ctypes.byref(opts), ctypes.byref(out)), "fp_pack_forest")
    del keep
    return Packed(out.value)


def fp_packed_free(p: Packed) -> None:
    """Release the packed forest now (otherwise released when garbage collected)."""
    if p.handle is not None and p.handle.value:
        lib().fp_packed_free(p.handle)
    p.handle = None
    p.device_buffer = None


def fp_packed_info_get(p: Packed) -> dict:
    info = fp_packed_info()
    _check(lib().fp_packed_info_get(p.handle, ctypes.byref(info)), "fp_packed_info_get")
    return {f: getattr(info, f) for f, _ in fp_packed_info._fields_}


def fp_packed_host_bytes(p: Packed) -> np.ndarray:
    ptr, n = _vp(), ctypes.c_size_t()
    _check(lib().fp_packed_host_bytes(p.handle, ctypes.byref(ptr), ctypes.byref(n)), "fp_packed_host_bytes")
    return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctypes.c_uint8)), (n.value,)).copy()


def fp_packed_from_bytes(buf) -> Packed:
    b = np.ascontiguousarray(np.frombuffer(buf, np.uint8) if not isinstance(buf, np.ndarray) else buf, np.uint8)
    out = _vp()
    _check(lib().fp_packed_from_bytes(b.ctypes.data, b.nbytes, ctypes.byref(out)), "fp_packed_from_bytes")
    return Packed(out.value)


def fp_packed_save(p: Packed, path: str) -> None:
    _check(lib().fp_packed_save(p.handle, path.encode()), "fp_packed_save")


def fp_packed_load(path: str) -> Packed:
    out = _vp()
    _check(lib().fp_packed_load(path.encode(), ctypes.byref(out)), "fp_packed_load")
    return Packed(out.value)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


def fp_packed_upload(p: Packed, dev_tensor=None, stream=None) -> Packed:
    """Copy the packed bytes to the GPU; allocates a torch uint8 buffer unless one is given."""
    import torch
    nbytes = fp_packed_info_get(p)["bytes"]
    if dev_tensor is None:
        dev_tensor = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    if not dev_tensor.is_cuda or dev_tensor.dtype != torch.uint8:
        raise FPError(FP_EINVAL, "fp_packed_upload", "device buffer must be a CUDA uint8 tensor")
    cap = dev_tensor.numel()
    _check(lib().fp_packed_upload(p.handle, _vp(dev_tensor.data_ptr()), cap, _stream_ptr(stream)),
           "fp_packed_upload")
    p.device_buffer = dev_tensor
    return p


def _tune_struct(tune):
    if tune is None:
        return None
    if isinstance(tune, fp_tune):
        return tune
    t = fp_tune()
    for k, v in dict(tune).items():
        if k not in TUNE_FIELDS:
            raise FPError(FP_EINVAL, "fp_tune", f"unknown field {k}")
        setattr(t, k, int(v))
    return t


def fp_packed_set_tune(p: Packed, tune) -> None:
    t = _tune_struct(tune)
    _check(lib().fp_packed_set_tune(p.handle, ctypes.byref(t) if t is not None else None), "fp_packed_set_tune")


def fp_packed_get_tune(p: Packed) -> dict:
    t = fp_tune()
    _check(lib().fp_packed_get_tune(p.handle, ctypes.byref(t)), "fp_packed_get_tune")
    return {k: getattr(t, k) for k in TUNE_FIELDS}


def _check_rows(X, n_features):
    import torch
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float32 and X.dim() == 2):
        raise FPError(FP_EINVAL, "fp_predict", "X must be a 2-D float32 CUDA tensor")
    n = X.shape[0]
    if n == 0:
        return 0, max(X.shape[1], n_features)
    if X.shape[1] > 1 and X.stride(1) != 1:
        raise FPError(FP_EINVAL, "fp_predict", "X rows must be contiguous (stride(1) == 1)")
    ld = X.stride(0) if n > 1 else X.shape[1]
    return n, ld


def _outputs(n, C, votes, cls, want_cls):
    import torch
    if votes is None:
        votes = torch.empty((n, C), dtype=torch.int32, device="cuda")
    if cls is None and want_cls:
        cls = torch.empty((n,), dtype=torch.int32, device="cuda")
    return votes, cls


def fp_predict(p: Packed, X, votes=None, cls=None, stream=None, want_cls: bool = True):
    """votes int32 [n, C] and argmax class int32 [n] (CUDA tensors) for rows X (CUDA fp32 [n, >=F])."""
    info = fp_packed_info_get(p)
    n, ld = _check_rows(X, info["n_features"])
    votes, cls = _outputs(n, info["n_classes"], votes, cls, want_cls)
    _check(lib().fp_predict(p.handle, _vp(X.data_ptr()), n, ld, _vp(votes.data_ptr()),
                            _vp(cls.data_ptr()) if cls is not None else None, _stream_ptr(stream)), "fp_predict")
    return votes, cls


def fp_predict_tuned(p: Packed, tune, X, votes=None, cls=None, stream=None, want_cls: bool = True):
    """fp_predict with explicit launch parameters (dict with fp_tune fields)."""
    info = fp_packed_info_get(p)
    n, ld = _check_rows(X, info["n_features"])
    votes, cls = _outputs(n, info["n_classes"], votes, cls, want_cls)
    t = _tune_struct(tune)
    _check(lib().fp_predict_tuned(p.handle, ctypes.byref(t) if t is not None else None, _vp(X.data_ptr()), n, ld,
                                  _vp(votes.data_ptr()), _vp(cls.data_ptr()) if cls is not None else None,
                                  _stream_ptr(stream)), "fp_predict_tuned")
    return votes, cls


def fp_tune_launch(p: Packed, X, block_threads: int = 0, cursors: int = 0, stream=None) -> dict:
    """Time launch candidates of p on rows X (CUDA fp32) and record the fastest
    for X's size bucket (process table, and the FP_TUNE_CACHE file if set)."""
    info = fp_packed_info_get(p)
    n, ld = _check_rows(X, info["n_features"])
    t = fp_tune()
    _check(lib().fp_tune_launch(p.handle, _vp(X.data_ptr()), n, ld, block_threads, cursors, ctypes.byref(t),
                                _stream_ptr(stream)), "fp_tune_launch")
    return {k: getattr(t, k) for k in TUNE_FIELDS}


def fp_predict_tune_get(p: Packed, n_rows: int):
    """(tune dict, source) fp_predict would use for n_rows rows: source 2 a
    recorded tune, 1 the forest's own, 0 library defaults."""
    t, src = fp_tune(), _i32()
    _check(lib().fp_predict_tune_get(p.handle, n_rows, ctypes.byref(t), ctypes.byref(src)), "fp_predict_tune_get")
    return {k: getattr(t, k) for k in TUNE_FIELDS}, src.value


def fp_infer_cardinality(forest, X, stream=None):
    """Per-node counts of the rows of X (CUDA fp32 [n, >= F]) that reach each
    node, int64 [tree_node_offset[T]]: a forest's access statistics inferred
    from observations, for fp_pack_forest's Stat order."""
    view, keep = _view_from(forest)
    n, ld = _check_rows(X, int(forest.n_features))
    card = np.zeros(int(np.asarray(forest.tree_node_offset)[-1]), np.int64)
    _check(lib().fp_infer_cardinality(ctypes.byref(view), _vp(X.data_ptr()), n, ld, _vp(card.ctypes.data),
                                      _stream_ptr(stream)), "fp_infer_cardinality")
    del keep
    return card


def fp_probe_stream(src, dst, stream=None) -> float:
    """HBM stream rate in GB/s (read + write) of copying CUDA tensor src into dst."""
    nbytes = min(src.numel() * src.element_size(), dst.numel() * dst.element_size()) // 16 * 16
    out = ctypes.c_double(0.0)
    _check(lib().fp_probe_stream(_vp(src.data_ptr()), _vp(dst.data_ptr()), nbytes, ctypes.byref(out),
                                 _stream_ptr(stream)), "fp_probe_stream")
    return out.value


def fp_probe_gather(buf, fetch_bytes: int = 16, chains: int = 1, steps: int = 256, stream=None) -> float:
    """Dependent random fetches per second through CUDA tensor buf (overwritten)."""
    out = ctypes.c_double(0.0)
    _check(lib().fp_probe_gather(_vp(buf.data_ptr()), buf.numel() * buf.element_size(), fetch_bytes, chains, steps,
                                 ctypes.byref(out), _stream_ptr(stream)), "fp_probe_gather")
    return out.value


# ---------------------------------------------------------------------------
# autotuning
# ---------------------------------------------------------------------------
def fp_autotune(forest, X, block_threads: int = 0, cursors: int = 0, reps: int = 3, sample_rows: int = 0,
                top_k: int = 0, stream=None) -> dict:
    """Score candidate packings with the cost model, time the best few per
    layout and search the launch mapping of the fastest, on rows X (CUDA
    fp32); returns {"pack": {...}, "tune": {...}, "best_ms", "default_ms",
    "n_tried", "cache_hit", "trials": [{"pack", "model_cost", "ms"}, ...]}."""
    view, keep = _view_from(forest)
    n, ld = _check_rows(X, int(forest.n_features))
    cap = 256
    trials = (fp_autotune_trial * cap)()
    opts = fp_autotune_opts(block_threads, cursors, reps, top_k, sample_rows, trials, cap, 0)
    res = fp_autotune_result()
    _check(lib().fp_autotune(ctypes.byref(view), _vp(X.data_ptr()), n, ld, ctypes.byref(opts), ctypes.byref(res),
                             _stream_ptr(stream)), "fp_autotune")
    del keep
    pk = lambda p: {"layout": p.layout, "bin_size": p.bin_size, "interleave_depth": p.interleave_depth,
                    "line_align": p.line_align}
    return {"pack": pk(res.pack), "tune": {k: getattr(res.tune, k) for k in TUNE_FIELDS},
            "best_ms": res.best_ms, "default_ms": res.default_ms, "n_tried": res.n_tried,
            "cache_hit": bool(res.cache_hit), "n_candidates": res.n_candidates,
            "trials": [{"pack": pk(trials[i].pack), "model_cost": trials[i].model_cost, "ms": trials[i].ms}
                       for i in range(res.n_trials)]}


# ---------------------------------------------------------------------------
# batched plans
# ---------------------------------------------------------------------------
class Plan:
    """Owns an ``fp_plan*``; keeps the jobs' forests and tensors alive."""

    def __init__(self, handle, keep):
        self.handle = _vp(handle)
        self._keep = keep

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.fp_plan_free(h)
            self.handle = None


def fp_plan_create(jobs, block_threads: int = 0, cursors: int = 0, use_graph: bool = True,
                   items_per_block: int = 0, lds_budget: int = 0, autotune: bool = False,
                   default_opts: bool = False) -> Plan:
    """jobs: list of (Packed, X, votes, cls-or-None) with CUDA tensors; pointers are fixed in the plan.
    default_opts passes NULL options (library defaults, autotune on)."""
    arr = (fp_job * len(jobs))()
    keep = []
    for i, (p, X, votes, cls) in enumerate(jobs):
        n, ld = _check_rows(X, fp_packed_info_get(p)["n_features"])
        arr[i] = fp_job(p.handle.value, X.data_ptr(), n, ld, votes.data_ptr(),
                        cls.data_ptr() if cls is not None else None)
        keep.append((p, X, votes, cls))
    opts = fp_plan_opts(block_threads, cursors, int(bool(use_graph)), items_per_block, lds_budget,
                        int(bool(autotune)), 0)
    out = _vp()
    _check(lib().fp_plan_create(arr, len(jobs), None if default_opts else ctypes.byref(opts), ctypes.byref(out)),
           "fp_plan_create")
    return Plan(out.value, keep)


def fp_predict_batched_noalloc(jobs, block_threads: int = 0, cursors: int = 0, items_per_block: int = 0,
                               lds_budget: int = 0, stream=None) -> None:
    """One batched run of jobs [(Packed, X, votes, cls-or-None)] that
    allocates no device memory (tables in the library's static scratch)."""
    arr = (fp_job * len(jobs))()
    for i, (p, X, votes, cls) in enumerate(jobs):
        n, ld = _check_rows(X, fp_packed_info_get(p)["n_features"])
        arr[i] = fp_job(p.handle.value, X.data_ptr(), n, ld, votes.data_ptr(),
                        cls.data_ptr() if cls is not None else None)
    opts = fp_plan_opts(block_threads, cursors, 0, items_per_block, lds_budget, 0, 0)
    _check(lib().fp_predict_batched_noalloc(arr, len(jobs), ctypes.byref(opts), _stream_ptr(stream)),
           "fp_predict_batched_noalloc")


def fp_predict_batched(plan: Plan, stream=None) -> None:
    _check(lib().fp_predict_batched(plan.handle, _stream_ptr(stream)), "fp_predict_batched")


def fp_plan_info_get(plan: Plan) -> dict:
    info = fp_plan_info()
    _check(lib().fp_plan_info_get(plan.handle, ctypes.byref(info)), "fp_plan_info_get")
    return {f: getattr(info, f) for f, _ in fp_plan_info._fields_ if f != "reserved"}


def fp_plan_free(plan: Plan) -> None:
    if plan.handle is not None and plan.handle.value:
        lib().fp_plan_free(plan.handle)
    plan.handle = None
    plan._keep = None


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------
class Server:
    """Owns an ``fp_server*``; keeps forests and pending output buffers alive."""

    def __init__(self, handle):
        self.handle = _vp(handle)
        self.forests = []
        self.outputs = {}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.fp_server_destroy(h)
            self.handle = None


def fp_server_create(hbm_budget_bytes: int = 0, max_rows_per_launch: int = 0, max_inflight: int = 0,
                     max_queue: int = 0, block_threads: int = 0, cursors: int = 0, max_retries: int = 0,
                     executor: int = FP_EXECUTOR_HIP, fake_delay_us: int = 0, fake_fail_every: int = 0) -> Server:
    opts = fp_server_opts(hbm_budget_bytes, max_rows_per_launch, max_inflight, max_queue, block_threads, cursors,
                          max_retries, executor, fake_delay_us, fake_fail_every)
    out = _vp()
    _check(lib().fp_server_create(ctypes.byref(opts), ctypes.byref(out)), "fp_server_create")
    return Server(out.value)


def fp_server_add_forest(server: Server, p: Packed) -> int:
    fid = _i32()
    _check(lib().fp_server_add_forest(server.handle, p.handle, ctypes.byref(fid)), "fp_server_add_forest")
    server.forests.append(p)
    return fid.value


def fp_serve_submit(server: Server, forest_id: int, X: np.ndarray, votes_out: np.ndarray) -> int:
    """Queue rows X (host fp32 [n, >=F], row-major); votes_out (host int32 [n, C],
    C-contiguous) is filled once fp_serve_poll reports the ticket ready."""
    if X.dtype != np.float32 or X.ndim != 2 or (X.shape[0] > 1 and X.strides[1] != 4):
        raise FPError(FP_EINVAL, "fp_serve_submit", "X must be a row-major float32 matrix")
    if votes_out.dtype != np.int32 or not votes_out.flags["C_CONTIGUOUS"]:
        raise FPError(FP_EINVAL, "fp_serve_submit", "votes_out must be a C-contiguous int32 array")
    n = X.shape[0]
    ld = X.strides[0] // 4 if n > 1 else X.shape[1]
    t = ctypes.c_uint64()
    _check(lib().fp_serve_submit(server.handle, forest_id, X.ctypes.data, n, ld, votes_out.ctypes.data,
                                 ctypes.byref(t)), "fp_serve_submit")
    server.outputs[t.value] = votes_out
    return t.value


def fp_serve_poll(server: Server, ticket: int, timeout_us: int = -1) -> bool:
    """True once the ticket's votes are written (the ticket is then retired)."""
    rc = lib().fp_serve_poll(server.handle, ticket, timeout_us)
    if rc == FP_ENOTREADY:
        return False
    server.outputs.pop(ticket, None)
    _check(rc, "fp_serve_poll")
    return True


def fp_server_stats(server: Server) -> dict:
    st = fp_serve_stats()
    _check(lib().fp_server_stats(server.handle, ctypes.byref(st)), "fp_server_stats")
    return {f: getattr(st, f) for f, _ in fp_serve_stats._fields_}


def fp_server_reset_stats(server: Server) -> None:
    _check(lib().fp_server_reset_stats(server.handle), "fp_server_reset_stats")


def fp_server_destroy(server: Server) -> None:
    if server.handle is not None and server.handle.value:
        lib().fp_server_destroy(server.handle)
    server.handle = None
    server.outputs.clear()


REPLAY_DTYPE = np.dtype([("forest_id", "<i4"), ("reserved", "<i4"), ("X", "<u8"), ("n_rows", "<i8"),
                         ("ld", "<i8"), ("votes", "<u8"), ("arrival_s", "<f8")])


def fp_serve_replay(server: Server, reqs: np.ndarray, submit_threads: int = 2):
    """Open-loop replay of a request schedule (structured array of REPLAY_DTYPE
    whose X / votes fields are host addresses the caller keeps alive).
    Returns (latency_ms, lag_ms) per request: ready - scheduled arrival, and
    actual submit - scheduled arrival."""
    reqs = np.ascontiguousarray(reqs, dtype=REPLAY_DTYPE)
    n = len(reqs)
    lat = np.zeros(n, np.float64)
    lag = np.zeros(n, np.float64)
    _check(lib().fp_serve_replay(server.handle, reqs.ctypes.data if n else None, n, submit_threads,
                                 lat.ctypes.data, lag.ctypes.data), "fp_serve_replay")
    return lat, lag
