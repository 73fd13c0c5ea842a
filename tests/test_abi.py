"""The C-ABI library loads and exports every entry point include/forestpack.h
declares; host-side argument checks work without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1806_07300_amd as fp
import synth

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "forestpack.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(fp_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 14
    L = ctypes.CDLL(fp.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_names_match_abi():
    for n in declared_functions():
        if n in ("fp_last_error", "fp_version"):
            continue
        assert hasattr(fp, n), f"python binding lacks {n}"


def test_version_and_error_strings():
    assert fp.fp_version().startswith("forestpack")
    with pytest.raises(fp.FPError) as e:
        fp.fp_pack_forest(synth.small().forest(), layout=9)
    assert "layout" in str(e.value)


def test_predict_host_checks_without_gpu():
    f = synth.small().forest()
    p = fp.fp_pack_forest(f, bin_size=8, interleave_depth=2)
    L = fp.lib()
    # n_rows == 0 is a no-op, even before upload
    assert L.fp_predict(p.handle, None, 0, 16, None, None, None) == fp.FP_OK
    # ld < n_features
    assert L.fp_predict(p.handle, ctypes.c_void_p(256), 4, 15, ctypes.c_void_p(256), None, None) == fp.FP_EINVAL
    assert "ld" in fp.fp_last_error()
    # NULL X with rows
    assert L.fp_predict(p.handle, None, 4, 16, ctypes.c_void_p(256), None, None) == fp.FP_EINVAL
    # not uploaded
    assert L.fp_predict(p.handle, ctypes.c_void_p(256), 4, 16, ctypes.c_void_p(256), None, None) == fp.FP_ENODEV
    # NULL forest
    assert L.fp_predict(None, None, 4, 16, None, None, None) == fp.FP_EINVAL
    # upload needs an aligned, big-enough buffer (checked before any HIP call)
    assert L.fp_packed_upload(p.handle, ctypes.c_void_p(257), 1 << 30, None) == fp.FP_EINVAL
    assert L.fp_packed_upload(p.handle, ctypes.c_void_p(256), 16, None) == fp.FP_E2BIG


def test_tune_roundtrip():
    p = fp.fp_pack_forest(synth.small().forest())
    fp.fp_packed_set_tune(p, {"rows_per_block": 8, "cursors": 4, "tree_groups": 2, "block_threads": 128})
    t = fp.fp_packed_get_tune(p)
    assert (t["rows_per_block"], t["cursors"], t["tree_groups"], t["block_threads"]) == (8, 4, 2, 128)
    fp.fp_packed_set_tune(p, None)
    assert all(v == 0 for v in fp.fp_packed_get_tune(p).values())
