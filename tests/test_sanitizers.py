"""Host code under the sanitizers, on the CPU: the packer (with a fuzz of
mutated packed buffers and malformed forests) built with AddressSanitizer
and UndefinedBehaviorSanitizer, and the serving scheduler on the CPU fake
executor built with ThreadSanitizer.  The drivers live in tests/native; the
library's device operations are replaced by stand-ins that report no device.
Built with ROCm's clang (it has the sanitizer runtimes and _Float16 on x86)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1806_07300_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
CLANG = "/opt/rocm/llvm/bin/clang++"

pytestmark = pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang++ not found")


def write_forest(path, f):
    with open(path, "wb") as fh:
        np.array([f.n_trees, f.n_features, f.n_classes], np.int32).tofile(fh)
        np.asarray(f.tree_node_offset, np.int64).tofile(fh)
        for k, dt in (("feature", np.int32), ("threshold", np.float32), ("left", np.int32), ("right", np.int32),
                      ("leaf_class", np.int32), ("cardinality", np.int64)):
            np.asarray(getattr(f, k), dt).tofile(fh)


@pytest.fixture(scope="module")
def forest_file(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    X, y = synth.gaussian_mixture(2000, 12, 4, seed=41)
    f = synth.train_forest(X, y, n_trees=12, n_classes=4, mtry=3, max_depth=10, seed=42)
    path = str(d / "forest.bin")
    write_forest(path, f)
    return path, d


def build(out, sanitize, sources):
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={sanitize}",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           "-I" + NATIVE, *sources, "-o", out, "-lpthread"]
    if "undefined" in sanitize:
        cmd.insert(5, "-fno-sanitize-recover=undefined")
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]


def test_packer_under_asan_ubsan(forest_file):
    path, d = forest_file
    exe = str(d / "pack_fuzz")
    build(exe, "address,undefined", [os.path.join(CSRC, "pack.cpp"), os.path.join(NATIVE, "pack_fuzz.cpp"),
                                     os.path.join(NATIVE, "device_stubs.cpp")])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, path, str(d), "200"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert "malformed views refused" in r.stdout


def test_server_under_tsan(forest_file):
    path, d = forest_file
    exe = str(d / "serve_tsan")
    build(exe, "thread", [os.path.join(CSRC, "serve.cpp"), os.path.join(CSRC, "pack.cpp"),
                          os.path.join(NATIVE, "serve_tsan.cpp"), os.path.join(NATIVE, "device_stubs.cpp")])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    r = subprocess.run([exe, path], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "WARNING: ThreadSanitizer" not in r.stderr
    assert "0 wrong" in r.stdout
