"""The tune-cache file (FP_TUNE_CACHE) on the CPU: records written by one
process are read by another, keyed by the forest's bytes and the batch-size
bucket ceil(log2 n_rows); later lines win; malformed lines are skipped; a
forest packed differently does not match.  fp_predict_tune_get shows the
tune fp_predict would use, which needs no GPU."""
import os
import subprocess
import sys

import numpy as np

import paper_1806_07300_amd as fp
import synth
from packed_format import decode

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
M64 = (1 << 64) - 1


def forest_key(p):
    """The table's key for a packed forest, restated: its checksum and size
    and layout mixed FNV-style."""
    h = decode(fp.fp_packed_host_bytes(p))["h"]
    k = (int(h["checksum"]) ^ 0x9E3779B97F4A7C15) & M64
    for v in (int(h["total_bytes"]), int(h["layout"]) & 0xFFFFFFFF):
        k = ((k ^ v) * 0x100000001B3) & M64
    return k


CHILD = r"""
import sys, json
sys.path.insert(0, {root!r})
import synth, paper_1806_07300_amd as fp
f = synth.small().forest()
p = fp.fp_pack_forest(f, layout={layout}, bin_size=8, interleave_depth=3)
print(json.dumps([fp.fp_predict_tune_get(p, n) for n in (1, 3000, 4096, 4097, 10000)]))
"""


def run_child(path, layout):
    env = dict(os.environ, FP_TUNE_CACHE=path)
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, layout=layout)], env=env,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    import json
    return json.loads(r.stdout.strip().splitlines()[-1])


def _line(key, bucket, threads, cursors, tune):
    return f"L {key:016x} {bucket} {threads} {cursors} " + " ".join(map(str, tune)) + "\n"


TUNE_A = [64, 1, 1, 1024, 0, 1, 32, 0, 2]
TUNE_B = [16, 2, 2, 512, -1, 0, 16, 0, 1]


def test_records_are_read_back_by_bucket(tmp_path):
    f = synth.small().forest()
    p = fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=8, interleave_depth=3)
    key = forest_key(p)
    path = str(tmp_path / "tunes.txt")
    with open(path, "w") as fh:
        fh.write(_line(key, 12, 0, 0, TUNE_A))        # 2,049 .. 4,096 rows
        fh.write("L garbage line\n")
        fh.write(_line(key, 13, 0, 0, TUNE_A))        # 4,097 .. 8,192 rows
        fh.write(_line(key, 13, 0, 0, TUNE_B))        # a later line wins
        fh.write(_line(key, 14, 1024, 2, TUNE_A))     # a plan's key (threads, cursors fixed): not fp_predict's
        fh.write(_line(key, 12, 0, 0, TUNE_B)[:-12] + "\n")   # truncated: skipped
        fh.write("A 12ab 1 2 3\n")                    # malformed autotune record: skipped
    got = run_child(path, fp.FP_LAYOUT_CLUSTERED)
    a, b = dict(zip(fp.TUNE_FIELDS, TUNE_A)), dict(zip(fp.TUNE_FIELDS, TUNE_B))
    assert got[0][1] != 2                 # 1 row: bucket 0, nothing recorded
    assert got[1] == [a, 2]               # 3,000 rows: bucket 12
    assert got[2] == [a, 2]               # 4,096 rows: still bucket 12
    assert got[3] == [b, 2]               # 4,097 rows: bucket 13, the later line
    assert got[4][1] != 2                 # 10,000 rows: bucket 14 has only the plan's record


def test_another_packing_of_the_forest_does_not_match(tmp_path):
    f = synth.small().forest()
    p = fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=8, interleave_depth=3)
    path = str(tmp_path / "tunes.txt")
    with open(path, "w") as fh:
        fh.write(_line(forest_key(p), 12, 0, 0, TUNE_A))
    got = run_child(path, fp.FP_LAYOUT_BLOCKED)
    assert all(src != 2 for _, src in got)
    got = run_child(path, fp.FP_LAYOUT_CLUSTERED)
    assert got[1][1] == 2 and got[3][1] != 2


def test_no_file_no_records(tmp_path):
    got = run_child(str(tmp_path / "absent.txt"), fp.FP_LAYOUT_CLUSTERED)
    assert all(src != 2 for _, src in got)
