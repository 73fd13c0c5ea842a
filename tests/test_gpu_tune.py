"""GPU tests of launch tuning at the boundary: fp_tune_launch records a tune
per (forest bytes, batch-size bucket); fp_predict then uses it; a batched
plan created with NULL options tunes its jobs or takes their recorded tunes;
with FP_TUNE_CACHE the records reach a second process through the file.
Votes always equal the CPU checker's."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_1806_07300_amd as fp
import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def forest_and_rows(i, n):
    Xt, yt = synth.gaussian_mixture(3000, 9 + i, 3, seed=900 + i)
    f = synth.train_forest(Xt, yt, n_trees=24 + 8 * i, n_classes=3, mtry=3, max_depth=10, seed=910 + i)
    X, _ = synth.gaussian_mixture(n, 9 + i, 3, seed=920 + i)
    return f, X


def test_tune_launch_is_used_per_bucket():
    f, X = forest_and_rows(0, 5000)
    want = oracle.predict(f, X)
    p = fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=8, interleave_depth=3)
    fp.fp_packed_upload(p)
    fp.fp_packed_set_tune(p, {"rows_per_block": 8, "cursors": 1})
    Xd = torch.from_numpy(X).cuda()
    assert fp.fp_predict_tune_get(p, 5000)[1] == 1  # the forest's own tune until one is recorded
    t = fp.fp_tune_launch(p, Xd)
    assert t["rows_per_block"] > 0 and t["block_threads"] > 0
    got, src = fp.fp_predict_tune_get(p, 5000)
    assert src == 2 and got == t
    assert fp.fp_predict_tune_get(p, 4097)[1] == 2      # same bucket: (4096, 8192]
    assert fp.fp_predict_tune_get(p, 4096)[1] == 1      # another bucket
    v, c = fp.fp_predict(p, Xd)
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy(), want[0]) and np.array_equal(c.cpu().numpy(), want[1])
    # a tiny batch gets its own record
    t1 = fp.fp_tune_launch(p, Xd[:3])
    assert fp.fp_predict_tune_get(p, 3) == (t1, 2)
    v, c = fp.fp_predict(p, Xd[:3])
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy(), want[0][:3])


def test_tune_launch_errors():
    f, X = forest_and_rows(1, 100)
    naive = fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_NAIVE)
    fp.fp_packed_upload(naive)
    with pytest.raises(fp.FPError) as e:
        fp.fp_tune_launch(naive, torch.from_numpy(X).cuda())
    assert e.value.code == fp.FP_EINVAL
    p = fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_PACKED, bin_size=4, interleave_depth=2)
    fp.fp_packed_upload(p)
    with pytest.raises(fp.FPError) as e:
        fp.fp_tune_launch(p, torch.from_numpy(X).cuda(), block_threads=100)
    assert e.value.code == fp.FP_EINVAL


def plan_jobs(layouts=(fp.FP_LAYOUT_CLUSTERED, fp.FP_LAYOUT_PACKED, fp.FP_LAYOUT_BLOCKED)):
    jobs = []
    for i, layout in enumerate(layouts):
        f, X = forest_and_rows(2 + i, 700 + 900 * i)
        p = fp.fp_pack_forest(f, layout=layout, bin_size=8, interleave_depth=3)
        fp.fp_packed_upload(p)
        Xd = torch.from_numpy(X).cuda()
        jobs.append({"forest": f, "X": X, "packed": p, "Xd": Xd,
                     "votes": torch.full((len(X), 3), -1, dtype=torch.int32, device="cuda"),
                     "cls": torch.full((len(X),), -1, dtype=torch.int32, device="cuda")})
    return jobs


def check(jobs):
    torch.cuda.synchronize()
    for j in jobs:
        wv, wc = oracle.predict(j["forest"], j["X"])
        assert np.array_equal(j["votes"].cpu().numpy(), wv) and np.array_equal(j["cls"].cpu().numpy(), wc)


def test_plan_with_null_options_tunes_then_reuses():
    jobs = plan_jobs()
    plan = fp.fp_plan_create([(j["packed"], j["Xd"], j["votes"], j["cls"]) for j in jobs], default_opts=True)
    info = fp.fp_plan_info_get(plan)
    assert info["block_threads"] == 1024 and info["cursors"] == 2 and info["graph"] == 1
    assert info["jobs_tuned"] + info["jobs_cached"] == len(jobs)
    for _ in range(2):
        fp.fp_predict_batched(plan)
        check(jobs)
        for j in jobs:
            j["votes"].fill_(-1)
            j["cls"].fill_(-1)
    again = fp.fp_plan_create([(j["packed"], j["Xd"], j["votes"], j["cls"]) for j in jobs], default_opts=True)
    info = fp.fp_plan_info_get(again)
    assert info["jobs_tuned"] == 0 and info["jobs_cached"] == len(jobs)
    fp.fp_predict_batched(again)
    check(jobs)


CHILD = r"""
import json, sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import torch, paper_1806_07300_amd as fp
import test_gpu_tune as t
jobs = t.plan_jobs()
plan = fp.fp_plan_create([(j["packed"], j["Xd"], j["votes"], j["cls"]) for j in jobs], default_opts=True)
fp.fp_predict_batched(plan)
t.check(jobs)
p = jobs[0]["packed"]
print(json.dumps({{"info": fp.fp_plan_info_get(plan), "predict_source": fp.fp_predict_tune_get(p, 700)[1]}}))
"""


def test_tune_cache_file_reaches_a_second_process(tmp_path):
    path = str(tmp_path / "tunes.txt")
    env = dict(os.environ, FP_TUNE_CACHE=path)
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"))
    outs = []
    for k in range(2):
        print(f"[tune] child process {k + 1}", flush=True)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(json.loads(r.stdout.strip().splitlines()[-1]))
    assert outs[0]["info"]["jobs_tuned"] == 3 and outs[0]["info"]["jobs_cached"] == 0
    assert outs[1]["info"]["jobs_tuned"] == 0 and outs[1]["info"]["jobs_cached"] == 3
    assert outs[0]["predict_source"] != 2  # plans record tunes for their own workgroup size and cursors
    lines = open(path).read().splitlines()
    assert len(lines) == 3 and all(l.startswith("L ") for l in lines)
