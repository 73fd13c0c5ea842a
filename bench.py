#!/usr/bin/env python3
"""Benchmark: forest classification throughput, packed vs naive layout, one MI355X.

A step is one pass of the whole hot path over one batch: every observation of
the batch walks every tree of the resident packed forest, and its votes and
class are written (fp_predict).  The headline workload is the large binary
tabular one: 10,000,000 rows of 28 fp32 features through 1,024 trees grown
to pure leaves on 1,000,000 rows, packed in bins of 16 trees (the
Higgs-shaped comparison of Sec. IV-B, Table I).  Rows are resident in HBM
before timing starts.  Prints one JSON line; the other workloads (the small
two-class case, the image-shaped forest, 64 batched forests in one graph
launch, the serving mix) are extra keys of the same line.

  python bench.py [--gpus 1] [--steps K] [--warmup W]

Extra modes:
  --only packed|naive|copy [--workload tabular|image|small]
                             run only that kernel, --steps times, no JSON
                             (profiling runs under rocprofv3)
  --ladder image|tabular|tabular_imb
                             the layout ablation of Sec. III-A (Fig. 4): BF,
                             DF, DF-, Stat (training statistics), Stat-obs
                             (statistics inferred from 100,000 of the rows),
                             Bin, Bin+, then the block layouts, same rows and
                             forest, every rung checked bit for bit against
                             BF; tabular_imb is the 10%-positive variant
                             (128 trees); prints one JSON line
  --probes                   the ceilings: HBM stream rate, dependent random
                             gathers (16/48-byte fetches, 1-4 chains per lane)
                             against working-set size, host-to-device copy
                             rate, and the naive kernel's workgroup-size sweep
                             on the image workload; prints one JSON line
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "observations/sec packed vs naive layout on 1 MI355X (bit-exact); p99 serve ms"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1806_07300_amd", "csrc", "traverse.hip")
LAYOUT_NAMES = {0: "naive", 1: "packed", 2: "compact", 3: "blocked", 4: "clustered"}
T_START = time.perf_counter()


def log(*a):
    print(f"[bench {time.perf_counter() - T_START:6.1f}s]", *a, file=sys.stderr, flush=True)


def elapsed() -> float:
    return time.perf_counter() - T_START


class Progress:
    """Training progress printed every 64 trees (training the 1,024-tree
    forest takes minutes of host time)."""
    chunk = 64

    def __init__(self, name):
        self.name = name

    def __call__(self, done, total):
        log(f"{self.name}: trained {done}/{total} trees")


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"packed_kernel_{workload}_traffic.txt")


def read_traffic_record(workload: str, tune: dict | None = None) -> dict | None:
    """The workload's counter record (profiles/packed_kernel_<workload>_traffic.txt)
    as a dict, or None when missing, taken on a different kernel source, or
    (when the record names its launch) with a launch other than `tune`."""
    path = traffic_file(workload)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    if tune is not None and "launch" in vals:
        try:
            if json.loads(vals["launch"]) != tune:
                return None
        except ValueError:
            return None
    return vals


def read_traffic(workload: str, tune: dict | None = None):
    """HBM bytes per step of the workload's packed kernel (all the step's
    launches: one per tree pass) measured by rocprofv3 --pmc (FETCH_SIZE,
    WRITE_SIZE, scaled by a copy-kernel calibration); None when the record
    is missing or does not match (read_traffic_record)."""
    vals = read_traffic_record(workload, tune)
    if vals is None:
        return None
    try:
        if "fetch_bytes_per_step" in vals:
            return float(vals["fetch_bytes_per_step"]) + float(vals["write_bytes_per_step"])
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_steps(fn, steps, warmup, torch):
    """Average ms per call of fn over `steps` calls after `warmup` calls, from
    HIP events recorded on the stream the kernels are launched on."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / max(steps, 1), wall


def cpu_baseline(forest, X, gpu_votes, gpu_cls, target_s=20.0):
    """The CPU checker, as it stands, on a bounded sample of the same batch
    (the first rows, sized for about `target_s` seconds of host time), and the
    GPU's votes and classes on those rows compared with it bit for bit."""
    import numpy as np
    import oracle
    n_threads = os.cpu_count() or 1
    n = min(len(X), 2_000)
    t0 = time.perf_counter()
    oracle.predict(forest, X[:n], n_threads=n_threads)
    dt = time.perf_counter() - t0
    m = min(len(X), max(n, int(n * target_s / max(dt, 1e-3))))
    t0 = time.perf_counter()
    votes, cls, visits = oracle.predict(forest, X[:m], n_threads=n_threads, return_visits=True)
    dt = time.perf_counter() - t0
    exact = bool(np.array_equal(votes, gpu_votes[:m]) and np.array_equal(cls, gpu_cls[:m]))
    return {"value": m / dt, "unit": "observations/s", "cores": n_threads, "kind": "oracle",
            "sample": f"first {m} rows of the batch, all {n_threads} host threads, {dt:.1f} s"}, \
        {"rows": m, "bit_exact": exact}, visits / m


def pack(fp, forest, **kw):
    t0 = time.perf_counter()
    p = fp.fp_pack_forest(forest, **kw)
    dt = time.perf_counter() - t0
    fp.fp_packed_upload(p)
    return p, dt


def single_forest_leg(name, w, preset, args, fp, torch, np, steps, warmup, naive_steps, with_cpu=False):
    """One workload through fp_predict: the packed layout of `preset` against
    the naive layout on the same resident rows, checked bit for bit on every
    row, timed with HIP events; optionally the CPU checker's baseline."""
    forest = w.forest(cache_dir=args.cache, progress=Progress(name))
    log(f"{name}: {forest.n_trees} trees, {forest.n_internal() / forest.n_trees:.0f} internal nodes/tree, "
        f"max depth {int(forest.depth.max())}")
    X, _ = w.predict_rows()
    n, F = X.shape
    C = forest.n_classes
    Xd = torch.from_numpy(X).cuda()
    log(f"{name}: {n} x {F} rows resident ({X.nbytes / 2**30:.2f} GiB)")
    votes = torch.empty((n, C), dtype=torch.int32, device="cuda")
    cls = torch.empty((n,), dtype=torch.int32, device="cuda")
    packed, pack_s = pack(fp, forest, **preset["pack"])
    info = fp.fp_packed_info_get(packed)
    naive, naive_pack_s = pack(fp, forest, layout=fp.FP_LAYOUT_NAIVE)
    log(f"{name}: packed {info['bytes'] / 2**20:.1f} MiB in {pack_s:.1f} s ({info['n_bins']} bins, "
        f"{info['expected_fetches']:.2f} fetches per walk); naive {fp.fp_packed_info_get(naive)['bytes'] / 2**20:.1f} MiB "
        f"in {naive_pack_s:.1f} s")
    run_packed = lambda: fp.fp_predict_tuned(packed, preset["tune"], Xd, votes, cls)
    run_naive = lambda: fp.fp_predict_tuned(naive, preset["naive_tune"], Xd, votes, cls)
    # the two layouts must agree bit for bit on the whole batch before timing
    run_naive()
    torch.cuda.synchronize()
    v_naive, c_naive = votes.clone(), cls.clone()
    votes.fill_(-1)
    cls.fill_(-1)
    run_packed()
    torch.cuda.synchronize()
    same = bool(torch.equal(votes, v_naive) and torch.equal(cls, c_naive))
    del v_naive, c_naive
    if not same:
        print(f"{name}: packed and naive votes differ", file=sys.stderr)
        sys.exit(3)
    ms_packed, wall = time_steps(run_packed, steps, warmup, torch)
    log(f"{name}: packed {ms_packed:.3f} ms/step = {n / ms_packed / 1e3:.2f} M obs/s")
    ms_naive, _ = time_steps(run_naive, naive_steps, 0, torch)
    log(f"{name}: naive  {ms_naive:.3f} ms/step ({ms_naive / ms_packed:.2f}x)")
    out = {
        "workload": w.name, "n_rows": n, "n_trees": forest.n_trees, "n_features": F, "n_classes": C,
        "internal_nodes": info["n_internal"], "layout": LAYOUT_NAMES[info["layout"]], "bin_size": info["bin_size"],
        "interleave_depth": info["interleave_depth"], "block_bytes_per_fetch": None, "tune": preset["tune"],
        "packed_bytes": info["bytes"], "expected_fetches_per_walk": info["expected_fetches"],
        "ms_per_step": ms_packed, "value": n / (ms_packed / 1e3), "wall_s_timed": wall,
        "naive": {"ms_per_step": ms_naive, "value": n / (ms_naive / 1e3), "steps": naive_steps},
        "speedup_vs_naive": ms_naive / ms_packed, "bit_exact_vs_naive_all_rows": same, "pack_s": pack_s,
    }
    if with_cpu and not args.no_cpu_baseline:
        # the GPU's own votes for the checked rows (packed layout)
        run_packed()
        torch.cuda.synchronize()
        cpu, check, visits_per_row = cpu_baseline(forest, X, votes.cpu().numpy(), cls.cpu().numpy())
        log(f"{name}: cpu checker {cpu['value']:.0f} obs/s ({cpu['sample']}); GPU == checker on "
            f"{check['rows']} rows: {check['bit_exact']}")
        if not check["bit_exact"]:
            print(f"{name}: GPU votes differ from the CPU checker", file=sys.stderr)
            sys.exit(3)
        out["cpu_baseline"] = cpu
        out["oracle_check"] = check
        out["node_visits_per_row"] = visits_per_row
        out["node_visits_per_s"] = visits_per_row * out["value"]
    out["_keep"] = (forest, packed, naive, Xd, votes, cls)
    return out


def roofline(res, workload):
    """The compulsory HBM bytes of one step (rows in, votes and classes out,
    the packed forest read once) over the step's time.  A step is the packed
    kernel alone (one tree group, no argmax pass), launched once per tree
    pass: per launch, the bytes and the time are both the step's divided by
    the number of passes, the same ratio."""
    n, F, C = res["n_rows"], res["n_features"], res["n_classes"]
    algo = n * (F * 4 + C * 4 + 4) + res["packed_bytes"]
    achieved = algo / (res["ms_per_step"] / 1e3) / 1e9
    traffic = read_traffic(workload, res.get("tune"))
    rec = read_traffic_record(workload, res.get("tune")) or {}
    try:
        l2 = float(rec["l2_hit_rate"])
    except (KeyError, ValueError):
        l2 = None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "algorithmic_bytes_per_launch": algo,
            "traffic_over_algorithmic": traffic / algo if traffic else None,
            "l2_hit_rate": l2}


def leg_batched(args, fp, synth, torch, np, n_forests=64):
    """64 resident forests of uneven size with uneven batches, every forest
    autotuned, one persistent launch replayed from a hipGraph, against every
    forest's naive-layout launch in turn."""
    threads, cursors = 1024, 2
    jobs = []
    t0 = time.perf_counter()
    for i in range(n_forests):
        w = synth.batched_workload(i)
        f = w.forest(cache_dir=args.cache)
        X, _ = w.predict_rows()
        Xd = torch.from_numpy(X).cuda()
        res = fp.fp_autotune(f, Xd, block_threads=threads, cursors=cursors, sample_rows=16384)
        p = fp.fp_pack_forest(f, **res["pack"])
        fp.fp_packed_upload(p)
        fp.fp_packed_set_tune(p, res["tune"])
        votes = torch.empty((len(X), f.n_classes), dtype=torch.int32, device="cuda")
        cls = torch.empty((len(X),), dtype=torch.int32, device="cuda")
        jobs.append({"forest": f, "Xd": Xd, "packed": p, "votes": votes, "cls": cls, "tried": res["n_tried"]})
    log(f"batched: {n_forests} forests trained and tuned in {time.perf_counter() - t0:.1f} s")
    # the plan searches each job's launch on its whole batch (the autotuner
    # timed packings on a 16,384-row sample); tunes are kept per forest and
    # batch-size bucket
    t1 = time.perf_counter()
    plan = fp.fp_plan_create([(j["packed"], j["Xd"], j["votes"], j["cls"]) for j in jobs],
                             block_threads=threads, cursors=cursors, autotune=True)
    plan_s = time.perf_counter() - t1
    rows = sum(int(j["Xd"].shape[0]) for j in jobs)
    ms, _ = time_steps(lambda: fp.fp_predict_batched(plan), 10, 2, torch)
    naive = []
    for j in jobs:
        q = fp.fp_pack_forest(j["forest"], layout=fp.FP_LAYOUT_NAIVE)
        fp.fp_packed_upload(q)
        naive.append(q)
    nv = [torch.empty_like(j["votes"]) for j in jobs]
    nc = [torch.empty_like(j["cls"]) for j in jobs]

    def run_naive():
        for q, j, v, c in zip(naive, jobs, nv, nc):
            fp.fp_predict_tuned(q, {"block_threads": 256}, j["Xd"], v, c)
    ms_naive, _ = time_steps(run_naive, 3, 1, torch)
    fp.fp_predict_batched(plan)
    torch.cuda.synchronize()
    exact = all(torch.equal(v, j["votes"]) and torch.equal(c, j["cls"]) for v, c, j in zip(nv, nc, jobs))
    layouts = [fp.fp_packed_info_get(j["packed"])["layout"] for j in jobs]
    out = {"workload": "64 forests: 16-2,048 trees, 4-784 features, 2-10 classes, 1-200,000 rows each",
           "n_forests": n_forests, "rows": rows, "trees": int(sum(j["forest"].n_trees for j in jobs)),
           "ms_per_step": ms, "value": rows / (ms / 1e3), "unit": "observations/s",
           "naive": {"ms_per_step": ms_naive, "value": rows / (ms_naive / 1e3), "launches": n_forests},
           "speedup_vs_naive": ms_naive / ms, "bit_exact_vs_naive_all_rows": bool(exact),
           "layouts_chosen": {LAYOUT_NAMES[k]: int(c) for k, c in enumerate(np.bincount(layouts, minlength=5)) if c},
           "autotune_candidates_timed": int(sum(j["tried"] for j in jobs)), "plan_create_s": plan_s,
           "plan": fp.fp_plan_info_get(plan)}
    log(f"batched: graph replay {ms:.3f} ms = {rows / ms / 1e3:.2f} M obs/s; naive {n_forests} launches {ms_naive:.3f} ms "
        f"({ms_naive / ms:.2f}x), exact={exact}")
    return out


def leg_serve(args, fp, synth, torch, np, image_w, image_forest, tabular_w, tabular_packed, seconds, warm, rate,
              pool_rows=1_000_000, submit_threads=2):
    """Open-loop serving measurement: 8 resident forests -- the image-shaped
    forest, the 1,024-tree tabular forest and six of the 64 batched-workload
    forests (chosen by seed 4) -- Poisson arrivals at `rate` requests/s, rows
    per request log-uniform in 1..4096, sliced at seeded offsets from a
    1,000,000-row pool per forest.  The library's replay driver submits each
    request at its scheduled arrival time; latency is votes ready minus
    scheduled arrival (open loop).  Every 97th request is checked bit for bit
    against fp_predict of the same rows on its own."""
    rng = np.random.default_rng(4)
    picks = sorted(int(i) for i in rng.choice(np.arange(64), 6, replace=False))
    server = fp.fp_server_create(hbm_budget_bytes=4 << 30, max_inflight=4, max_rows_per_launch=262144)
    entries = [("image", image_w, image_forest, None), ("tabular", tabular_w, None, tabular_packed)]
    entries += [(f"batched_{i}", synth.batched_workload(i), None, None) for i in picks]
    forests = []
    for name, w, f, p in entries:
        if p is None:
            f = f if f is not None else w.forest(cache_dir=args.cache)
            try:  # clustered blocks where the forest's fields fit them, else plain blocks
                p = fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=f.n_trees, interleave_depth=3)
            except fp.FPError:
                p = fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_BLOCKED, bin_size=f.n_trees, interleave_depth=3)
            fp.fp_packed_upload(p)
        info = fp.fp_packed_info_get(p)
        # serving is latency-bound at this load: small tiles, and a forest of
        # many bins split into 8 tree groups, spread each request over more
        # workgroups (tabular forest: p50 0.55 -> 0.26 ms, p99 2.1 -> 0.97 ms;
        # 16-row tiles for the others: p50 0.22 ms, p99 0.93 ms)
        tune = {"rows_per_block": 16, "refill_lanes": 16}
        if info["n_bins"] >= 8:
            tune["tree_groups"] = 8
        fp.fp_packed_set_tune(p, tune)
        pool, _ = w.rows(pool_rows, w.predict_seed + 1000)
        forests.append({"name": name, "pool": pool, "C": info["n_classes"], "packed": p,
                        "id": fp.fp_server_add_forest(server, p)})
    log("serve forests: " + ", ".join(x["name"] for x in forests))
    # warm the serving path before the replay: the first launches load the
    # kernels' code and first touch the staging rings
    for x in forests:
        for n in (1, 4096):
            out = np.empty((n, x["C"]), np.int32)
            fp.fp_serve_poll(server, fp.fp_serve_submit(server, x["id"], x["pool"][:n], out))
    fp.fp_server_reset_stats(server)
    total = int(rate * (warm + seconds))
    gen = np.random.default_rng(5000)
    arrival = np.cumsum(gen.exponential(1.0 / rate, size=total))
    fid = gen.integers(0, len(forests), size=total)
    rows = np.clip(np.floor(np.exp(gen.uniform(0.0, np.log(4097.0), size=total))), 1, 4096).astype(np.int64)
    offs = (gen.random(total) * (pool_rows - rows + 1)).astype(np.int64)
    # checked requests get their own output buffers; the others share one
    # scratch buffer per forest (only the scheduler thread writes outputs)
    scratch = [np.empty((4096, f["C"]), np.int32) for f in forests]
    checked = {int(i): np.empty((rows[i], forests[fid[i]]["C"]), np.int32) for i in range(0, total, 97)}
    sched = np.zeros(total, fp.REPLAY_DTYPE)
    sched["forest_id"] = [forests[k]["id"] for k in fid]
    feats = np.array([f["pool"].shape[1] for f in forests], np.int64)
    base = np.array([f["pool"].ctypes.data for f in forests], np.uint64)
    sched["X"] = base[fid] + (offs * feats[fid] * 4).astype(np.uint64)
    sched["n_rows"] = rows
    sched["ld"] = feats[fid]
    sched["votes"] = np.array([scratch[k].ctypes.data for k in fid], np.uint64)
    for i, buf in checked.items():
        sched["votes"][i] = buf.ctypes.data
    sched["arrival_s"] = arrival
    lat, lag = fp.fp_serve_replay(server, sched, submit_threads=submit_threads)
    st = fp.fp_server_stats(server)
    fp.fp_server_destroy(server)
    # the checked requests' rows predicted alone, one launch per forest
    exact = True
    for k, x in enumerate(forests):
        idx = [i for i in checked if fid[i] == k]
        if not idx:
            continue
        Xc = np.concatenate([x["pool"][offs[i]:offs[i] + rows[i]] for i in idx])
        v, _ = fp.fp_predict(x["packed"], torch.from_numpy(Xc).cuda(), want_cls=False)
        v = v.cpu().numpy()
        o = 0
        for i in idx:
            exact &= bool(np.array_equal(checked[i], v[o:o + rows[i]]))
            o += rows[i]
    m = arrival >= warm
    span = float(arrival[m][-1] - arrival[m][0]) if m.sum() > 1 else 1.0
    out = {
        "workload": "8 resident forests (image, tabular 1,024 trees, six batched), Poisson arrivals, "
                    "1-4,096 rows per request",
        "forests": [x["name"] for x in forests],
        "requests_measured": int(m.sum()),
        "offered_req_per_s": float(m.sum()) / span,
        "offered_rows_per_s": float(rows[m].sum()) / span,
        "served_rows_per_s": float(rows.sum()) / float((arrival + lat / 1e3).max() - arrival[0]),
        "p50_ms": float(np.percentile(lat[m], 50)), "p99_ms": float(np.percentile(lat[m], 99)),
        "mean_ms": float(lat[m].mean()), "max_ms": float(lat[m].max()),
        "latency_definition": "votes ready minus scheduled arrival (open loop)",
        "launches": st["launches"], "mean_rows_per_launch": st["mean_rows_per_launch"],
        "submit_lag_p99_ms": float(np.percentile(lag[m], 99)),
        "saturated": bool(np.percentile(lat[m][-1000:], 50) > 10 * max(np.percentile(lat[m][:1000], 50), 0.1)),
        "bit_exact_checked_requests": len(checked), "bit_exact_vs_alone": bool(exact),
        "seconds": seconds, "rate": rate, "pool_rows": pool_rows,
    }
    log(f"serve: p50 {out['p50_ms']:.2f} ms, p99 {out['p99_ms']:.2f} ms, {out['served_rows_per_s'] / 1e6:.2f} M rows/s, "
        f"saturated={out['saturated']}, exact={exact}")
    return out


def leg_small(args, fp, synth, torch, np, steps):
    """The small two-class case (10,000 rows, 32 trees of depth <= 12): launch
    bound, so device time per step and host wall time per call are both given."""
    from paper_1806_07300_amd import presets
    res = single_forest_leg("small", synth.small(), presets.SMALL, args, fp, torch, np, steps, 3, 10)
    forest, packed, naive, Xd, votes, cls = res.pop("_keep")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(100):
        fp.fp_predict_tuned(packed, presets.SMALL["tune"], Xd, votes, cls)
    torch.cuda.synchronize()
    res["wall_ms_per_call_incl_launch"] = (time.perf_counter() - t0) * 10.0
    return res


# The paper's layout ablation (Sec. III-A, Fig. 4) mapped to this GPU path:
# BF and DF run the naive kernel (a lane per row, trees in turn, leaves
# stored, features from memory); DF-, Stat and Bin run the packed kernel
# with one walk per lane (no round-robin), Bin+ with four walks per lane
# interleaved; the block layouts follow with their own launches.
def ladder_rungs(workload: str, fp, presets):
    wide = dict(rows_per_block=48, block_threads=1024) if workload == "image" else \
        dict(rows_per_block=256, block_threads=1024)
    one = dict(wide, cursors=1)
    rr = dict(wide, cursors=4)
    blk = dict(wide, cursors=1, refill_lanes=32 if workload == "image" else 16)
    B = 16
    clustered = presets.IMAGE["pack"] if workload == "image" else \
        {"layout": fp.FP_LAYOUT_CLUSTERED, "bin_size": 16, "interleave_depth": 3}
    return [
        ("BF", {"layout": fp.FP_LAYOUT_NAIVE}, {"block_threads": 256}),
        ("DF", {"layout": fp.FP_LAYOUT_NAIVE, "node_order": fp.FP_ORDER_DF}, {"block_threads": 256}),
        ("DF-", {"layout": fp.FP_LAYOUT_PACKED, "bin_size": 1, "interleave_depth": 0,
                 "node_order": fp.FP_ORDER_DF}, one),
        ("Stat", {"layout": fp.FP_LAYOUT_PACKED, "bin_size": 1, "interleave_depth": 0}, one),
        ("Stat-obs", {"layout": fp.FP_LAYOUT_PACKED, "bin_size": 1, "interleave_depth": 0}, one),
        ("Bin", {"layout": fp.FP_LAYOUT_PACKED, "bin_size": B, "interleave_depth": 3}, one),
        ("Bin+", {"layout": fp.FP_LAYOUT_PACKED, "bin_size": B, "interleave_depth": 3}, rr),
        ("COMPACT", {"layout": fp.FP_LAYOUT_COMPACT, "bin_size": B, "interleave_depth": 3}, rr),
        ("BLOCKED", {"layout": fp.FP_LAYOUT_BLOCKED, "bin_size": B, "interleave_depth": 3}, blk),
        ("CLUSTERED", clustered, presets.IMAGE["tune"] if workload == "image" else presets.TABULAR["tune"]),
    ]


def eu_stat(bias: float) -> float:
    """Expected uses of a fetched cache line (Sec. III-A): one node for sure,
    then each further node of the line (two per line, plus the adjacent line
    the prefetcher brings) with probability `bias` per level."""
    return 1.0 + bias * (1.0 + bias * (1.0 + bias))


def eu_model(name: str, info: dict, D: int) -> tuple:
    """(fetches, well-used nodes, EU) of a ladder rung for the run-time
    estimate of Eqs. 1-2: time = (BF time / BF fetches) * (fetches - WuN) / EU.
    DF has no access statistics, so its bias is 1/2; the interleaved levels of
    a bin are its well-used nodes; a block is one fetch whatever it holds."""
    f, d, b = info["expected_fetches"], info["expected_depth"], info["mean_bias"]
    if name == "BF":
        return f, 0.0, 1.0
    if name in ("DF", "DF-"):
        return f, 0.0, eu_stat(0.5)
    if name in ("Stat", "Stat-obs"):
        return f, 0.0, eu_stat(b)
    if name in ("Bin", "Bin+", "COMPACT"):
        return f, min(D + 1.0, d), eu_stat(b)
    return f, 0.0, 1.0


def ladder(args, fp, synth, torch):
    import numpy as np
    from paper_1806_07300_amd import presets
    t0 = time.perf_counter()
    if args.ladder == "image":
        w = synth.image(n_predict=args.rows or 1_000_000)
    elif args.ladder == "tabular":
        w = synth.tabular(n_predict=args.rows or 1_000_000)
    else:
        w = synth.tabular(n_train=200_000, n_trees=128, n_predict=args.rows or 1_000_000, imbalanced=True)
    forest = w.forest(cache_dir=args.cache, progress=Progress(args.ladder))
    X, y = w.predict_rows()
    n, C = X.shape[0], forest.n_classes
    log(f"ladder {args.ladder}: {forest.n_trees} trees, {n} rows, class shares "
        f"{[round(float(v), 3) for v in np.bincount(y, minlength=C) / max(n, 1)]} ({time.perf_counter() - t0:.1f} s)")
    Xd = torch.from_numpy(X).cuda()
    # Stat-obs: the same packing with node statistics inferred from observations
    observed = forest.subset(range(forest.n_trees))
    observed.cardinality = fp.fp_infer_cardinality(forest, Xd[:min(n, 100_000)])
    votes = torch.empty((n, C), dtype=torch.int32, device="cuda")
    cls = torch.empty((n,), dtype=torch.int32, device="cuda")
    ref = None
    rungs = []
    for name, pk, tune in ladder_rungs(args.ladder, fp, presets):
        p = fp.fp_pack_forest(observed if name == "Stat-obs" else forest, **pk)
        fp.fp_packed_upload(p)
        run = lambda: fp.fp_predict_tuned(p, tune, Xd, votes, cls)
        votes.fill_(-1)
        run()
        torch.cuda.synchronize()
        if ref is None:
            ref = votes.clone()
        exact = bool(torch.equal(votes, ref))
        ms, _ = time_steps(run, args.steps, args.warmup, torch)
        info = fp.fp_packed_info_get(p)
        fetches, wun, eu = eu_model(name, info, pk.get("interleave_depth", 0))
        rungs.append({"name": name, "pack": pk, "tune": tune, "ms": ms, "obs_per_s": n / (ms / 1e3),
                      "bytes": info["bytes"], "bit_exact_vs_BF": exact, "expected_depth": info["expected_depth"],
                      "mean_bias": info["mean_bias"], "expected_fetches": fetches, "well_used_nodes": wun,
                      "eu": eu})
        log(f"{name:9s} {ms:9.3f} ms  {n / ms / 1e3:8.2f} M obs/s  {info['bytes'] / 2**20:8.1f} MiB  "
            f"fetches/walk {fetches:6.2f}  EU {eu:5.3f}  exact={exact}")
        del p
        if not exact:
            print(f"{name}: votes differ from BF", file=sys.stderr)
            sys.exit(3)
    bf = rungs[0]["ms"]
    miss = bf / rungs[0]["expected_fetches"]  # Eq. 1: BF time per fetched node
    for r in rungs:
        r["speedup_vs_BF"] = bf / r["ms"]
        r["eu_model_ms"] = miss * (r["expected_fetches"] - r["well_used_nodes"]) / r["eu"]  # Eq. 2
        log(f"{r['name']:9s} measured {r['ms']:9.3f} ms, Eq. 2 estimate {r['eu_model_ms']:9.3f} ms")
    # the autotuner's cost-model prior (Eq. 2 with EU) on the same forest: the
    # score of every candidate packing beside the time of the ones it timed.
    # It packs every candidate, so a forest of more than 128 trees is tuned
    # on its first 32 (packing the 1,024-tree forest 66 times takes half an
    # hour of host time)
    sample = min(n, 65536)
    tuned_forest = forest if forest.n_trees <= 128 else forest.subset(range(32))
    log(f"autotune on {tuned_forest.n_trees} trees, {sample} rows: packing and scoring every candidate")
    tuned = fp.fp_autotune(tuned_forest, Xd[:sample], block_threads=1024, sample_rows=sample)
    for t in sorted(tuned["trials"], key=lambda t: (t["pack"]["layout"], t["model_cost"])):
        pk = t["pack"]
        log(f"autotune {LAYOUT_NAMES[pk['layout']]:9s} B={pk['bin_size']:5d} D={pk['interleave_depth']}  "
            f"model {t['model_cost']:10.1f}  " + (f"measured {t['ms']:8.3f} ms" if t["ms"] >= 0 else "not timed"))
    log(f"autotune: {tuned['n_candidates']} packings scored, {tuned['n_tried']} launches timed; chose "
        f"{LAYOUT_NAMES[tuned['pack']['layout']]} B={tuned['pack']['bin_size']} D={tuned['pack']['interleave_depth']} "
        f"{tuned['tune']} at {tuned['best_ms']:.3f} ms per {sample} rows")
    print(json.dumps({"ladder": args.ladder, "n_rows": n, "n_trees": forest.n_trees, "steps": args.steps,
                      "rungs": rungs, "autotune_trees": tuned_forest.n_trees, "autotune": tuned}), flush=True)


def gather_ceiling(fp, torch, working_set: int, fetch_bytes: int, chains=(1, 2, 4)) -> dict:
    """Best dependent-gather rate over chains per lane through a buffer of
    about `working_set` bytes (the probe rounds the element count down to a
    power of two)."""
    buf = torch.empty(max(working_set, 64 * fetch_bytes) // 4 + 16, dtype=torch.int32, device="cuda")
    n = 1
    while n * 2 * fetch_bytes <= buf.numel() * 4:
        n *= 2
    best = max((fp.fp_probe_gather(buf, fetch_bytes, c, steps=max(64, 1024 // c)), c) for c in chains)
    del buf
    return {"working_set_bytes": n * fetch_bytes, "fetch_bytes": fetch_bytes, "fetches_per_s": best[0],
            "gbps": best[0] * fetch_bytes / 1e9, "chains_per_lane": best[1]}


def vmem_ceiling(fp, torch, res, fetch_bytes):
    """The kernel's block fetches per second against the most the load path
    returns at all: the gather probe over a 16 KB working set (every CU's L1
    holds it) with 4 or 8 chains per lane.  The kernel's count is the
    training-distributed fetches per walk from the packed header times the
    walks of a step; blocks served from LDS are included, so the fraction is
    an upper estimate."""
    g = gather_ceiling(fp, torch, 16 << 10, fetch_bytes, chains=(4, 8))
    walks = res["n_rows"] * res["n_trees"]
    kernel = res["expected_fetches_per_walk"] * walks / (res["ms_per_step"] / 1e3)
    return {"probe_block_fetches_per_s": g["fetches_per_s"], "probe_working_set_bytes": g["working_set_bytes"],
            "probe_chains_per_lane": g["chains_per_lane"], "fetch_bytes": fetch_bytes,
            "kernel_block_fetches_per_s": kernel, "frac": kernel / g["fetches_per_s"]}


def probes(args, fp, synth, torch):
    out = {"probes": True}
    a = torch.ones(1 << 29, dtype=torch.int32, device="cuda")  # 2 GiB
    b = torch.empty_like(a)
    out["stream_gbps"] = max(fp.fp_probe_stream(a, b) for _ in range(3))
    log(f"stream copy: {out['stream_gbps']:.0f} GB/s (read + write)")
    del a, b
    curve = []
    for ws in (1 << 20, 4 << 20, 16 << 20, 64 << 20, 256 << 20, 1 << 30, 4 << 30, 8 << 30):
        for fb in (16, 48, 64):
            g = gather_ceiling(fp, torch, ws, fb)
            curve.append(g)
            log(f"gather {g['working_set_bytes'] / 2**20:8.1f} MiB x {fb:2d} B: {g['fetches_per_s'] / 1e9:7.1f} G fetches/s "
                f"= {g['gbps']:7.0f} GB/s ({g['chains_per_lane']} chains per lane)")
    out["gather"] = curve
    # host-to-device rate of the image batch from pinned memory
    w = synth.image(n_predict=args.rows or 1_000_000)
    forest = w.forest(cache_dir=args.cache)
    X, _ = w.predict_rows()
    Xh = torch.from_numpy(X).pin_memory()
    Xd = torch.empty_like(Xh, device="cuda")
    Xd.copy_(Xh, non_blocking=True)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    Xd.copy_(Xh, non_blocking=True)
    t1.record()
    torch.cuda.synchronize()
    h2d_ms = t0.elapsed_time(t1)
    out["h2d"] = {"bytes": X.nbytes, "ms": h2d_ms, "gbps": X.nbytes / (h2d_ms * 1e-3) / 1e9}
    log(f"host to device (pinned): {X.nbytes / 2**30:.2f} GiB in {h2d_ms:.1f} ms = {out['h2d']['gbps']:.1f} GB/s")
    # the naive kernel's own workgroup-size sweep (same layout, flags and resident rows)
    naive = fp.fp_pack_forest(forest, layout=fp.FP_LAYOUT_NAIVE)
    fp.fp_packed_upload(naive)
    votes = torch.empty((X.shape[0], forest.n_classes), dtype=torch.int32, device="cuda")
    cls = torch.empty((X.shape[0],), dtype=torch.int32, device="cuda")
    sweep = {}
    for th in (64, 128, 256, 512, 1024):
        ms, _ = time_steps(lambda: fp.fp_predict_tuned(naive, {"block_threads": th}, Xd, votes, cls), 5, 1, torch)
        sweep[th] = ms
        log(f"naive, {th:4d}-thread workgroups: {ms:.2f} ms")
    out["naive_sweep_ms"] = sweep
    print(json.dumps(out), flush=True)


def only(args, fp, synth, torch):
    """One kernel, --steps launches, no measurement of its own (for rocprofv3)."""
    from paper_1806_07300_amd import presets
    if args.only == "copy":
        # calibration kernel of known size for the HBM byte counters: 1 GiB copy
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print("copy done: bytes read per launch", a.numel() * 4, "written", b.numel() * 4, flush=True)
        return
    w = {"tabular": synth.tabular, "image": synth.image, "small": synth.small}[args.workload]()
    preset = {"tabular": presets.TABULAR, "image": presets.IMAGE, "small": presets.SMALL}[args.workload]
    forest = w.forest(cache_dir=args.cache, progress=Progress(args.workload))
    X, _ = w.predict_rows(args.rows or None)
    Xd = torch.from_numpy(X).cuda()
    del X
    kw = preset["pack"] if args.only == "packed" else {"layout": fp.FP_LAYOUT_NAIVE}
    tune = preset["tune"] if args.only == "packed" else preset["naive_tune"]
    p, pack_s = pack(fp, forest, **kw)
    log(f"{args.workload} {args.only}: packed in {pack_s:.1f} s")
    votes = torch.empty((Xd.shape[0], forest.n_classes), dtype=torch.int32, device="cuda")
    cls = torch.empty((Xd.shape[0],), dtype=torch.int32, device="cuda")
    for i in range(args.steps):
        fp.fp_predict_tuned(p, tune, Xd, votes, cls)
        torch.cuda.synchronize()
        log(f"{args.only} launch {i + 1}/{args.steps} done")


def headline(args, fp, torch, np, presets, tab_w):
    """The benchmark's line: the tabular workload, 10M rows through 1,024
    trees in bins of 16, packed (the preset's launch) against naive, with the
    CPU checker's baseline and bit-exact check, the HBM roofline and the
    vector-memory ceiling."""
    res = single_forest_leg("tabular", tab_w, presets.TABULAR, args, fp, torch, np, args.steps,
                            args.warmup, 3, with_cpu=True)
    forest, packed, naive, Xd, votes, cls = res.pop("_keep")
    del naive, Xd, votes, cls
    torch.cuda.empty_cache()
    res["block_bytes_per_fetch"] = 64
    rl = roofline(res, "tabular")
    vm = vmem_ceiling(fp, torch, res, 64)
    log(f"vector-memory ceiling: {vm['probe_block_fetches_per_s'] / 1e9:.0f} G 64-byte blocks/s (L1-resident probe); "
        f"kernel {vm['kernel_block_fetches_per_s'] / 1e9:.0f} G/s = {vm['frac']:.2f}")
    out = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "observations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "large binary tabular: 28 fp32 features (21 normal, 7 products), 1,024 trees grown to "
                        "pure leaves on 1,000,000 rows, bins of 16 trees, 10,000,000 rows per step",
            **{k: res[k] for k in ("n_rows", "n_trees", "n_features", "n_classes", "internal_nodes", "layout",
                                   "bin_size", "interleave_depth", "tune", "packed_bytes",
                                   "expected_fetches_per_walk")},
            "compare": "fp32 x <= fp32 threshold (64-byte clustered blocks)",
        },
        "naive": res["naive"],
        "speedup_vs_naive": res["speedup_vs_naive"],
        # context, not a target: the paper's own measurements, on CPUs
        "paper_reported": {"speedup_over_ranger_cpp": 4, "speedup_over_r_rerf": 50,
                           "hardware": "4 x Intel Xeon E7-4860 v2, 2.6 GHz (single-core experiments); "
                                       "AWS t2.xlarge nodes (multi-node)",
                           "where": "Sec. I (speedups), Sec. IV-A (hardware)"},
        "bit_exact_vs_naive_all_rows": res["bit_exact_vs_naive_all_rows"],
        "roofline": rl,
        "vmem_ceiling": vm,
        "wall_s_timed": res["wall_s_timed"],
        "pack_s": res["pack_s"],
    }
    for k in ("cpu_baseline", "oracle_check", "node_visits_per_row", "node_visits_per_s"):
        if k in res:
            out[k] = res[k]
    return out, packed


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rows", type=int, default=0, help="rows per step for --only/--ladder/--probes (0: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["packed", "naive", "copy"], default=None)
    ap.add_argument("--workload", choices=["tabular", "image", "small"], default="tabular")
    ap.add_argument("--cache", default=os.environ.get("FP_BENCH_CACHE", "/tmp/forestpack_cache"))
    ap.add_argument("--headline", choices=["tabular", "none"], default="tabular",
                    help="none: only the extra workloads (profiling sessions; no benchmark line)")
    ap.add_argument("--legs", default="small,image,batched,serve",
                    help="extra workloads after the headline, comma-separated (or 'none')")
    ap.add_argument("--budget-s", type=float, default=480.0,
                    help="start no extra leg after this many seconds of the run")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=20000.0)
    ap.add_argument("--ladder", choices=["image", "tabular", "tabular_imb"], default=None)
    ap.add_argument("--probes", action="store_true")
    ap.add_argument("--lite", action="store_true",
                    help="small sizes for every leg, to check the code paths quickly (not a measurement)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); rows shard across GPUs with the "
              "forest replicated and no exchange, which is not run here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1806_07300_amd as fp
    from paper_1806_07300_amd import presets
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.only:
        only(args, fp, synth, torch)
        return
    if args.ladder:
        ladder(args, fp, synth, torch)
        return
    if args.probes:
        probes(args, fp, synth, torch)
        return

    tab_w = synth.tabular(n_train=20_000, n_trees=32, n_predict=200_000) if args.lite else synth.tabular()
    img_w = synth.image(n_train=6000, n_trees=16, n_predict=100_000) if args.lite else synth.image()
    if args.headline == "none":  # the extra workloads alone (profiling sessions); not the benchmark's line
        out, packed = {"headline": None}, None
    else:
        out, packed = headline(args, fp, torch, np, presets, tab_w)
    legs = [x for x in args.legs.split(",") if x and x != "none"]
    extra = {}
    image_forest = None
    for leg in legs:
        if elapsed() > args.budget_s:
            log(f"{leg}: skipped, {elapsed():.0f} s spent (budget {args.budget_s:.0f} s)")
            extra[leg] = {"skipped": f"time budget of {args.budget_s:.0f} s spent"}
            continue
        t0 = time.perf_counter()
        if leg == "small":
            r = leg_small(args, fp, synth, torch, np, 50)
        elif leg == "image":
            r = single_forest_leg("image", img_w, presets.IMAGE, args, fp, torch, np, 20, 3, 3)
            image_forest = r.pop("_keep")[0]
            r["block_bytes_per_fetch"] = 48
            r["compare"] = ("fp16: rows staged in LDS rounded toward +inf, every threshold exact in fp16 "
                            "(48-byte clustered blocks); decides every x <= t exactly as fp32")
            r["roofline"] = roofline(r, "image")
            r["vmem_ceiling"] = vmem_ceiling(fp, torch, r, 48)
            torch.cuda.empty_cache()
        elif leg == "batched":
            r = leg_batched(args, fp, synth, torch, np, 8 if args.lite else 64)
        elif leg == "serve":
            if image_forest is None:
                image_forest = img_w.forest(cache_dir=args.cache)
            if packed is None:
                tf = tab_w.forest(cache_dir=args.cache, progress=Progress("tabular"))
                packed, _ = pack(fp, tf, **presets.TABULAR["pack"])
            r = leg_serve(args, fp, synth, torch, np, img_w, image_forest, tab_w, packed,
                          2.0 if args.lite else args.serve_seconds, 1.0,
                          2000.0 if args.lite else args.serve_rate, pool_rows=100_000 if args.lite else 1_000_000)
        else:
            raise SystemExit(f"unknown leg {leg}")
        r["leg_s"] = time.perf_counter() - t0
        extra[leg] = r
    out["workloads"] = extra
    if "serve" in extra and "p99_ms" in extra["serve"]:
        out["serve_p50_ms"] = extra["serve"]["p50_ms"]
        out["serve_p99_ms"] = extra["serve"]["p99_ms"]
    out["bench_wall_s"] = elapsed()
    if args.lite:
        out["lite"] = "small sizes: a check of the code paths, not a measurement"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
