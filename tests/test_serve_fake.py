"""The serving scheduler on the CPU fake executor (no GPU): admission under
the HBM budget (waiting heap copies, ring wrap-around), FP_E2BIG and
FP_EAGAIN, injected launch failures followed by re-queue and retry with
unchanged results, retries running out, and poll time-outs.

The fake executor's "votes" are a checksum of each row (the FNV-1a hash of
its fp32 bytes, mixed with the class index), so every request's output
shows whether the scheduler copied the right rows in and the right votes
out, whatever it was coalesced with."""
import threading
import time

import numpy as np
import pytest

import paper_1806_07300_amd as fp
import synth

FAKE = fp.FP_EXECUTOR_CPU_FAKE


def fake_votes(X, F, C):
    """The fake executor's output, restated: FNV-1a over each row's bytes."""
    rows = np.ascontiguousarray(X[:, :F], dtype=np.float32).view(np.uint8).reshape(len(X), F * 4)
    h = np.full(len(X), 2166136261, np.uint64)
    for k in range(F * 4):
        h = ((h ^ rows[:, k].astype(np.uint64)) * np.uint64(16777619)) & np.uint64(0xFFFFFFFF)
    c = (np.arange(C, dtype=np.uint64) * np.uint64(0x9E3779B9)) & np.uint64(0xFFFFFFFF)
    return ((h[:, None] ^ c[None, :]) & np.uint64(0x7FFFFFFF)).astype(np.int32)


@pytest.fixture(scope="module")
def forests():
    out = []
    for F, C, seed in ((6, 3, 1), (17, 5, 2)):
        Xt, yt = synth.gaussian_mixture(500, F, C, seed=seed)
        f = synth.train_forest(Xt, yt, n_trees=4, n_classes=C, mtry=2, max_depth=5, seed=seed)
        p = fp.fp_pack_forest(f, layout=fp.FP_LAYOUT_CLUSTERED, bin_size=2, interleave_depth=3)
        pool, _ = synth.gaussian_mixture(20_000, F, C, seed=10 + seed)
        out.append({"packed": p, "pool": pool, "F": F, "C": C, "want": fake_votes(pool, F, C)})
    return out


def submit_all(server, ids, forests, reqs, n_threads=3, outs=None):
    outs = outs if outs is not None else [None] * len(reqs)
    tickets = [None] * len(reqs)
    errors = []

    def run(k):
        try:
            for i in range(k, len(reqs), n_threads):
                fi, off, rows = reqs[i]
                f = forests[fi]
                outs[i] = np.full((rows, f["C"]), -1, np.int32)
                tickets[i] = fp.fp_serve_submit(server, ids[fi], f["pool"][off:off + rows], outs[i])
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(e)

    th = [threading.Thread(target=run, args=(k,)) for k in range(n_threads)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    return outs, tickets


def requests(forests, n, seed, max_rows=900):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        fi = int(rng.integers(0, len(forests)))
        rows = int(min(max_rows, max(1, np.floor(np.exp(rng.uniform(0, np.log(max_rows + 1)))))))
        out.append((fi, int(rng.integers(0, len(forests[fi]["pool"]) - rows + 1)), rows))
    return out


def check(outs, forests, reqs):
    for (fi, off, rows), o in zip(reqs, outs):
        assert np.array_equal(o, forests[fi]["want"][off:off + rows]), (fi, off, rows)


def test_fake_votes_restatement(forests):
    f = forests[0]
    server = fp.fp_server_create(executor=FAKE)
    fid = fp.fp_server_add_forest(server, f["packed"])
    out = np.zeros((3, f["C"]), np.int32)
    assert fp.fp_serve_poll(server, fp.fp_serve_submit(server, fid, f["pool"][:3], out), 5_000_000)
    assert np.array_equal(out, f["want"][:3])
    fp.fp_server_destroy(server)


@pytest.mark.parametrize("budget,inflight,delay", [(0, 4, 0), (1 << 20, 2, 200), (1 << 20, 1, 50)])
def test_admission_under_budget(forests, budget, inflight, delay):
    """A 1 MiB budget holds a few requests at a time: the rest wait as heap
    copies and enter the rings in arrival order as space frees up."""
    server = fp.fp_server_create(hbm_budget_bytes=budget, max_inflight=inflight, max_rows_per_launch=4096,
                                 executor=FAKE, fake_delay_us=delay)
    ids = [fp.fp_server_add_forest(server, f["packed"]) for f in forests]
    reqs = requests(forests, 300, seed=budget + inflight)
    outs, tickets = submit_all(server, ids, forests, reqs)
    for t in tickets:
        assert fp.fp_serve_poll(server, t, 20_000_000)
    check(outs, forests, reqs)
    st = fp.fp_server_stats(server)
    assert st["completed"] == st["submitted"] == len(reqs) and st["failed"] == 0
    assert st["launches"] < len(reqs) or inflight == 4  # requests coalesce while launches run
    fp.fp_server_destroy(server)


def test_e2big_and_einval(forests):
    server = fp.fp_server_create(hbm_budget_bytes=1 << 20, max_rows_per_launch=1000, executor=FAKE)
    fid = fp.fp_server_add_forest(server, forests[1]["packed"])
    f = forests[1]
    with pytest.raises(fp.FPError) as e:  # more rows than one launch takes
        fp.fp_serve_submit(server, fid, f["pool"][:1001], np.zeros((1001, f["C"]), np.int32))
    assert e.value.code == fp.FP_E2BIG
    big = np.zeros((9000, 17), np.float32)  # more staging than the whole budget
    server2 = fp.fp_server_create(hbm_budget_bytes=1 << 20, executor=FAKE)
    fid2 = fp.fp_server_add_forest(server2, f["packed"])
    with pytest.raises(fp.FPError) as e:
        fp.fp_serve_submit(server2, fid2, big, np.zeros((9000, f["C"]), np.int32))
    assert e.value.code == fp.FP_E2BIG
    with pytest.raises(fp.FPError) as e:
        fp.fp_serve_submit(server, 7, f["pool"][:2], np.zeros((2, f["C"]), np.int32))
    assert e.value.code == fp.FP_EINVAL
    with pytest.raises(fp.FPError) as e:
        fp.fp_serve_poll(server, 99999, 0)
    assert e.value.code == fp.FP_EINVAL
    fp.fp_server_destroy(server)
    fp.fp_server_destroy(server2)


def test_eagain_when_the_queue_is_full(forests):
    f = forests[0]
    server = fp.fp_server_create(max_inflight=1, max_queue=4, executor=FAKE, fake_delay_us=300_000)
    fid = fp.fp_server_add_forest(server, f["packed"])
    outs, tickets, rejected = [], [], 0
    for i in range(12):
        o = np.zeros((5, f["C"]), np.int32)
        try:
            tickets.append((i, fp.fp_serve_submit(server, fid, f["pool"][5 * i:5 * i + 5], o)))
            outs.append((i, o))
        except fp.FPError as e:
            assert e.code == fp.FP_EAGAIN
            rejected += 1
    # the first launch takes the 0-4 requests queued when the scheduler wakes
    # (none if it has not woken before the last submission), then four more
    # queue behind it for the launch's 300 ms: 4-8 are refused
    assert 4 <= rejected <= 8, rejected
    assert fp.fp_server_stats(server)["rejected"] == rejected
    for _, t in tickets:
        assert fp.fp_serve_poll(server, t, 20_000_000)
    for i, o in outs:
        assert np.array_equal(o, f["want"][5 * i:5 * i + 5])
    fp.fp_server_destroy(server)


@pytest.mark.parametrize("fail_every,inflight", [(2, 1), (3, 2), (5, 4)])
def test_failed_launches_are_retried(forests, fail_every, inflight):
    """Every k-th launch fails: its requests go back to the head of the queue
    and the next launch serves them; every result is the same as without
    failures (the retry is idempotent)."""
    server = fp.fp_server_create(max_inflight=inflight, max_rows_per_launch=2048, executor=FAKE,
                                 fake_delay_us=100, fake_fail_every=fail_every, max_retries=3)
    ids = [fp.fp_server_add_forest(server, f["packed"]) for f in forests]
    reqs = requests(forests, 200, seed=fail_every)
    outs, tickets = submit_all(server, ids, forests, reqs)
    for t in tickets:
        assert fp.fp_serve_poll(server, t, 20_000_000)
    check(outs, forests, reqs)
    st = fp.fp_server_stats(server)
    assert st["failed_launches"] >= 1 and st["retried"] >= 1 and st["failed"] == 0
    assert st["completed"] == len(reqs)
    fp.fp_server_destroy(server)


def test_retries_run_out(forests):
    """With every launch failing, a request fails after 1 + max_retries
    launches and poll reports FP_EHIP; the server stays usable."""
    f = forests[0]
    server = fp.fp_server_create(max_inflight=1, executor=FAKE, fake_fail_every=1, max_retries=2)
    fid = fp.fp_server_add_forest(server, f["packed"])
    t = fp.fp_serve_submit(server, fid, f["pool"][:10], np.zeros((10, f["C"]), np.int32))
    with pytest.raises(fp.FPError) as e:
        fp.fp_serve_poll(server, t, 10_000_000)
    assert e.value.code == fp.FP_EHIP and "injected" in str(e.value)
    st = fp.fp_server_stats(server)
    assert st["failed_launches"] == 3 and st["retried"] == 2 and st["failed"] == 1
    fp.fp_server_destroy(server)


def test_no_retry_when_disabled(forests):
    f = forests[0]
    server = fp.fp_server_create(max_inflight=1, executor=FAKE, fake_fail_every=1, max_retries=-1)
    fid = fp.fp_server_add_forest(server, f["packed"])
    t = fp.fp_serve_submit(server, fid, f["pool"][:10], np.zeros((10, f["C"]), np.int32))
    with pytest.raises(fp.FPError):
        fp.fp_serve_poll(server, t, 10_000_000)
    assert fp.fp_server_stats(server)["failed_launches"] == 1
    fp.fp_server_destroy(server)


def test_poll_timeouts(forests):
    f = forests[1]
    server = fp.fp_server_create(executor=FAKE, fake_delay_us=200_000)
    fid = fp.fp_server_add_forest(server, f["packed"])
    out = np.zeros((50, f["C"]), np.int32)
    t = fp.fp_serve_submit(server, fid, f["pool"][:50], out)
    assert not fp.fp_serve_poll(server, t, 0)
    t0 = time.perf_counter()
    assert not fp.fp_serve_poll(server, t, 20_000)
    assert time.perf_counter() - t0 >= 0.015
    assert fp.fp_serve_poll(server, t, -1)
    assert np.array_equal(out, f["want"][:50])
    with pytest.raises(fp.FPError):  # a retired ticket is unknown
        fp.fp_serve_poll(server, t, 0)
    fp.fp_server_destroy(server)


def test_destroy_drops_pending(forests):
    f = forests[0]
    server = fp.fp_server_create(max_inflight=1, executor=FAKE, fake_delay_us=50_000)
    fid = fp.fp_server_add_forest(server, f["packed"])
    keep = [np.zeros((20, f["C"]), np.int32) for _ in range(30)]
    for i, o in enumerate(keep):
        fp.fp_serve_submit(server, fid, f["pool"][20 * i:20 * i + 20], o)
    fp.fp_server_destroy(server)  # waits for the launch in flight, drops the rest


def test_replay_on_the_fake(forests):
    server = fp.fp_server_create(max_inflight=2, executor=FAKE, fake_delay_us=100)
    ids = [fp.fp_server_add_forest(server, f["packed"]) for f in forests]
    reqs = requests(forests, 400, seed=77, max_rows=600)
    sched = np.zeros(len(reqs), fp.REPLAY_DTYPE)
    outs = []
    for i, (fi, off, rows) in enumerate(reqs):
        f = forests[fi]
        o = np.full((rows, f["C"]), -1, np.int32)
        outs.append(o)
        sched[i] = (ids[fi], 0, f["pool"].ctypes.data + off * f["F"] * 4, rows, f["F"], o.ctypes.data, i * 100e-6)
    lat, lag = fp.fp_serve_replay(server, sched, submit_threads=2)
    assert (lat > 0).all() and (lag >= 0).all()
    check(outs, forests, reqs)
    fp.fp_server_destroy(server)
