// Serving loop: continuous batching of prediction requests on resident
// packed forests.
//
// Staging memory is two rings (observations, votes) that the executor
// keeps on the device and mirrors in host memory at the same offsets; the
// HBM budget is their total.  Admission = getting ring space.
// fp_serve_submit reserves space for the request (in arrival order) and
// copies its rows straight into the host ring; when the rings are full it
// keeps a heap copy instead and the request waits (requests behind it wait
// too, so admission stays first-come first-served and nothing can starve).
// A scheduler thread
//   1. retires finished launches: copies each request's votes to the
//      caller's buffer, releases its ring space, records submit -> ready
//      time; a launch that failed puts its requests back at the head of the
//      queue, in order, with their ring space kept (a request fails after
//      max_retries such attempts);
//   2. when a launch slot is free, takes the longest run of admitted requests
//      at the head of the queue (up to the coalescing cap) and issues one
//      launch for all of them: rows to the device, the batched persistent
//      kernel over every request, votes back.  Requests admitted one after
//      another sit next to each other in the rings, so a launch needs one or
//      two copies each way.
// Up to max_inflight launches overlap.  Requests arriving while launches run
// join the next launch: continuous batching.  The device work is behind an
// executor interface (serve_exec.h): HIP on the GPU, or a CPU fake for tests
// of the scheduler.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <system_error>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fp_internal.h"
#include "serve_exec.h"

using Clock = std::chrono::steady_clock;

namespace {

constexpr size_t kAlign = 256;
constexpr int32_t kMaxJobsPerLaunch = 4096;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

enum State { kStaging = 0, kWaiting, kQueued, kInflight, kDone, kFailed };

struct Request {
    uint64_t ticket = 0;
    const fp_packed* packed = nullptr;
    int64_t n_rows = 0, ld = 0;
    int32_t F = 0, C = 0;
    int32_t attempts = 0;       // launches that failed for this request
    std::vector<float> heap;    // rows kept here while the rings are full
    int32_t* out = nullptr;     // caller's votes buffer
    Clock::time_point t_submit, t_done;
    size_t x_start = 0, x_size = 0, v_start = 0, v_size = 0;
    State state = kStaging;
};

// Ring allocator over [0, cap): blocks are taken at the head and released in
// any order; the tail advances over released blocks.
struct Ring {
    struct Block {
        size_t start, size;
        bool done;
    };
    size_t cap = 0;
    std::deque<Block> blocks;

    bool alloc(size_t size, size_t* start) {
        if (size > cap) return false;
        if (blocks.empty()) {
            *start = 0;
        } else {
            const size_t tail = blocks.front().start;
            const size_t head = blocks.back().start + blocks.back().size;
            const bool wrapped = blocks.back().start < blocks.front().start;
            if (!wrapped) {
                if (head + size <= cap) *start = head;
                else if (size <= tail) *start = 0;
                else return false;
            } else {
                if (head + size <= tail) *start = head;
                else return false;
            }
        }
        blocks.push_back(Block{*start, size, false});
        return true;
    }
    void release(size_t start) {
        for (auto& b : blocks)
            if (b.start == start && !b.done) {
                b.done = true;
                break;
            }
        while (!blocks.empty() && blocks.front().done) blocks.pop_front();
    }
};

struct Slot {
    bool busy = false;
    std::vector<Request*> reqs;
};

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    size_t k = (size_t)std::min<double>((double)v.size() - 1, std::floor(q * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + (long)k, v.end());
    return v[k];
}

// ---------------------------------------------------------------------------
// CPU fake executor: host rings, launches that complete after a set delay,
// an injectable failure every k-th launch, and a row checksum in place of
// the classification (documented with FP_EXECUTOR_CPU_FAKE).
// ---------------------------------------------------------------------------
class FakeExecutor final : public fp::ServeExecutor {
   public:
    int init(const fp_server_opts& o, size_t xcap, size_t vcap, int n_slots) override {
        opts_ = o;
        x_.assign(xcap, 0);
        v_.assign(vcap, 0);
        slots_.resize(n_slots);
        return FP_OK;
    }
    uint8_t* host_rows() override { return x_.data(); }
    uint8_t* host_votes() override { return v_.data(); }
    int device() const override { return -1; }
    int check_forest(const fp_packed*) override { return FP_OK; }

    int issue(int slot, const std::vector<fp::ServeItem>& batch) override {
        FakeSlot& s = slots_[slot];
        s.batch = batch;
        s.due = Clock::now() + std::chrono::microseconds(std::max(0, opts_.fake_delay_us));
        s.fail = opts_.fake_fail_every > 0 && ++launches_ % opts_.fake_fail_every == 0;
        s.done = false;
        return FP_OK;
    }

    int query(int slot) override {
        FakeSlot& s = slots_[slot];
        if (!s.done) {
            if (Clock::now() < s.due) return FP_ENOTREADY;
            if (!s.fail)
                for (const fp::ServeItem& it : s.batch) checksum_votes(it);
            s.done = true;
        }
        return s.fail ? fp_set_error(FP_EHIP, "injected launch failure") : FP_OK;
    }

    void drain(int slot) override { slots_[slot].done = true; }

   private:
    void checksum_votes(const fp::ServeItem& it) {
        const uint8_t* rows = x_.data() + it.x_start;
        int32_t* votes = reinterpret_cast<int32_t*>(v_.data() + it.v_start);
        for (int64_t i = 0; i < it.n_rows; i++) {
            uint32_t h = 2166136261u;
            const uint8_t* b = rows + (size_t)i * it.F * sizeof(float);
            for (size_t k = 0; k < (size_t)it.F * sizeof(float); k++) h = (h ^ b[k]) * 16777619u;
            for (int32_t c = 0; c < it.C; c++) votes[i * it.C + c] = (int32_t)((h ^ ((uint32_t)c * 0x9E3779B9u)) & 0x7FFFFFFFu);
        }
    }

    struct FakeSlot {
        std::vector<fp::ServeItem> batch;
        Clock::time_point due;
        bool fail = false, done = true;
    };
    fp_server_opts opts_{};
    std::vector<uint8_t> x_, v_;
    std::vector<FakeSlot> slots_;
    int64_t launches_ = 0;
};

}  // namespace

namespace fp {
std::unique_ptr<ServeExecutor> make_fake_executor() { return std::unique_ptr<ServeExecutor>(new FakeExecutor()); }
}  // namespace fp

struct fp_server {
    fp_server_opts opts{};
    std::unique_ptr<fp::ServeExecutor> exec;
    std::vector<const fp_packed*> forests;
    uint8_t *h_x = nullptr, *h_v = nullptr;
    Ring xring, vring;
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;  // arrival order; Staging / Waiting / Queued
    int64_t n_waiting = 0;       // requests holding a heap copy (rings were full)
    std::unordered_map<uint64_t, Request*> tickets;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool completed_notify = false;
    std::thread sched;

    int64_t submitted = 0, completed = 0, rejected = 0, launches = 0, rows = 0;
    int64_t failed_launches = 0, retried = 0, failed = 0;
    std::vector<double> lat_ms;
    Clock::time_point t0 = Clock::now();
    std::string thread_error;

    ~fp_server() {
        exec.reset();  // releases device memory before the requests' bookkeeping
        for (auto& kv : tickets) delete kv.second;
    }

    // Reserve ring space for r (under the lock).
    bool reserve(Request* r) {
        size_t xs = 0, vs = 0;
        if (!xring.alloc(r->x_size, &xs)) return false;
        if (!vring.alloc(r->v_size, &vs)) {
            xring.blocks.pop_back();
            return false;
        }
        r->x_start = xs;
        r->v_start = vs;
        return true;
    }

    // Retires slot s (under the lock).  ok: the votes are in the host ring.
    // Failed: requests with attempts left go back to the head of the queue,
    // in their order, keeping their ring space; the others fail.
    void finish_slot(Slot& s, bool ok) {
        const auto now = Clock::now();
        if (!ok) failed_launches++;
        std::vector<Request*> again;
        for (Request* r : s.reqs) {
            if (!ok && (opts.max_retries < 0 || r->attempts < opts.max_retries)) {
                r->attempts++;
                r->state = kQueued;
                again.push_back(r);
                retried++;
                continue;
            }
            if (ok) memcpy(r->out, h_v + r->v_start, (size_t)r->n_rows * r->C * sizeof(int32_t));
            r->t_done = now;
            r->state = ok ? kDone : kFailed;
            xring.release(r->x_start);
            vring.release(r->v_start);
            lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
            completed++;
            if (!ok) failed++;
        }
        for (auto it = again.rbegin(); it != again.rend(); ++it) queue.push_front(*it);
        s.reqs.clear();
        s.busy = false;
        completed_notify = true;
    }

    // Move waiting requests (heap copies) into the rings, oldest first; stop
    // at the first one that does not fit or is still being copied, so ring
    // space is always handed out in arrival order.
    void admit_waiting() {
        for (Request* r : queue) {
            if (r->state == kQueued || (r->state == kStaging && r->heap.empty())) continue;  // already in the rings
            if (r->state != kWaiting) return;  // heap copy still in progress
            if (!reserve(r)) return;
            memcpy(h_x + r->x_start, r->heap.data(), r->heap.size() * sizeof(float));
            std::vector<float>().swap(r->heap);
            r->state = kQueued;
            n_waiting--;
        }
    }

    void run() {
        exec->bind_thread();
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            bool any_busy = false;
            for (size_t k = 0; k < slots.size(); k++) {
                Slot& s = slots[k];
                if (!s.busy) continue;
                const int q = exec->query((int)k);
                if (q == FP_OK) {
                    finish_slot(s, true);
                } else if (q != FP_ENOTREADY) {
                    thread_error = fp_last_error();
                    exec->drain((int)k);
                    finish_slot(s, false);
                } else {
                    any_busy = true;
                }
            }
            if (completed_notify) {
                completed_notify = false;
                cv_done.notify_all();
            }
            if (stop && !any_busy) break;
            if (n_waiting) admit_waiting();
            int free_slot = -1;
            for (size_t k = 0; k < slots.size(); k++)
                if (!slots[k].busy) {
                    free_slot = (int)k;
                    break;
                }
            if (!stop && free_slot >= 0 && !queue.empty() && queue.front()->state == kQueued) {
                std::vector<Request*> batch;
                std::vector<fp::ServeItem> items;
                int64_t rows_total = 0;
                while (!queue.empty() && queue.front()->state == kQueued && (int32_t)batch.size() < kMaxJobsPerLaunch) {
                    Request* r = queue.front();
                    if (!batch.empty() && rows_total + r->n_rows > opts.max_rows_per_launch) break;
                    rows_total += r->n_rows;
                    r->state = kInflight;
                    batch.push_back(r);
                    items.push_back(fp::ServeItem{r->packed, r->n_rows, r->F, r->C, r->x_start, r->x_size, r->v_start,
                                                  r->v_size});
                    queue.pop_front();
                }
                Slot& s = slots[free_slot];
                s.busy = true;
                s.reqs = batch;
                launches++;
                rows += rows_total;
                lk.unlock();
                const int rc = exec->issue(free_slot, items);
                lk.lock();
                if (rc) {
                    thread_error = fp_last_error();
                    finish_slot(s, false);
                }
                continue;
            }
            if (any_busy) cv_work.wait_for(lk, std::chrono::microseconds(20));
            else if (!stop) cv_work.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
};

extern "C" int fp_server_create(const fp_server_opts* opts, fp_server** out) {
    fp_clear_error();
    if (!out) return fp_set_error(FP_EINVAL, "out is NULL");
    *out = nullptr;
    try {
        std::unique_ptr<fp_server> s(new fp_server());
        if (opts) s->opts = *opts;
        fp_server_opts& o = s->opts;
        if (o.hbm_budget_bytes <= 0) o.hbm_budget_bytes = 1ll << 30;
        if (o.max_rows_per_launch <= 0) o.max_rows_per_launch = 262144;
        if (o.max_inflight <= 0) o.max_inflight = 4;
        if (o.max_queue <= 0) o.max_queue = 1 << 20;
        // as batched plans: two 1024-thread workgroups per CU (p50 0.19 ms,
        // p99 0.9 ms at 20,000 requests/s, against 0.25 / 1.1 ms for 512 x 4)
        if (o.block_threads <= 0) o.block_threads = 1024;
        if (o.cursors <= 0) o.cursors = 2;
        if (o.max_retries == 0) o.max_retries = 2;
        else if (o.max_retries < 0) o.max_retries = 0;
        if (o.block_threads % 64 || o.block_threads > 1024)
            return fp_set_error(FP_EINVAL, "block_threads %d must be a multiple of 64 in [64, 1024]", o.block_threads);
        if (o.cursors != 1 && o.cursors != 2 && o.cursors != 4 && o.cursors != 8)
            return fp_set_error(FP_EINVAL, "cursors must be 1, 2, 4 or 8");
        if (o.max_inflight > 64) return fp_set_error(FP_EINVAL, "max_inflight %d exceeds 64", o.max_inflight);
        if (o.hbm_budget_bytes < (int64_t)(1 << 20)) return fp_set_error(FP_EINVAL, "hbm_budget_bytes below 1 MiB");
        if (o.executor != FP_EXECUTOR_HIP && o.executor != FP_EXECUTOR_CPU_FAKE)
            return fp_set_error(FP_EINVAL, "unknown executor %d", o.executor);
        if (o.fake_delay_us < 0 || o.fake_fail_every < 0)
            return fp_set_error(FP_EINVAL, "fake_delay_us and fake_fail_every must be >= 0");
        // votes take 1/8 of the budget: C*4 bytes per row against F*4 for rows
        const size_t vcap = align_up((size_t)o.hbm_budget_bytes / 8);
        const size_t xcap = align_up((size_t)o.hbm_budget_bytes - vcap);
        s->xring.cap = xcap;
        s->vring.cap = vcap;
        s->exec = o.executor == FP_EXECUTOR_CPU_FAKE ? fp::make_fake_executor() : fp::make_hip_executor();
        int rc = s->exec->init(o, xcap, vcap, o.max_inflight);
        if (rc) return rc;
        s->h_x = s->exec->host_rows();
        s->h_v = s->exec->host_votes();
        s->slots.resize(o.max_inflight);
        fp_server* raw = s.get();
        s->sched = std::thread([raw] { raw->run(); });
        *out = s.release();
        return FP_OK;
    } catch (const std::bad_alloc&) {
        return fp_set_error(FP_ENOMEM, "out of host memory");
    } catch (const std::system_error&) {
        return fp_set_error(FP_ENOMEM, "cannot start the scheduler thread");
    }
}

extern "C" int fp_server_add_forest(fp_server* s, const fp_packed* p, int32_t* forest_id) {
    fp_clear_error();
    if (!s || !p || !forest_id) return fp_set_error(FP_EINVAL, "NULL argument");
    if (p->hdr.layout == FP_LAYOUT_NAIVE)
        return fp_set_error(FP_EINVAL, "forest is not in a packed layout");
    int rc = s->exec->check_forest(p);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(s->mu);
    s->forests.push_back(p);
    *forest_id = (int32_t)s->forests.size() - 1;
    return FP_OK;
}

extern "C" int fp_serve_submit(fp_server* s, int32_t forest_id, const float* X, int64_t n_rows, int64_t ld,
                               int32_t* votes_out, uint64_t* ticket) {
    fp_clear_error();
    if (!s || !ticket) return fp_set_error(FP_EINVAL, "NULL argument");
    Request* r = nullptr;
    bool staged = false;
    try {
        std::unique_ptr<Request> req(new Request());
        std::lock_guard<std::mutex> lk(s->mu);
        if (forest_id < 0 || forest_id >= (int32_t)s->forests.size())
            return fp_set_error(FP_EINVAL, "unknown forest id %d", forest_id);
        const fp_packed* p = s->forests[forest_id];
        const int32_t F = p->hdr.n_features, C = p->hdr.n_classes;
        if (n_rows < 1 || n_rows > INT32_MAX) return fp_set_error(FP_EINVAL, "n_rows %lld must be >= 1", (long long)n_rows);
        if (ld < F) return fp_set_error(FP_EINVAL, "ld %lld < n_features %d", (long long)ld, F);
        if (!X || !votes_out) return fp_set_error(FP_EINVAL, "X or votes is NULL");
        req->packed = p;
        req->n_rows = n_rows;
        req->ld = ld;
        req->F = F;
        req->C = C;
        req->out = votes_out;
        req->x_size = align_up((size_t)n_rows * F * sizeof(float));
        req->v_size = align_up((size_t)n_rows * C * sizeof(int32_t));
        if (req->x_size > s->xring.cap || req->v_size > s->vring.cap)
            return fp_set_error(FP_E2BIG, "request needs %zu + %zu bytes of staging; the HBM budget allows %zu + %zu",
                                req->x_size, req->v_size, s->xring.cap, s->vring.cap);
        if (n_rows > s->opts.max_rows_per_launch)
            return fp_set_error(FP_E2BIG, "request of %lld rows exceeds max_rows_per_launch %lld", (long long)n_rows,
                                (long long)s->opts.max_rows_per_launch);
        if ((int64_t)s->queue.size() >= s->opts.max_queue) {
            s->rejected++;
            return fp_set_error(FP_EAGAIN, "request queue full (%d pending)", s->opts.max_queue);
        }
        // admission: ring space now (and nobody older is waiting), else a heap copy
        staged = s->n_waiting == 0 && s->reserve(req.get());
        if (!staged) req->heap.resize((size_t)n_rows * F);
        req->state = kStaging;
        req->t_submit = Clock::now();
        req->ticket = s->next_ticket++;
        *ticket = req->ticket;
        r = req.release();
        s->tickets[r->ticket] = r;
        s->queue.push_back(r);
        s->submitted++;
        if (!staged) s->n_waiting++;
    } catch (const std::bad_alloc&) {
        return fp_set_error(FP_ENOMEM, "out of host memory");
    }
    // copy the rows outside the lock; the request cannot launch or be moved
    // into the rings before its state leaves kStaging
    float* dst = staged ? reinterpret_cast<float*>(s->h_x + r->x_start) : r->heap.data();
    if (r->ld == r->F) {
        memcpy(dst, X, (size_t)n_rows * r->F * sizeof(float));
    } else {
        for (int64_t i = 0; i < n_rows; i++) memcpy(dst + i * r->F, X + i * r->ld, (size_t)r->F * sizeof(float));
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->state = staged ? kQueued : kWaiting;
    }
    s->cv_work.notify_one();
    return FP_OK;
}

extern "C" int fp_serve_poll(fp_server* s, uint64_t ticket, int64_t timeout_us) {
    fp_clear_error();
    if (!s) return fp_set_error(FP_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fp_set_error(FP_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second;
    auto ready = [&] { return r->state == kDone || r->state == kFailed; };
    if (!ready()) {
        if (timeout_us == 0) return FP_ENOTREADY;
        if (timeout_us < 0) s->cv_done.wait(lk, ready);
        else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) return FP_ENOTREADY;
    }
    const State state = r->state;
    s->tickets.erase(ticket);
    delete r;
    if (state == kFailed) return fp_set_error(FP_EHIP, "the request's launch failed: %s", s->thread_error.c_str());
    return FP_OK;
}

extern "C" int fp_server_stats(fp_server* s, fp_serve_stats* out) {
    fp_clear_error();
    if (!s || !out) return fp_set_error(FP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    memset(out, 0, sizeof *out);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->rejected = s->rejected;
    out->launches = s->launches;
    out->rows = s->rows;
    out->pending = (int64_t)s->queue.size();
    for (auto& sl : s->slots) out->inflight += sl.busy ? 1 : 0;
    if (!s->lat_ms.empty()) {
        double sum = 0, mx = 0;
        for (double v : s->lat_ms) {
            sum += v;
            mx = std::max(mx, v);
        }
        out->mean_ms = sum / (double)s->lat_ms.size();
        out->max_ms = mx;
        out->p50_ms = percentile(s->lat_ms, 0.50);
        out->p99_ms = percentile(s->lat_ms, 0.99);
    }
    out->mean_rows_per_launch = s->launches ? (double)s->rows / (double)s->launches : 0.0;
    out->elapsed_s = std::chrono::duration<double>(Clock::now() - s->t0).count();
    out->failed_launches = s->failed_launches;
    out->retried = s->retried;
    out->failed = s->failed;
    return FP_OK;
}

extern "C" int fp_server_reset_stats(fp_server* s) {
    fp_clear_error();
    if (!s) return fp_set_error(FP_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    s->submitted = s->completed = s->rejected = s->launches = s->rows = 0;
    s->failed_launches = s->retried = s->failed = 0;
    s->lat_ms.clear();
    s->t0 = Clock::now();
    return FP_OK;
}

extern "C" void fp_server_destroy(fp_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->sched.joinable()) s->sched.join();
    delete s;  // requests never launched are dropped with their tickets
}

// ---------------------------------------------------------------------------
// open-loop load driver
// ---------------------------------------------------------------------------
extern "C" int fp_serve_replay(fp_server* s, const fp_replay_request* reqs, int64_t n, int32_t submit_threads,
                               double* latency_ms, double* lag_ms) {
    fp_clear_error();
    if (!s || (n > 0 && (!reqs || !latency_ms || !lag_ms))) return fp_set_error(FP_EINVAL, "NULL argument");
    if (n <= 0) return FP_OK;
    const int T = std::max(1, std::min<int32_t>(submit_threads, 64));
    std::vector<uint64_t> tickets((size_t)n, 0);
    std::vector<int> rcs((size_t)n, FP_OK);
    std::vector<std::atomic<int>> posted((size_t)n);
    for (auto& p : posted) p.store(0);
    const Clock::time_point start = Clock::now() + std::chrono::milliseconds(2);
    auto due = [&](int64_t i) {
        return start + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(reqs[i].arrival_s));
    };
    std::vector<std::thread> th;
    try {
        for (int k = 0; k < T; k++)
            th.emplace_back([&, k] {
                for (int64_t i = k; i < n; i += T) {
                    const auto d = due(i);
                    auto now = Clock::now();
                    if (d - now > std::chrono::microseconds(200)) std::this_thread::sleep_until(d - std::chrono::microseconds(100));
                    while (Clock::now() < d) {
                    }
                    const fp_replay_request& q = reqs[i];
                    rcs[i] = fp_serve_submit(s, q.forest_id, q.X_host, q.n_rows, q.ld, q.votes_host_out, &tickets[i]);
                    lag_ms[i] = std::chrono::duration<double, std::milli>(Clock::now() - d).count();
                    posted[i].store(1, std::memory_order_release);
                }
            });
    } catch (const std::system_error&) {
        for (auto& t : th) t.join();
        return fp_set_error(FP_ENOMEM, "cannot start submit threads");
    }
    int first_error = FP_OK;
    for (int64_t i = 0; i < n; i++) {
        while (!posted[i].load(std::memory_order_acquire)) std::this_thread::yield();
        if (rcs[i] != FP_OK) {
            latency_ms[i] = -1.0;
            if (!first_error) first_error = rcs[i];
            continue;
        }
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->tickets.find(tickets[i]);
        if (it == s->tickets.end()) {
            latency_ms[i] = -1.0;
            continue;
        }
        Request* r = it->second;
        s->cv_done.wait(lk, [&] { return r->state == kDone || r->state == kFailed; });
        latency_ms[i] = r->state == kDone ? std::chrono::duration<double, std::milli>(r->t_done - due(i)).count() : -1.0;
        if (r->state == kFailed && !first_error) first_error = FP_EHIP;
        s->tickets.erase(it);
        delete r;
    }
    for (auto& t : th) t.join();
    if (first_error) return fp_set_error(first_error, "replay: some requests failed (latency -1)");
    return FP_OK;
}
