// Serving loop: continuous batching of prediction requests on resident
// packed forests.
//
// Staging memory is two rings in HBM (observations, votes), each mirrored by
// a pinned host ring at the same offsets; the HBM budget is their total.
// Admission = getting ring space.  fp_serve_submit reserves space for the
// request (in arrival order) and copies its rows straight into the pinned
// ring; when the rings are full it keeps a heap copy instead and the request
// waits (requests behind it wait too, so admission stays first-come
// first-served and nothing can starve).  A scheduler thread
//   1. retires finished launches (event query): copies each request's votes
//      to the caller's buffer, releases its ring space, records
//      submit -> ready time;
//   2. when a launch slot is free, takes the longest run of admitted requests
//      at the head of the queue (up to the coalescing cap) and issues one
//      launch for all of them on the slot's stream: H2D of their rows, the
//      batched persistent kernel over every request, D2H of their votes.
//      Requests admitted one after another sit next to each other in the
//      rings, so a launch needs one or two copies each way.
// Up to max_inflight launches overlap.  Requests arriving while launches run
// join the next launch: continuous batching.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <system_error>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fp_internal.h"

using Clock = std::chrono::steady_clock;
using fp::JobDesc;
using fp::WorkItem;

namespace {

constexpr size_t kAlign = 256;
constexpr int32_t kMaxJobsPerLaunch = 4096;
constexpr size_t kTableBytes = 4u << 20;  // per slot: job table + work items

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Writes one byte of every 4 KiB page of a fresh host buffer (several
// threads for large buffers), so that its pages are mapped before requests
// stream through it: left to the first pass of requests through the rings,
// the page faults held submits back by up to half a second.
void touch_pages(void* p, size_t n) {
    volatile uint8_t* b = static_cast<uint8_t*>(p);
    auto run = [b](size_t lo, size_t hi) {
        for (size_t i = lo; i < hi; i += 4096) b[i] = 0;
    };
    const size_t kSlice = size_t(256) << 20;
    if (n <= kSlice) {
        run(0, n);
        return;
    }
    const size_t T = std::min<size_t>(8, (n + kSlice - 1) / kSlice);
    const size_t per = (n / T + 4095) / 4096 * 4096;
    std::vector<std::thread> th;
    try {
        for (size_t t = 1; t < T; t++) th.emplace_back(run, t * per, std::min(n, (t + 1) * per));
    } catch (const std::system_error&) {
        for (size_t t = 1 + th.size(); t < T; t++) run(t * per, std::min(n, (t + 1) * per));  // no more threads
    }
    run(0, std::min(n, per));
    for (auto& t : th) t.join();
}

enum State { kStaging = 0, kWaiting, kQueued, kInflight, kDone, kFailed };

struct Request {
    uint64_t ticket = 0;
    const fp_packed* packed = nullptr;
    int64_t n_rows = 0, ld = 0;
    int32_t F = 0, C = 0;
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
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void* d_tables = nullptr;
    void* h_tables = nullptr;
    bool busy = false;
    std::vector<Request*> reqs;
};

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    size_t k = (size_t)std::min<double>((double)v.size() - 1, std::floor(q * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + (long)k, v.end());
    return v[k];
}

}  // namespace

struct fp_server {
    fp_server_opts opts{};
    int dev = -1;
    fp::DeviceProps dp;
    size_t lds_block = 0;
    std::vector<const fp_packed*> forests;
    uint8_t *d_x = nullptr, *h_x = nullptr, *d_v = nullptr, *h_v = nullptr;
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
    std::vector<double> lat_ms;
    Clock::time_point t0 = Clock::now();
    std::string thread_error;

    ~fp_server() {
        for (auto& s : slots) {
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            if (s.d_tables) (void)hipFree(s.d_tables);
            if (s.h_tables) (void)hipHostFree(s.h_tables);
        }
        if (d_x) (void)hipFree(d_x);
        if (d_v) (void)hipFree(d_v);
        if (h_x) (void)hipHostFree(h_x);
        if (h_v) (void)hipHostFree(h_v);
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

    // Issue one launch for `batch` on slot s (without the lock).
    int issue(Slot& s, const std::vector<Request*>& batch) {
        std::vector<JobDesc> jobs(batch.size());
        std::vector<double> depth(batch.size());
        size_t lds = 0;
        for (size_t i = 0; i < batch.size(); i++) {
            Request* r = batch[i];
            fp_tune t = r->packed->tune;
            int rc = fp::resolve_job(r->packed, &t, reinterpret_cast<const float*>(d_x + r->x_start), r->n_rows, r->F,
                                     reinterpret_cast<int32_t*>(d_v + r->v_start), nullptr, lds_block, &jobs[i]);
            if (rc) return rc;
            lds = std::max(lds, (size_t)jobs[i].lds_bytes);
            depth[i] = r->packed->hdr.expected_depth;
        }
        int occ = 1;
        int rc = fp::batched_occupancy(opts.cursors, opts.block_threads, lds, &occ);
        if (rc) return rc;
        const int64_t resident = (int64_t)dp.cus * occ;
        std::vector<WorkItem> items;
        double cost = 0;
        const size_t jobs_bytes = align_up(jobs.size() * sizeof(JobDesc));
        for (int ipb = 4;; ipb /= 2) {
            fp::build_items(jobs, depth, resident, ipb, &items, &cost);
            if (jobs_bytes + items.size() * sizeof(WorkItem) + kAlign <= kTableBytes) break;
            if (ipb == 1) return fp_set_error(FP_E2BIG, "launch tables exceed %zu bytes", kTableBytes);
        }
        memcpy(s.h_tables, jobs.data(), jobs.size() * sizeof(JobDesc));
        memcpy(static_cast<uint8_t*>(s.h_tables) + jobs_bytes, items.data(), items.size() * sizeof(WorkItem));
        uint8_t* dt = static_cast<uint8_t*>(s.d_tables);
        int32_t* counter = reinterpret_cast<int32_t*>(dt + kTableBytes - kAlign);
        hipError_t e = hipMemcpyAsync(dt, s.h_tables, jobs_bytes + items.size() * sizeof(WorkItem),
                                      hipMemcpyHostToDevice, s.stream);
        // rows: one copy per run of adjacent ring blocks
        for (size_t i = 0; i < batch.size() && e == hipSuccess;) {
            size_t j = i + 1, end = batch[i]->x_start + batch[i]->x_size;
            while (j < batch.size() && batch[j]->x_start == end) end += batch[j++]->x_size;
            e = hipMemcpyAsync(d_x + batch[i]->x_start, h_x + batch[i]->x_start, end - batch[i]->x_start,
                               hipMemcpyHostToDevice, s.stream);
            i = j;
        }
        if (e != hipSuccess) return fp_set_error(FP_EHIP, "hipMemcpyAsync: %s", hipGetErrorString(e));
        const JobDesc* jobs_dev = reinterpret_cast<const JobDesc*>(dt);
        const WorkItem* items_dev = reinterpret_cast<const WorkItem*>(dt + jobs_bytes);
        rc = fp::launch_batched_prologue(jobs_dev, (int32_t)jobs.size(), counter, s.stream);
        if (rc) return rc;
        const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(resident, (int64_t)items.size()));
        rc = fp::launch_batched(jobs_dev, items_dev, (int32_t)items.size(), counter, opts.cursors, opts.block_threads,
                                lds, blocks, s.stream);
        if (rc) return rc;
        for (size_t i = 0; i < batch.size() && e == hipSuccess;) {
            size_t j = i + 1, end = batch[i]->v_start + batch[i]->v_size;
            while (j < batch.size() && batch[j]->v_start == end) end += batch[j++]->v_size;
            e = hipMemcpyAsync(h_v + batch[i]->v_start, d_v + batch[i]->v_start, end - batch[i]->v_start,
                               hipMemcpyDeviceToHost, s.stream);
            i = j;
        }
        if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
        if (e != hipSuccess) return fp_set_error(FP_EHIP, "launch copy-back: %s", hipGetErrorString(e));
        return FP_OK;
    }

    void finish_slot(Slot& s, bool ok) {
        const auto now = Clock::now();
        for (Request* r : s.reqs) {
            if (ok) memcpy(r->out, h_v + r->v_start, (size_t)r->n_rows * r->C * sizeof(int32_t));
            r->t_done = now;
            r->state = ok ? kDone : kFailed;
            xring.release(r->x_start);
            vring.release(r->v_start);
            lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
            completed++;
        }
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
        if (hipSetDevice(dev) != hipSuccess) thread_error = "hipSetDevice failed in the scheduler";
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            bool any_busy = false;
            for (auto& s : slots) {
                if (!s.busy) continue;
                const hipError_t q = hipEventQuery(s.done);
                if (q == hipSuccess) finish_slot(s, true);
                else if (q != hipErrorNotReady) finish_slot(s, false);
                else any_busy = true;
            }
            if (completed_notify) {
                completed_notify = false;
                cv_done.notify_all();
            }
            if (stop && !any_busy) break;
            if (n_waiting) admit_waiting();
            Slot* free_slot = nullptr;
            for (auto& s : slots)
                if (!s.busy) {
                    free_slot = &s;
                    break;
                }
            if (!stop && free_slot && !queue.empty() && queue.front()->state == kQueued) {
                std::vector<Request*> batch;
                int64_t rows_total = 0;
                while (!queue.empty() && queue.front()->state == kQueued && (int32_t)batch.size() < kMaxJobsPerLaunch) {
                    Request* r = queue.front();
                    if (!batch.empty() && rows_total + r->n_rows > opts.max_rows_per_launch) break;
                    rows_total += r->n_rows;
                    r->state = kInflight;
                    batch.push_back(r);
                    queue.pop_front();
                }
                free_slot->busy = true;
                free_slot->reqs = batch;
                launches++;
                rows += rows_total;
                lk.unlock();
                const int rc = issue(*free_slot, batch);
                lk.lock();
                if (rc) {
                    thread_error = fp_last_error();
                    (void)hipStreamSynchronize(free_slot->stream);
                    finish_slot(*free_slot, false);
                }
                continue;
            }
            if (any_busy) cv_work.wait_for(lk, std::chrono::microseconds(20));
            else if (!stop) cv_work.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
};

#define HIPCHK(call)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) return fp_set_error(FP_EHIP, "%s: %s", #call, hipGetErrorString(e_));   \
    } while (0)

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
        if (o.block_threads % 64 || o.block_threads > 1024)
            return fp_set_error(FP_EINVAL, "block_threads %d must be a multiple of 64 in [64, 1024]", o.block_threads);
        if (o.cursors != 1 && o.cursors != 2 && o.cursors != 4 && o.cursors != 8)
            return fp_set_error(FP_EINVAL, "cursors must be 1, 2, 4 or 8");
        if (o.max_inflight > 64) return fp_set_error(FP_EINVAL, "max_inflight %d exceeds 64", o.max_inflight);
        if (o.hbm_budget_bytes < (int64_t)(1 << 20)) return fp_set_error(FP_EINVAL, "hbm_budget_bytes below 1 MiB");
        int rc = fp::current_device(&s->dev);
        if (rc) return rc;
        rc = fp::device_props(s->dev, &s->dp);
        if (rc) return rc;
        s->lds_block = fp::default_lds_block(s->dp);
        // votes take 1/8 of the budget: C*4 bytes per row against F*4 for rows
        const size_t vcap = align_up((size_t)o.hbm_budget_bytes / 8);
        const size_t xcap = align_up((size_t)o.hbm_budget_bytes - vcap);
        s->xring.cap = xcap;
        s->vring.cap = vcap;
        hipError_t e = hipMalloc((void**)&s->d_x, xcap);
        if (e == hipSuccess) e = hipMalloc((void**)&s->d_v, vcap);
        if (e != hipSuccess) return fp_set_error(FP_ENOMEM, "hipMalloc staging: %s", hipGetErrorString(e));
        e = hipHostMalloc((void**)&s->h_x, xcap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_v, vcap, hipHostMallocDefault);
        if (e != hipSuccess) return fp_set_error(FP_ENOMEM, "hipHostMalloc staging: %s", hipGetErrorString(e));
        touch_pages(s->h_x, xcap);
        touch_pages(s->h_v, vcap);
        s->slots.resize(o.max_inflight);
        for (auto& sl : s->slots) {
            HIPCHK(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
            e = hipMalloc(&sl.d_tables, kTableBytes);
            if (e != hipSuccess) return fp_set_error(FP_ENOMEM, "hipMalloc tables: %s", hipGetErrorString(e));
            e = hipHostMalloc(&sl.h_tables, kTableBytes, hipHostMallocDefault);
            if (e != hipSuccess) return fp_set_error(FP_ENOMEM, "hipHostMalloc tables: %s", hipGetErrorString(e));
        }
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
    if (!p->dev) return fp_set_error(FP_ENODEV, "forest is not uploaded");
    if (p->dev_id != s->dev) return fp_set_error(FP_ENODEV, "forest on device %d, server on device %d", p->dev_id, s->dev);
    fp::JobDesc j;  // the forest's launch parameters must fit the server's LDS budget
    fp_tune t = p->tune;
    int rc = fp::resolve_job(p, &t, nullptr, 1, p->hdr.n_features, nullptr, nullptr, s->lds_block, &j);
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
    return FP_OK;
}

extern "C" int fp_server_reset_stats(fp_server* s) {
    fp_clear_error();
    if (!s) return fp_set_error(FP_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    s->submitted = s->completed = s->rejected = s->launches = s->rows = 0;
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
