// HIP executor of the serving loop: staging rings in HBM mirrored by pinned
// host rings at the same offsets, and per launch slot a stream, a completion
// event and a table buffer.  A launch copies the batch's rows to the device
// (one copy per run of adjacent ring blocks), runs the batched persistent
// kernel over every request of the batch, copies the votes back and
// records the slot's event.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <system_error>
#include <thread>

#include "fp_internal.h"
#include "serve_exec.h"

namespace {

constexpr size_t kAlign = 256;
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

struct HipSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void* d_tables = nullptr;
    void* h_tables = nullptr;
};

class HipExecutor final : public fp::ServeExecutor {
   public:
    ~HipExecutor() override {
        for (auto& s : slots_) {
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            if (s.d_tables) (void)hipFree(s.d_tables);
            if (s.h_tables) (void)hipHostFree(s.h_tables);
        }
        if (d_x_) (void)hipFree(d_x_);
        if (d_v_) (void)hipFree(d_v_);
        if (h_x_) (void)hipHostFree(h_x_);
        if (h_v_) (void)hipHostFree(h_v_);
    }

    int init(const fp_server_opts& o, size_t xcap, size_t vcap, int n_slots) override {
        opts_ = o;
        int rc = fp::current_device(&dev_);
        if (rc) return rc;
        rc = fp::device_props(dev_, &dp_);
        if (rc) return rc;
        // jobs may fill half a CU's LDS, so that with the launch's item slot
        // one workgroup holds a CU: serving launches are small, and a launch
        // spread over more workgroups than CUs measured higher latency on
        // the 8-forest Poisson stream (p50 0.64 ms against 0.55 ms)
        lds_block_ = std::min(fp::default_lds_block(dp_),
                              fp::batched_job_budget(dp_.lds_per_block ? dp_.lds_per_block : 65536));
        hipError_t e = hipMalloc((void**)&d_x_, xcap);
        if (e == hipSuccess) e = hipMalloc((void**)&d_v_, vcap);
        if (e != hipSuccess) return fp_set_error(FP_ENOMEM, "hipMalloc staging: %s", hipGetErrorString(e));
        e = hipHostMalloc((void**)&h_x_, xcap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&h_v_, vcap, hipHostMallocDefault);
        if (e != hipSuccess) return fp_set_error(FP_ENOMEM, "hipHostMalloc staging: %s", hipGetErrorString(e));
        touch_pages(h_x_, xcap);
        touch_pages(h_v_, vcap);
        slots_.resize(n_slots);
        for (auto& sl : slots_) {
            e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
            if (e != hipSuccess) return fp_set_error(FP_EHIP, "slot stream / event: %s", hipGetErrorString(e));
            e = hipMalloc(&sl.d_tables, kTableBytes);
            if (e == hipSuccess) e = hipHostMalloc(&sl.h_tables, kTableBytes, hipHostMallocDefault);
            if (e != hipSuccess) return fp_set_error(FP_ENOMEM, "slot tables: %s", hipGetErrorString(e));
        }
        return FP_OK;
    }

    uint8_t* host_rows() override { return h_x_; }
    uint8_t* host_votes() override { return h_v_; }
    int device() const override { return dev_; }

    int check_forest(const fp_packed* p) override {
        if (!p->dev) return fp_set_error(FP_ENODEV, "forest is not uploaded");
        if (p->dev_id != dev_) return fp_set_error(FP_ENODEV, "forest on device %d, server on device %d", p->dev_id, dev_);
        fp::JobDesc j;  // the forest's launch parameters must fit the server's LDS budget
        fp_tune t = p->tune;
        return fp::resolve_job(p, &t, nullptr, 1, p->hdr.n_features, nullptr, nullptr, lds_block_, &j);
    }

    void bind_thread() override { (void)hipSetDevice(dev_); }

    int issue(int slot, const std::vector<fp::ServeItem>& batch) override {
        HipSlot& s = slots_[slot];
        std::vector<fp::JobDesc> jobs(batch.size());
        std::vector<double> depth(batch.size());
        size_t lds = 0;
        for (size_t i = 0; i < batch.size(); i++) {
            const fp::ServeItem& r = batch[i];
            fp_tune t = r.packed->tune;
            int rc = fp::resolve_job(r.packed, &t, reinterpret_cast<const float*>(d_x_ + r.x_start), r.n_rows, r.F,
                                     reinterpret_cast<int32_t*>(d_v_ + r.v_start), nullptr, lds_block_, &jobs[i]);
            if (rc) return rc;
            fp::flatten_passes(&jobs[i]);
            lds = std::max(lds, (size_t)jobs[i].lds_bytes);
            depth[i] = r.packed->hdr.expected_depth;
        }
        int occ = 1;
        const bool blocks_only = fp::jobs_blocks_only(jobs.data(), (int32_t)jobs.size());
        int rc = fp::batched_occupancy(opts_.cursors, blocks_only, opts_.block_threads, lds, &occ);
        if (rc) return rc;
        const int64_t resident = (int64_t)dp_.cus * occ;
        std::vector<fp::WorkItem> items;
        double cost = 0;
        const size_t jobs_bytes = align_up(jobs.size() * sizeof(fp::JobDesc));
        for (int ipb = 4;; ipb /= 2) {
            fp::build_items(jobs, depth, resident, ipb, &items, &cost);
            if (jobs_bytes + items.size() * sizeof(fp::WorkItem) + kAlign <= kTableBytes) break;
            if (ipb == 1) return fp_set_error(FP_E2BIG, "launch tables exceed %zu bytes", kTableBytes);
        }
        memcpy(s.h_tables, jobs.data(), jobs.size() * sizeof(fp::JobDesc));
        memcpy(static_cast<uint8_t*>(s.h_tables) + jobs_bytes, items.data(), items.size() * sizeof(fp::WorkItem));
        uint8_t* dt = static_cast<uint8_t*>(s.d_tables);
        int32_t* counter = reinterpret_cast<int32_t*>(dt + kTableBytes - kAlign);
        hipError_t e = hipMemcpyAsync(dt, s.h_tables, jobs_bytes + items.size() * sizeof(fp::WorkItem),
                                      hipMemcpyHostToDevice, s.stream);
        // rows: one copy per run of adjacent ring blocks
        for (size_t i = 0; i < batch.size() && e == hipSuccess;) {
            size_t j = i + 1, end = batch[i].x_start + batch[i].x_size;
            while (j < batch.size() && batch[j].x_start == end) end += batch[j++].x_size;
            e = hipMemcpyAsync(d_x_ + batch[i].x_start, h_x_ + batch[i].x_start, end - batch[i].x_start,
                               hipMemcpyHostToDevice, s.stream);
            i = j;
        }
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(s.stream);
            return fp_set_error(FP_EHIP, "hipMemcpyAsync: %s", hipGetErrorString(e));
        }
        const fp::JobDesc* jobs_dev = reinterpret_cast<const fp::JobDesc*>(dt);
        const fp::WorkItem* items_dev = reinterpret_cast<const fp::WorkItem*>(dt + jobs_bytes);
        rc = fp::launch_batched_prologue(jobs_dev, (int32_t)jobs.size(), counter, s.stream);
        const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(resident, (int64_t)items.size()));
        if (!rc)
            rc = fp::launch_batched(jobs_dev, items_dev, (int32_t)items.size(), counter, opts_.cursors, blocks_only,
                                    opts_.block_threads, lds, blocks, s.stream);
        if (rc) {
            (void)hipStreamSynchronize(s.stream);
            return rc;
        }
        for (size_t i = 0; i < batch.size() && e == hipSuccess;) {
            size_t j = i + 1, end = batch[i].v_start + batch[i].v_size;
            while (j < batch.size() && batch[j].v_start == end) end += batch[j++].v_size;
            e = hipMemcpyAsync(h_v_ + batch[i].v_start, d_v_ + batch[i].v_start, end - batch[i].v_start,
                               hipMemcpyDeviceToHost, s.stream);
            i = j;
        }
        if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(s.stream);
            return fp_set_error(FP_EHIP, "launch copy-back: %s", hipGetErrorString(e));
        }
        return FP_OK;
    }

    int query(int slot) override {
        const hipError_t q = hipEventQuery(slots_[slot].done);
        if (q == hipSuccess) return FP_OK;
        if (q == hipErrorNotReady) return FP_ENOTREADY;
        return fp_set_error(FP_EHIP, "launch failed: %s", hipGetErrorString(q));
    }

    void drain(int slot) override { (void)hipStreamSynchronize(slots_[slot].stream); }

   private:
    fp_server_opts opts_{};
    int dev_ = -1;
    fp::DeviceProps dp_;
    size_t lds_block_ = 0;
    uint8_t *d_x_ = nullptr, *h_x_ = nullptr, *d_v_ = nullptr, *h_v_ = nullptr;
    std::vector<HipSlot> slots_;
};

}  // namespace

namespace fp {
std::unique_ptr<ServeExecutor> make_hip_executor() { return std::unique_ptr<ServeExecutor>(new HipExecutor()); }
}  // namespace fp
