// Batched prediction: many resident forests with uneven batches in one
// persistent launch, captured in a hipGraph.
//
// Work list.  Every (job, tree group) is cut into chunks of row tiles; a chunk
// is one work item.  Its estimated cost is rows x trees x expected depth --
// the node-visit count that Eqs. 1-2 of the paper use as the driver of
// run time.  Chunks are sized so that the list holds a few items per
// persistent workgroup, and sorted largest first so the long items start
// early and the small ones fill the tail.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>

#include "fp_internal.h"

using fp::JobDesc;
using fp::WorkItem;

struct fp_plan {
    int dev = -1;
    std::vector<JobDesc> jobs;
    std::vector<WorkItem> items;
    void* dev_mem = nullptr;        // [jobs | items | counter]
    JobDesc* jobs_dev = nullptr;
    WorkItem* items_dev = nullptr;
    int32_t* counter_dev = nullptr;
    int K = 2, threads = 1024, blocks = 1;
    bool blocks_only = false;  // every job in a block layout: the lean kernel variant
    size_t lds_bytes = 0;
    double total_cost = 0.0;
    int32_t jobs_tuned = 0, jobs_cached = 0;
    bool use_graph = true;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~fp_plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        if (dev_mem) (void)hipFree(dev_mem);
    }
};

static int enqueue(fp_plan* p, hipStream_t s) {
    const int32_t n_jobs = (int32_t)p->jobs.size();
    int rc = fp::launch_batched_prologue(p->jobs_dev, n_jobs, p->counter_dev, s);
    if (rc) return rc;
    rc = fp::launch_batched(p->jobs_dev, p->items_dev, (int32_t)p->items.size(), p->counter_dev, p->K,
                            p->blocks_only, p->threads, p->lds_bytes, p->blocks, s);
    if (rc) return rc;
    return fp::launch_batched_epilogue(p->jobs_dev, n_jobs, s);
}

namespace fp {

size_t build_items_into(const JobDesc* jobs, const double* expected_depth, size_t n, int64_t resident,
                        int items_per_block, WorkItem* out, size_t cap, double* total_cost) {
    auto depth = [&](size_t i) { return std::max(1.0, expected_depth[i]); };
    auto tile_cost = [&](size_t i) { return (double)jobs[i].R * jobs[i].trees_per_group * depth(i); };
    double total = 0.0;
    for (size_t i = 0; i < n; i++) {
        const JobDesc& j = jobs[i];
        const int64_t trees = std::min<int64_t>((int64_t)j.n_bins * j.bin_size, (int64_t)j.trees_per_group * j.G);
        total += (double)j.n_rows * trees * depth(i);
    }
    const double target = total / (double)std::max<int64_t>(1, resident * std::max(1, items_per_block));
    size_t k = 0;
    for (size_t i = 0; i < n; i++) {
        const JobDesc& j = jobs[i];
        if (j.n_rows == 0) continue;
        const int chunk =
            (int)std::max(1.0, std::min((double)j.n_tiles, std::floor(target / std::max(tile_cost(i), 1.0))));
        for (int32_t g = 0; g < j.G; g++) {
            if (g * j.bins_per_group >= j.n_bins) break;
            for (int32_t t = 0; t < j.n_tiles; t += chunk, k++)
                if (k < cap) out[k] = WorkItem{(int32_t)i, g, t, std::min(j.n_tiles, t + chunk)};
        }
    }
    *total_cost = total;
    if (k > cap) return k;
    // largest estimated cost first; equal costs keep the order of creation
    // (job, group, first tile), so the list is the same on every call
    std::sort(out, out + k, [&](const WorkItem& a, const WorkItem& b) {
        const double ca = tile_cost(a.job) * (a.tile_end - a.tile_begin);
        const double cb = tile_cost(b.job) * (b.tile_end - b.tile_begin);
        if (ca != cb) return ca > cb;
        if (a.job != b.job) return a.job < b.job;
        if (a.group != b.group) return a.group < b.group;
        return a.tile_begin < b.tile_begin;
    });
    return k;
}

void build_items(const std::vector<JobDesc>& jobs, const std::vector<double>& expected_depth, int64_t resident,
                 int items_per_block, std::vector<WorkItem>* items, double* total_cost) {
    const size_t k = build_items_into(jobs.data(), expected_depth.data(), jobs.size(), resident, items_per_block,
                                      nullptr, 0, total_cost);
    items->resize(k);
    build_items_into(jobs.data(), expected_depth.data(), jobs.size(), resident, items_per_block, items->data(), k,
                     total_cost);
}

}  // namespace fp

#define HIPCHK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) return fp_set_error(FP_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

extern "C" int fp_plan_create(const fp_job* jobs, int32_t n_jobs, const fp_plan_opts* opts, fp_plan** out) {
    fp_clear_error();
    if (!out) return fp_set_error(FP_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_jobs < 1 || !jobs) return fp_set_error(FP_EINVAL, "need at least one job");
    try {
        std::unique_ptr<fp_plan> p(new fp_plan());
        int rc = fp::current_device(&p->dev);
        if (rc) return rc;
        fp::DeviceProps dp;
        rc = fp::device_props(p->dev, &dp);
        if (rc) return rc;
        // 1024-thread workgroups and two cursors: with at most 64 VGPRs two such
        // workgroups share a CU (8 waves per SIMD); 64 forests run 1.9x faster
        // than with 512 threads and four cursors (5 waves per SIMD)
        p->threads = opts && opts->block_threads > 0 ? opts->block_threads : 1024;
        p->K = opts && opts->cursors > 0 ? opts->cursors : 2;
        p->use_graph = opts ? opts->use_graph != 0 : true;
        const bool autotune = opts ? opts->autotune != 0 : true;
        const int items_per_block = opts && opts->items_per_block > 0 ? opts->items_per_block : fp::kDefaultItemsPerBlock;
        if (p->threads % 64 || p->threads < 64 || p->threads > 1024)
            return fp_set_error(FP_EINVAL, "block_threads %d must be a multiple of 64 in [64, 1024]", p->threads);
        if (p->K != 1 && p->K != 2 && p->K != 4 && p->K != 8)
            return fp_set_error(FP_EINVAL, "cursors must be 1, 2, 4 or 8");
        const size_t blk_max = dp.lds_per_block ? dp.lds_per_block : 65536;
        // the jobs' share of the workgroup's LDS (the launch adds the item slot)
        const size_t lds_block = fp::batched_job_budget(
            opts && opts->lds_budget > 0 ? std::min((size_t)opts->lds_budget, blk_max) : fp::default_lds_block(dp));

        // the plan's own stream: launch tuning at creation, then graph capture
        HIPCHK(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking));

        // 1) job descriptors
        p->jobs.resize(n_jobs);
        std::vector<double> depth(n_jobs, 1.0);
        for (int32_t i = 0; i < n_jobs; i++) {
            const fp_job& jb = jobs[i];
            if (!jb.forest) return fp_set_error(FP_EINVAL, "job %d: forest is NULL", i);
            const fp::Header& h = jb.forest->hdr;
            if (jb.n_rows < 0 || jb.n_rows > INT32_MAX) return fp_set_error(FP_EINVAL, "job %d: bad n_rows", i);
            if (jb.ld < h.n_features) return fp_set_error(FP_EINVAL, "job %d: ld %lld < n_features %d", i, (long long)jb.ld, h.n_features);
            if (jb.n_rows > 0 && (!jb.X || !jb.votes)) return fp_set_error(FP_EINVAL, "job %d: X or votes is NULL", i);
            if (!jb.forest->dev) return fp_set_error(FP_ENODEV, "job %d: forest is not uploaded", i);
            if (jb.forest->dev_id != p->dev)
                return fp_set_error(FP_ENODEV, "job %d: forest on device %d, plan on device %d", i, jb.forest->dev_id, p->dev);
            fp_tune t = jb.forest->tune;
            if (autotune && jb.n_rows > 0 && h.layout != FP_LAYOUT_NAIVE) {
                // the tune recorded for (forest, size bucket, threads, cursors), else time it now
                if (fp::launch_tune_get(jb.forest, jb.n_rows, p->threads, p->K, &t)) {
                    p->jobs_cached++;
                } else {
                    double ms = 0.0;
                    int32_t tried = 0;
                    rc = fp::search_launch(jb.forest, jb.X, jb.n_rows, jb.ld, p->threads, p->K, p->capture_stream, &t,
                                           &ms, &tried);
                    if (rc) {
                        std::string msg = fp_last_error();
                        return fp_set_error(rc, "job %d: tuning: %s", i, msg.c_str());
                    }
                    fp::launch_tune_put(jb.forest, jb.n_rows, p->threads, p->K, t);
                    p->jobs_tuned++;
                }
                // candidates are timed with the default LDS budget: a smaller
                // plan budget falls back to the forest's own parameters
                if (fp::resolve_job(jb.forest, &t, jb.X, jb.n_rows, jb.ld, jb.votes, jb.cls, lds_block, &p->jobs[i]) ==
                    FP_E2BIG)
                    t = jb.forest->tune;
            }
            rc = fp::resolve_job(jb.forest, &t, jb.X, jb.n_rows, jb.ld, jb.votes, jb.cls, lds_block, &p->jobs[i]);
            if (rc) {
                std::string msg = fp_last_error();
                return fp_set_error(rc, "job %d: %s", i, msg.c_str());
            }
            fp::flatten_passes(&p->jobs[i]);
            p->lds_bytes = std::max(p->lds_bytes, (size_t)p->jobs[i].lds_bytes);
            depth[i] = h.expected_depth;
        }

        // 2) persistent grid and work items
        int occ = 1;
        p->blocks_only = fp::jobs_blocks_only(p->jobs.data(), (int32_t)p->jobs.size());
        rc = fp::batched_occupancy(p->K, p->blocks_only, p->threads, p->lds_bytes, &occ);
        if (rc) return rc;
        const int64_t resident = (int64_t)dp.cus * occ;
        fp::build_items(p->jobs, depth, resident, items_per_block, &p->items, &p->total_cost);
        p->blocks = (int)std::max<int64_t>(1, std::min<int64_t>(resident, (int64_t)p->items.size()));

        // 3) device tables
        const size_t jobs_b = sizeof(JobDesc) * p->jobs.size();
        const size_t items_off = (jobs_b + 255) / 256 * 256;
        const size_t items_b = sizeof(WorkItem) * std::max<size_t>(1, p->items.size());
        const size_t counter_off = (items_off + items_b + 255) / 256 * 256;
        const size_t total = counter_off + 256;
        hipError_t e = hipMalloc(&p->dev_mem, total);
        if (e != hipSuccess) return fp_set_error(FP_ENOMEM, "hipMalloc(%zu): %s", total, hipGetErrorString(e));
        uint8_t* base = static_cast<uint8_t*>(p->dev_mem);
        p->jobs_dev = reinterpret_cast<JobDesc*>(base);
        p->items_dev = reinterpret_cast<WorkItem*>(base + items_off);
        p->counter_dev = reinterpret_cast<int32_t*>(base + counter_off);
        HIPCHK(hipMemcpy(p->jobs_dev, p->jobs.data(), jobs_b, hipMemcpyHostToDevice));
        if (!p->items.empty())
            HIPCHK(hipMemcpy(p->items_dev, p->items.data(), sizeof(WorkItem) * p->items.size(), hipMemcpyHostToDevice));

        // 4) graph: captured on the plan's own stream, replayed on any stream
        if (p->use_graph) {
            HIPCHK(hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal));
            rc = enqueue(p.get(), p->capture_stream);
            hipGraph_t g = nullptr;
            hipError_t ec = hipStreamEndCapture(p->capture_stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (ec != hipSuccess) return fp_set_error(FP_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
            p->graph = g;
            HIPCHK(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
        }
        *out = p.release();
        return FP_OK;
    } catch (const std::bad_alloc&) {
        return fp_set_error(FP_ENOMEM, "out of host memory");
    }
}

extern "C" int fp_predict_batched(fp_plan* p, void* stream) {
    fp_clear_error();
    if (!p) return fp_set_error(FP_EINVAL, "plan is NULL");
    int dev = -1;
    int rc = fp::current_device(&dev);
    if (rc) return rc;
    if (dev != p->dev) return fp_set_error(FP_ENODEV, "plan built on device %d, current device is %d", p->dev, dev);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->exec) {
        HIPCHK(hipGraphLaunch(p->exec, s));
        return FP_OK;
    }
    return enqueue(p, s);
}

extern "C" int fp_plan_info_get(const fp_plan* p, fp_plan_info* out) {
    fp_clear_error();
    if (!p || !out) return fp_set_error(FP_EINVAL, "NULL argument");
    memset(out, 0, sizeof *out);
    out->n_jobs = (int32_t)p->jobs.size();
    out->n_items = (int32_t)p->items.size();
    out->blocks = p->blocks;
    out->block_threads = p->threads;
    out->cursors = p->K;
    out->graph = p->exec != nullptr;
    out->lds_bytes = (int32_t)p->lds_bytes;
    out->total_cost = p->total_cost;
    out->jobs_tuned = p->jobs_tuned;
    out->jobs_cached = p->jobs_cached;
    return FP_OK;
}

extern "C" void fp_plan_free(fp_plan* p) { delete p; }
