// Batched prediction that allocates nothing: for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving
// loops).  The job table, the work list and the work counter that
// fp_plan_create allocates for a plan live here in a file-scope device
// array of kScratchBytes, one copy per device, held until the process ends.
// The kernels are the batched path's (prologue, persistent kernel,
// epilogue); only where their tables live differs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "fp_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(1) << 20;  // job table + work items + counter
constexpr int kMaxDevices = 64;
constexpr int32_t kMaxJobs = 4096;

// The device array.  In host code its name is a host-side stand-in: the
// device address comes from hipGetSymbolAddress, once per device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;                      // one call at a time builds tables in g_host
void* g_scratch_dev[kMaxDevices];     // per device: scratch's device address
alignas(256) unsigned char g_host[kScratchBytes];  // host image of the tables
double g_depth[kMaxJobs];             // each job's expected depth (the work list's cost model)

int scratch_for(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return fp_set_error(FP_ENODEV, "device id %d out of range", dev);
    if (!g_scratch_dev[dev]) {  // first call on this device (it is current)
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fp_set_error(FP_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return FP_OK;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

extern "C" int fp_predict_batched_noalloc(const fp_job* jobs, int32_t n_jobs, const fp_plan_opts* opts,
                                          void* stream_v) {
    fp_clear_error();
    if (n_jobs < 1 || !jobs) return fp_set_error(FP_EINVAL, "need at least one job");
    if (n_jobs > kMaxJobs) return fp_set_error(FP_E2BIG, "%d jobs exceed the limit of %d", n_jobs, kMaxJobs);
    if (opts && opts->autotune) return fp_set_error(FP_EINVAL, "autotune times candidates and allocates: set it to 0");
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    int dev = -1;
    int rc = fp::current_device(&dev);
    if (rc) return rc;
    fp::DeviceProps dp;
    rc = fp::device_props(dev, &dp);
    if (rc) return rc;
    const int threads = opts && opts->block_threads > 0 ? opts->block_threads : 1024;
    const int K = opts && opts->cursors > 0 ? opts->cursors : 2;
    const int ipb = opts && opts->items_per_block > 0 ? opts->items_per_block : fp::kDefaultItemsPerBlock;
    if (threads % 64 || threads < 64 || threads > 1024)
        return fp_set_error(FP_EINVAL, "block_threads %d must be a multiple of 64 in [64, 1024]", threads);
    if (K != 1 && K != 2 && K != 4 && K != 8) return fp_set_error(FP_EINVAL, "cursors must be 1, 2, 4 or 8");
    const size_t blk_max = dp.lds_per_block ? dp.lds_per_block : 65536;
    const size_t lds_block = fp::batched_job_budget(
        opts && opts->lds_budget > 0 ? std::min((size_t)opts->lds_budget, blk_max) : fp::default_lds_block(dp));
    const size_t jobs_bytes = align256(sizeof(fp::JobDesc) * (size_t)n_jobs);
    if (jobs_bytes + 512 > kScratchBytes)
        return fp_set_error(FP_E2BIG, "%d jobs need %zu bytes of tables; the scratch holds %zu", n_jobs, jobs_bytes,
                            kScratchBytes);
    std::lock_guard<std::mutex> lk(g_mu);
    void* sp = nullptr;
    rc = scratch_for(dev, &sp);
    if (rc) return rc;
    // job descriptors, built in the static host image (no allocation): each
    // job's launch parameters are its forest's (or a recorded tune for the
    // plan's workgroup size and cursors)
    fp::JobDesc* jd = reinterpret_cast<fp::JobDesc*>(g_host);
    size_t lds = 0;
    for (int32_t i = 0; i < n_jobs; i++) {
        const fp_job& jb = jobs[i];
        if (!jb.forest) return fp_set_error(FP_EINVAL, "job %d: forest is NULL", i);
        const fp::Header& h = jb.forest->hdr;
        if (jb.n_rows < 0 || jb.n_rows > INT32_MAX) return fp_set_error(FP_EINVAL, "job %d: bad n_rows", i);
        if (jb.ld < h.n_features) return fp_set_error(FP_EINVAL, "job %d: ld < n_features", i);
        if (jb.n_rows > 0 && (!jb.X || !jb.votes)) return fp_set_error(FP_EINVAL, "job %d: X or votes is NULL", i);
        if (!jb.forest->dev || jb.forest->dev_id != dev)
            return fp_set_error(FP_ENODEV, "job %d: forest not uploaded on the current device", i);
        fp_tune t = jb.forest->tune;
        fp_tune rec;
        if (jb.n_rows > 0 && fp::launch_tune_get(jb.forest, jb.n_rows, threads, K, &rec)) t = rec;
        rc = fp::resolve_job(jb.forest, &t, jb.X, jb.n_rows, jb.ld, jb.votes, jb.cls, lds_block, &jd[i]);
        if (rc) return rc;
        fp::flatten_passes(&jd[i]);
        lds = std::max(lds, (size_t)jd[i].lds_bytes);
    }
    int occ = 1;
    const bool blocks_only = fp::jobs_blocks_only(jd, n_jobs);
    rc = fp::batched_occupancy(K, blocks_only, threads, lds, &occ);
    if (rc) return rc;
    const int64_t resident = (int64_t)dp.cus * occ;
    // the plan's work list, written straight after the job table
    for (int32_t i = 0; i < n_jobs; i++) g_depth[i] = jobs[i].forest->hdr.expected_depth;
    fp::WorkItem* items = reinterpret_cast<fp::WorkItem*>(g_host + jobs_bytes);
    const size_t max_items = (kScratchBytes - jobs_bytes - 256) / sizeof(fp::WorkItem);
    double cost = 0.0;
    const size_t n_items = fp::build_items_into(jd, g_depth, (size_t)n_jobs, resident, ipb, items, max_items, &cost);
    if (n_items > max_items)
        return fp_set_error(FP_E2BIG, "%zu work items exceed the scratch's %zu", n_items, max_items);
    uint8_t* base = static_cast<uint8_t*>(sp);
    const size_t table_bytes = jobs_bytes + n_items * sizeof(fp::WorkItem);
    int32_t* counter = reinterpret_cast<int32_t*>(base + kScratchBytes - 256);
    // g_host is pageable, so HIP performs this copy synchronously (its
    // documented behaviour for unpinned memory): g_host may be rebuilt as
    // soon as the call returns; the copy is ordered after earlier work on
    // `stream`
    const hipError_t e = hipMemcpyAsync(base, g_host, table_bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return fp_set_error(FP_EHIP, "hipMemcpyAsync (tables): %s", hipGetErrorString(e));
    const fp::JobDesc* jobs_dev = reinterpret_cast<const fp::JobDesc*>(base);
    const fp::WorkItem* items_dev = reinterpret_cast<const fp::WorkItem*>(base + jobs_bytes);
    // the prologue kernel clears the counter (and the votes of atomic jobs)
    rc = fp::launch_batched_prologue(jobs_dev, n_jobs, counter, stream);
    if (rc) return rc;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(resident, (int64_t)n_items));
    rc = fp::launch_batched(jobs_dev, items_dev, (int32_t)n_items, counter, K, blocks_only, threads, lds, blocks, stream);
    if (rc) return rc;
    return fp::launch_batched_epilogue(jobs_dev, n_jobs, stream);
}
