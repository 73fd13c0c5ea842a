// Launch tuning per (packed forest, batch-size bucket) and the tune cache.
//
// Sec. III-A settles the stripe width and interleave depth with a design
// experiment on the target machine (Fig. 2); on the GPU the launch mapping
// (rows per workgroup, workgroup size, cursors per lane, refill threshold,
// tree groups, LDS per workgroup, tree passes) matters as much and depends
// on the batch size as well.
// fp_tune_launch times candidate mappings of one packed forest on the
// caller's rows and records the fastest for the batch's size bucket
// (ceil(log2(n_rows))).  Records live in a process-wide table keyed by the
// forest's bytes (checksum and size), so equal forests packed again, or
// loaded from a file, share them; with FP_TUNE_CACHE set they are also
// appended to that text file and read back by later processes.  fp_predict
// and fp_plan_create look the table up.
//
// File lines (whitespace separated, later lines win):
//   L <forest key hex> <bucket> <threads> <cursors> <9 fp_tune fields>
//   A <forest view fingerprint hex> <5 fp_pack_opts fields> <9 fp_tune fields> <best_ms> <default_ms> <n_tried>
#include <hip/hip_runtime_api.h>

#include <fcntl.h>
#include <unistd.h>

#include <algorithm>
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fp_internal.h"

namespace {

using LaunchKey = std::tuple<uint64_t, int32_t, int32_t, int32_t>;  // forest, bucket, threads, cursors

std::mutex g_mu;
bool g_loaded = false;
std::map<LaunchKey, fp_tune> g_launch;
std::map<uint64_t, fp_autotune_result> g_auto;

const char* cache_path() {
    const char* p = getenv("FP_TUNE_CACHE");
    return p && *p ? p : nullptr;
}

bool parse_tune(const char*& s, fp_tune* t) {
    int32_t v[9];
    int used = 0;
    if (sscanf(s, "%d %d %d %d %d %d %d %d %d%n", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6], &v[7], &v[8],
               &used) != 9)
        return false;
    s += used;
    *t = fp_tune{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], 0};
    return true;
}

void print_tune(char* buf, size_t n, const fp_tune& t) {
    snprintf(buf, n, "%d %d %d %d %d %d %d %d %d", t.rows_per_block, t.cursors, t.tree_groups, t.block_threads,
             t.lds_top_nodes, t.feature_lds, t.refill_lanes, t.lds_bytes, t.tree_passes);
}

// Reads the cache file once (under g_mu); malformed lines are skipped.
void load_locked() {
    if (g_loaded) return;
    g_loaded = true;
    const char* path = cache_path();
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        const char* s = line;
        unsigned long long key = 0;
        int used = 0;
        if (line[0] == 'L') {
            int32_t b, th, k;
            if (sscanf(s + 1, "%llx %d %d %d%n", &key, &b, &th, &k, &used) != 4) continue;
            s += 1 + used;
            fp_tune t;
            if (!parse_tune(s, &t)) continue;
            g_launch[LaunchKey{key, b, th, k}] = t;
        } else if (line[0] == 'A') {
            fp_autotune_result r;
            memset(&r, 0, sizeof r);
            if (sscanf(s + 1, "%llx %d %d %d %d %d%n", &key, &r.pack.layout, &r.pack.bin_size, &r.pack.interleave_depth,
                       &r.pack.line_align, &r.pack.node_order, &used) != 6)
                continue;
            s += 1 + used;
            if (!parse_tune(s, &r.tune)) continue;
            if (sscanf(s, "%lf %lf %d", &r.best_ms, &r.default_ms, &r.n_tried) != 3) continue;
            g_auto[key] = r;
        }
    }
    fclose(f);
}

// Appends one line with a single write(2) on an O_APPEND descriptor, so
// lines of processes sharing the file do not interleave.  A failure to write
// only costs the cache.
void append_line(const char* line) {
    const char* path = cache_path();
    if (!path) return;
    const int fd = open(path, O_WRONLY | O_CREAT | O_APPEND, 0644);
    if (fd < 0) return;
    const size_t n = strlen(line);
    if (write(fd, line, n) != (ssize_t)n) { /* the cache is best effort */ }
    close(fd);
}

}  // namespace

namespace fp {

// Forest bytes per tree pass that the launch search starts from.
constexpr int64_t kPassBytes = int64_t(176) << 20;

int32_t rows_bucket(int64_t n_rows) {
    int32_t b = 0;
    while (b < 62 && (int64_t(1) << b) < n_rows) b++;
    return b;
}

uint64_t forest_key(const fp_packed* p) {
    uint64_t h = p->hdr.checksum ^ 0x9E3779B97F4A7C15ull;
    const uint64_t extra[2] = {(uint64_t)p->hdr.total_bytes, (uint64_t)(uint32_t)p->hdr.layout};
    for (uint64_t v : extra) h = (h ^ v) * 0x100000001b3ull;
    return h;
}

bool launch_tune_get(const fp_packed* p, int64_t n_rows, int32_t threads, int32_t cursors, fp_tune* out) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_launch.find(LaunchKey{forest_key(p), rows_bucket(n_rows), threads, cursors});
    if (it == g_launch.end()) return false;
    *out = it->second;
    return true;
}

void launch_tune_put(const fp_packed* p, int64_t n_rows, int32_t threads, int32_t cursors, const fp_tune& t) {
    const uint64_t key = forest_key(p);
    const int32_t b = rows_bucket(n_rows);
    char tb[160], line[256];
    print_tune(tb, sizeof tb, t);
    snprintf(line, sizeof line, "L %016" PRIx64 " %d %d %d %s\n", key, b, threads, cursors, tb);
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_launch[LaunchKey{key, b, threads, cursors}] = t;
    append_line(line);
}

bool autotune_cache_get(uint64_t key, fp_autotune_result* out) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_auto.find(key);
    if (it == g_auto.end()) return false;
    *out = it->second;
    return true;
}

void autotune_cache_put(uint64_t key, const fp_autotune_result& r) {
    char tb[160], line[384];
    print_tune(tb, sizeof tb, r.tune);
    snprintf(line, sizeof line, "A %016" PRIx64 " %d %d %d %d %d %s %.6f %.6f %d\n", key, r.pack.layout,
             r.pack.bin_size, r.pack.interleave_depth, r.pack.line_align, r.pack.node_order, tb, r.best_ms,
             r.default_ms, r.n_tried);
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_auto[key] = r;
    append_line(line);
}

// Times candidate launch mappings of p on the first rows of X (at most
// 2^18) and returns the fastest.  threads / cursors > 0 are kept fixed.
int search_launch(const fp_packed* p, const float* X, int64_t n_rows, int64_t ld, int32_t threads, int32_t cursors,
                  hipStream_t stream, fp_tune* best_out, double* best_ms_out, int32_t* tried_out) {
    // a forest larger than the last-level cache is timed on more rows: the
    // launch shapes that suit it (tree passes, a CU's whole LDS) amortise
    // per-pass costs over many tiles
    const bool big = p->hdr.total_bytes > kPassBytes;
    const int64_t n = std::min<int64_t>(n_rows, int64_t(1) << (big ? 20 : 18));
    const int C = p->hdr.n_classes;
    DevBuf votes;
    int rc = votes.ensure((size_t)std::max<int64_t>(n, 1) * C * sizeof(int32_t));
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fp_set_error(FP_EHIP, "hipEventCreate failed");
    }
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } evg{e0, e1};
    // more repetitions for small batches, whose launches take microseconds
    const int reps = n >= (1 << 16) ? 3 : n >= (1 << 10) ? 6 : 12;
    double best = 1e30;
    fp_tune best_t{};
    int32_t tried = 0;
    auto time_one = [&](const fp_tune& t) -> int {
        int r = fp_predict_tuned(p, &t, X, n, ld, static_cast<int32_t*>(votes.p), nullptr, stream);
        if (r == FP_E2BIG) return FP_OK;  // does not fit the workgroup's LDS: not a candidate
        if (r) return r;
        if (hipEventRecord(e0, stream) != hipSuccess) return fp_set_error(FP_EHIP, "hipEventRecord failed");
        for (int i = 0; i < reps; i++) {
            r = fp_predict_tuned(p, &t, X, n, ld, static_cast<int32_t*>(votes.p), nullptr, stream);
            if (r) return r;
        }
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return fp_set_error(FP_EHIP, "hipEventRecord / hipEventSynchronize failed");
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return fp_set_error(FP_EHIP, "hipEventElapsedTime failed");
        tried++;
        if (ms / reps < best) {
            best = ms / reps;
            best_t = t;
        }
        return FP_OK;
    };
    const bool blocks = p->hdr.layout >= FP_LAYOUT_BLOCKED;
    std::vector<int> th_set = threads > 0 ? std::vector<int>{threads} : std::vector<int>{512, 1024};
    if (!blocks && threads <= 0) th_set.insert(th_set.begin(), 256);
    std::vector<int> k_set = cursors > 0 ? std::vector<int>{cursors} : blocks ? std::vector<int>{1} : std::vector<int>{1, 2, 4};
    std::vector<int> r_set = blocks ? std::vector<int>{16, 32, 64, 96, 128, 256, 512} : std::vector<int>{16, 32, 64, 128};
    // a tile never needs more rows than the batch has
    r_set.erase(std::remove_if(r_set.begin() + 1, r_set.end(), [&](int r) { return r > 2 * n; }), r_set.end());
    // pass 1: workgroup size, cursors, rows per workgroup
    for (int th : th_set)
        for (int k : k_set)
            for (int r : r_set) {
                fp_tune t{};
                t.rows_per_block = r;
                t.cursors = k;
                t.block_threads = th;
                t.tree_groups = 1;
                t.refill_lanes = blocks ? 32 : 16;
                rc = time_one(t);
                if (rc) return rc;
            }
    if (best >= 1e30) return fp_set_error(FP_E2BIG, "no launch candidate fits this forest");
    // pass 2: refill threshold; pass 3: tree groups (several workgroups per tile)
    const fp_tune p1 = best_t;
    for (int rl : {8, 16, 32, 48}) {
        if (rl == p1.refill_lanes) continue;
        fp_tune t = p1;
        t.refill_lanes = rl;
        if ((rc = time_one(t))) return rc;
    }
    const fp_tune p2 = best_t;
    for (int g : {2, 4}) {
        if (g > p->hdr.n_bins) break;
        fp_tune t = p2;
        t.tree_groups = g;
        if ((rc = time_one(t))) return rc;
    }
    // pass 4 (single-forest searches, forests larger than the last-level
    // cache): tree passes, so that each pass's bins (about kPassBytes of
    // forest, a share of MI355X's 256 MB MALL) stay cached while every row
    // walks them; around that count, half and twice it
    if (threads <= 0 && big && p->hdr.n_bins >= 2) {
        const fp_tune p3 = best_t;
        const int64_t base = std::min<int64_t>(p->hdr.n_bins, (p->hdr.total_bytes + kPassBytes - 1) / kPassBytes);
        for (int64_t P : {base / 2, base, 2 * base}) {
            if (P < 2 || P > p->hdr.n_bins) continue;
            fp_tune t = p3;
            t.tree_passes = (int32_t)P;
            t.tree_groups = 1;
            if ((rc = time_one(t))) return rc;
        }
    }
    // pass 5 (single-forest searches, whose workgroup size is free): one
    // 1024-thread workgroup per CU holding all of the CU's LDS, so that its
    // bin tops are not duplicated across workgroups, at the tile found so
    // far and at one 1.5 and 3 times as large (what does not fit is skipped).
    // A plan's workgroups share one LDS budget, so plans (threads fixed)
    // skip it.
    int dev = 0;
    DeviceProps dp;
    if (threads <= 0 && current_device(&dev) == FP_OK && device_props(dev, &dp) == FP_OK &&
        dp.lds_per_block > (size_t)default_lds_block(dp)) {
        const fp_tune p4 = best_t;
        for (int grow : {2, 3, 6}) {
            fp_tune t = p4;
            t.block_threads = 1024;
            t.lds_bytes = (int32_t)dp.lds_per_block;
            t.rows_per_block = std::min(4096, t.rows_per_block * grow / 2);
            if (t.rows_per_block > 2 * n) break;
            if ((rc = time_one(t))) return rc;
        }
        const fp_tune p5 = best_t;
        if (p5.lds_bytes > 0)
            for (int rl : {16, 24}) {
                if (rl == p5.refill_lanes) continue;
                fp_tune t = p5;
                t.refill_lanes = rl;
                if ((rc = time_one(t))) return rc;
            }
    }
    *best_out = best_t;
    *best_ms_out = best;
    *tried_out = tried;
    return FP_OK;
}

}  // namespace fp

extern "C" int fp_tune_launch(fp_packed* p, const float* X_dev, int64_t n_rows, int64_t ld, int32_t block_threads,
                              int32_t cursors, fp_tune* out, void* stream) {
    fp_clear_error();
    if (!p) return fp_set_error(FP_EINVAL, "packed forest is NULL");
    if (n_rows < 1 || n_rows > INT32_MAX || !X_dev) return fp_set_error(FP_EINVAL, "tuning needs 1 .. 2^31-1 device rows");
    if (ld < p->hdr.n_features) return fp_set_error(FP_EINVAL, "ld %lld < n_features %d", (long long)ld, p->hdr.n_features);
    if (p->hdr.layout == FP_LAYOUT_NAIVE) return fp_set_error(FP_EINVAL, "the naive layout has no launch to tune");
    if (block_threads < 0 || block_threads > 1024 || block_threads % 64)
        return fp_set_error(FP_EINVAL, "block_threads %d must be 0 or a multiple of 64 up to 1024", block_threads);
    if (cursors != 0 && cursors != 1 && cursors != 2 && cursors != 4 && cursors != 8)
        return fp_set_error(FP_EINVAL, "cursors must be 0, 1, 2, 4 or 8");
    fp_tune best{};
    double ms = 0.0;
    int32_t tried = 0;
    try {
        int rc = fp::search_launch(p, X_dev, n_rows, ld, block_threads, cursors, static_cast<hipStream_t>(stream), &best,
                                   &ms, &tried);
        if (rc) return rc;
    } catch (const std::bad_alloc&) {
        return fp_set_error(FP_ENOMEM, "out of host memory");
    }
    fp::launch_tune_put(p, n_rows, block_threads, cursors, best);
    if (out) *out = best;
    return FP_OK;
}
