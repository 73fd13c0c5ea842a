// Autotuner: the design experiment of Sec. III-A (Fig. 2 sweeps stripe width
// and interleave depth) run on the GPU, with the paper's cost model (Eqs.
// 1-2 and the expected uses EU of a fetched line, Sec. III-A) as its prior.
//
//   1. every candidate packing -- layout (PACKED, COMPACT, BLOCKED,
//      CLUSTERED), bin size B and interleave depth D -- is packed on the
//      host and scored with Eq. 2's estimate from its header statistics;
//   2. per layout, only the top_k packings by score are timed (HIP events
//      on a sample of the caller's rows), with one launch shape per layout
//      kind;
//   3. the launch mapping of the fastest packing is searched as
//      fp_tune_launch does (tune.cpp).
// Votes never depend on the candidate; only time does.  Results are kept
// in the process-wide tune table and the FP_TUNE_CACHE file (tune.cpp).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "fp_internal.h"

namespace {

using fp::DevBuf;

uint64_t mix(uint64_t h, const void* p, size_t n) {
    const uint8_t* b = static_cast<const uint8_t*>(p);
    for (size_t i = 0; i < n; i++) h = (h ^ b[i]) * 0x100000001b3ull;
    return h;
}

uint64_t fingerprint(const fp_forest_view* v, int64_t sample, int threads, int K, int reps, int top_k) {
    uint64_t h = 0xcbf29ce484222325ull;
    int32_t dims[3] = {v->n_trees, v->n_features, v->n_classes};
    h = mix(h, dims, sizeof dims);
    const int64_t n = v->tree_node_offset[v->n_trees];
    h = mix(h, v->tree_node_offset, sizeof(int64_t) * (v->n_trees + 1));
    h = mix(h, v->feature, 4 * (size_t)n);
    h = mix(h, v->threshold, 4 * (size_t)n);
    h = mix(h, v->left, 4 * (size_t)n);
    h = mix(h, v->right, 4 * (size_t)n);
    h = mix(h, v->leaf_class, 4 * (size_t)n);
    if (v->cardinality) h = mix(h, v->cardinality, 8 * (size_t)n);
    int64_t cfg[6] = {sample, threads, K, reps, top_k, 2 /* autotuner revision */};
    return mix(h, cfg, sizeof cfg);
}

struct PackedPtr {
    fp_packed* p = nullptr;
    ~PackedPtr() { fp_packed_free(p); }
};

bool block_layout(int L) { return L == FP_LAYOUT_BLOCKED || L == FP_LAYOUT_CLUSTERED; }

// Eq. 2 with the EU of Sec. III-A, per row: T x (fetches - well-used) / EU.
// Node layouts fetch nodes; the interleaved depths 0..D are the well-used
// ones and EU = 1 + b(1 + b(1 + b)) for the forest's mean split bias b.  A
// block layout fetches blocks (EU 1: one fetch serves the block's nodes);
// its interleaved block levels 0..D/3 are the well-used ones.
double model_cost(const fp::Header& h, int L, int D) {
    const double f = h.expected_fetches, b = h.mean_bias;
    double wun, eu;
    if (block_layout(L)) {
        wun = std::min((double)(D / 3 + 1), f);
        eu = 1.0;
    } else {
        wun = std::min((double)(D + 1), h.expected_depth);
        eu = 1.0 + b * (1.0 + b * (1.0 + b));
    }
    return (double)h.n_trees * std::max(0.0, f - wun) / eu;
}

struct Cand {
    fp_pack_opts pack;
    double cost;
    double ms;
};

}  // namespace

extern "C" int fp_autotune(const fp_forest_view* forest, const float* X, int64_t n_rows, int64_t ld,
                           const fp_autotune_opts* opts, fp_autotune_result* out, void* stream_v) {
    fp_clear_error();
    if (!forest || !out) return fp_set_error(FP_EINVAL, "NULL argument");
    if (!X || n_rows < 1) return fp_set_error(FP_EINVAL, "autotuning needs at least one device row");
    if (ld < forest->n_features) return fp_set_error(FP_EINVAL, "ld %lld < n_features %d", (long long)ld, forest->n_features);
    if (!forest->tree_node_offset || forest->n_trees < 1) return fp_set_error(FP_EINVAL, "empty forest view");
    if (opts && (opts->max_trials < 0 || (opts->max_trials > 0 && !opts->trials)))
        return fp_set_error(FP_EINVAL, "trials is NULL with max_trials %d", opts->max_trials);
    memset(out, 0, sizeof *out);
    const int fixed_threads = opts ? opts->block_threads : 0;
    const int fixed_K = opts ? opts->cursors : 0;
    const int reps = opts && opts->reps > 0 ? opts->reps : 3;
    const int top_k = opts && opts->top_k > 0 ? opts->top_k : 2;
    const int64_t sample = std::min<int64_t>(n_rows, opts && opts->sample_rows > 0 ? opts->sample_rows : 65536);
    hipStream_t stream = static_cast<hipStream_t>(stream_v);

    const uint64_t key = fingerprint(forest, sample, fixed_threads, fixed_K, reps, top_k);
    if (fp::autotune_cache_get(key, out)) {
        out->cache_hit = 1;
        out->n_trials = 0;
        return FP_OK;
    }

    try {
        DevBuf votes, packed_buf;
        int rc = votes.ensure((size_t)sample * forest->n_classes * 4);
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

        std::unique_ptr<PackedPtr> current;
        // pack (and with upload, copy to the device buffer); FP_E2BIG when the
        // layout's encoding cannot hold this forest
        auto pack = [&](const fp_pack_opts& po, bool upload) -> int {
            current.reset(new PackedPtr());
            int r = fp_pack_forest(forest, &po, &current->p);
            if (r || !upload) return r;
            r = packed_buf.ensure(current->p->bytes.size());
            if (r) return r;
            return fp_packed_upload(current->p, packed_buf.p, packed_buf.cap, stream);
        };
        auto time_one = [&](const fp_tune& t, double* ms) -> int {
            int r = fp_predict_tuned(current->p, &t, X, sample, ld, static_cast<int32_t*>(votes.p), nullptr, stream);
            if (r) return r;
            if (hipEventRecord(e0, stream) != hipSuccess) return fp_set_error(FP_EHIP, "hipEventRecord failed");
            for (int i = 0; i < reps; i++) {
                r = fp_predict_tuned(current->p, &t, X, sample, ld, static_cast<int32_t*>(votes.p), nullptr, stream);
                if (r) return r;
            }
            if (hipEventRecord(e1, stream) != hipSuccess) return fp_set_error(FP_EHIP, "hipEventRecord failed");
            if (hipEventSynchronize(e1) != hipSuccess) return fp_set_error(FP_EHIP, "hipEventSynchronize failed");
            float f = 0.0f;
            if (hipEventElapsedTime(&f, e0, e1) != hipSuccess) return fp_set_error(FP_EHIP, "hipEventElapsedTime failed");
            *ms = f / reps;
            out->n_tried++;
            return FP_OK;
        };

        const int T = forest->n_trees;
        // reference: library defaults (one bin of all trees, interleave depth 4)
        rc = pack(fp_pack_opts{FP_LAYOUT_PACKED, T, 4, 0, FP_ORDER_DEFAULT}, true);
        if (rc) return rc;
        const int max_depth = current->p->hdr.max_depth;
        rc = time_one(fp_tune{}, &out->default_ms);
        if (rc) return rc;

        // 1. every candidate packing, scored by the model
        std::vector<Cand> cands;
        std::vector<int> bins{T};
        for (int B : {64, 16})
            if (B < T) bins.push_back(B);
        for (int L : {FP_LAYOUT_PACKED, FP_LAYOUT_COMPACT, FP_LAYOUT_BLOCKED, FP_LAYOUT_CLUSTERED})
            for (int B : bins)
                for (int D = 0; D <= std::min(7, max_depth); D++) {
                    if (block_layout(L) && D % 3) continue;  // whole three-level blocks are interleaved
                    const fp_pack_opts po{L, B, D, 0, FP_ORDER_DEFAULT};
                    rc = pack(po, false);
                    if (rc == FP_E2BIG) break;  // this layout's encoding does not fit the forest
                    if (rc) return rc;
                    cands.push_back(Cand{po, model_cost(current->p->hdr, L, D), -1.0});
                }
        out->n_candidates = (int32_t)cands.size();

        // 2. per layout, the top_k packings by model score, timed with one
        // launch shape per layout kind
        const int th = fixed_threads > 0 ? fixed_threads : 1024;
        double best = 1e30;
        size_t best_c = 0;
        for (int L : {FP_LAYOUT_PACKED, FP_LAYOUT_COMPACT, FP_LAYOUT_BLOCKED, FP_LAYOUT_CLUSTERED}) {
            std::vector<size_t> idx;
            for (size_t i = 0; i < cands.size(); i++)
                if (cands[i].pack.layout == L) idx.push_back(i);
            std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return cands[a].cost < cands[b].cost; });
            if ((int)idx.size() > top_k) idx.resize(top_k);
            for (size_t i : idx) {
                rc = pack(cands[i].pack, true);
                if (rc) return rc;
                fp_tune t{};
                t.rows_per_block = 32;
                t.block_threads = th;
                t.cursors = block_layout(L) ? 1 : (fixed_K > 0 ? fixed_K : 2);
                t.refill_lanes = block_layout(L) ? 32 : 16;
                double ms = 0.0;
                rc = time_one(t, &ms);
                if (rc == FP_E2BIG) continue;
                if (rc) return rc;
                cands[i].ms = ms;
                if (ms < best) {
                    best = ms;
                    best_c = i;
                }
            }
        }
        if (best >= 1e30) return fp_set_error(FP_E2BIG, "no candidate packing fits the workgroup's LDS");

        // 3. the launch mapping of the fastest packing
        rc = pack(cands[best_c].pack, true);
        if (rc) return rc;
        fp_tune tuned{};
        double tuned_ms = 0.0;
        int32_t tried = 0;
        rc = fp::search_launch(current->p, X, sample, ld, fixed_threads, fixed_K, stream, &tuned, &tuned_ms, &tried);
        if (rc) return rc;
        out->n_tried += tried;
        out->pack = cands[best_c].pack;
        out->tune = tuned;
        out->best_ms = std::min(best, tuned_ms);
        if (opts && opts->trials) {
            const int32_t n = std::min<int32_t>(opts->max_trials, (int32_t)cands.size());
            for (int32_t i = 0; i < n; i++)
                opts->trials[i] = fp_autotune_trial{cands[i].pack, cands[i].cost, cands[i].ms};
            out->n_trials = n;
        }
        if (hipStreamSynchronize(stream) != hipSuccess) return fp_set_error(FP_EHIP, "hipStreamSynchronize failed");
        fp_autotune_result rec = *out;
        rec.n_trials = 0;
        fp::autotune_cache_put(key, rec);
        return FP_OK;
    } catch (const std::bad_alloc&) {
        return fp_set_error(FP_ENOMEM, "out of host memory");
    }
}
