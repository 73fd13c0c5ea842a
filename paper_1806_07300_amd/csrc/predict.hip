// Traversal kernels for gfx950 and the fp_predict entry points.
//
// Two kernels compute the same votes:
//
//  naive_kernel   the baseline: one lane per observation, trees one after the
//                 other, every node (leaves included) fetched from memory in
//                 breadth-first order, features read from memory.  This is the
//                 GPU form of the BF layout the paper measures against.
//
//  packed_kernel  Forest Packing (Sec. III) on CDNA4:
//                 - a workgroup owns a tile of R observations; their features
//                   are staged once in LDS;
//                 - each bin's interleaved top levels (Sec. III-A, Bin) are
//                   staged in LDS and serve the most used nodes of every tree;
//                 - each lane owns one (observation, tree slot) pair and walks K
//                   trees of the bin round-robin (Bin+, Sec. III-B): the K next
//                   node loads are all issued before any compare, so K
//                   independent fetches per lane are in flight instead of one;
//                 - leaves are class references (DF-), so a walk ends without
//                   fetching a leaf; the deep region follows the Stat order;
//                 - votes are counted with LDS atomics per (observation, class),
//                   then stored (one tree group) or added to global memory with
//                   integer atomics (several tree groups; order-independent,
//                   so still exact).
//
// Split test everywhere: x <= threshold in fp32 (v_cmp_le_f32; NaN -> right).
// Built without fast-math and without denormal flushing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <mutex>

#include "fp_internal.h"

using fp::BinEntry;
using fp::Node16;

namespace {

constexpr int32_t kDone = INT32_MIN;

struct DeviceProps {
    int cus = 0;
    size_t lds_per_block = 0;
    bool ok = false;
};

DeviceProps g_props[64];
std::mutex g_props_mu;

int device_props(int dev, DeviceProps* out) {
    if (dev < 0 || dev >= 64) return fp_set_error(FP_ENODEV, "device id %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_props_mu);
    if (!g_props[dev].ok) {
        hipDeviceProp_t pr;
        hipError_t e = hipGetDeviceProperties(&pr, dev);
        if (e != hipSuccess) return fp_set_error(FP_EHIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
        g_props[dev].cus = pr.multiProcessorCount;
        g_props[dev].lds_per_block = pr.sharedMemPerBlock;
        g_props[dev].ok = true;
    }
    *out = g_props[dev];
    return FP_OK;
}

// ---------------------------------------------------------------------------
// naive kernel
// ---------------------------------------------------------------------------
struct NaiveArgs {
    const int64_t* tree_off;
    const Node16* nodes;
    const float* X;
    int64_t ld;
    int64_t n_rows;
    int32_t* votes;
    int32_t* cls;
    int32_t n_trees, C;
};

template <bool LDS_VOTES>
__global__ __launch_bounds__(1024) void naive_kernel(NaiveArgs a) {
    extern __shared__ int32_t vl[];  // [C][blockDim] when LDS_VOTES
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = row < a.n_rows;
    const int bd = blockDim.x, tid = threadIdx.x;
    int32_t* vg = a.votes + (live ? row : 0) * a.C;
    if (LDS_VOTES) {
        for (int c = 0; c < a.C; c++) vl[c * bd + tid] = 0;
    } else if (live) {
        for (int c = 0; c < a.C; c++) vg[c] = 0;
    }
    if (live) {
        const float* x = a.X + row * a.ld;
        for (int32_t t = 0; t < a.n_trees; t++) {
            const Node16* tn = a.nodes + a.tree_off[t];
            int32_t n = 0;
            while (true) {
                const Node16 nd = tn[n];
                if (nd.feat < 0) {
                    if (LDS_VOTES) vl[nd.left * bd + tid] += 1;
                    else vg[nd.left] += 1;
                    break;
                }
                n = (x[nd.feat] <= nd.thr) ? nd.left : nd.right;
            }
        }
        int32_t best = 0, bestv = INT_MIN;
        for (int c = 0; c < a.C; c++) {
            const int32_t v = LDS_VOTES ? vl[c * bd + tid] : vg[c];
            if (LDS_VOTES) vg[c] = v;
            if (v > bestv) { bestv = v; best = c; }
        }
        if (a.cls) a.cls[row] = best;
    }
}

// ---------------------------------------------------------------------------
// packed kernel
// ---------------------------------------------------------------------------
struct PackedArgs {
    const BinEntry* bins;
    const int32_t* roots;
    const Node16* nodes;
    const float* X;
    int64_t ld;
    int64_t n_rows;
    int32_t* votes;
    int32_t* cls;
    int32_t F, C, Fp;       // features, classes, LDS row stride (floats)
    int32_t n_bins;
    int32_t R, S;           // rows per block, tree slots per block (R * S == blockDim)
    int32_t G, bins_per_group;
    int32_t top_cap;        // bin-top nodes staged in LDS
    int32_t n_tiles;
    int32_t atomic_votes;   // 1: add into global votes (several groups)
};

__device__ __forceinline__ Node16 load_node(const Node16* p) {
    return *p;  // 16-byte aligned: one dwordx4 load
}

template <int K, bool FEAT_LDS>
__global__ __launch_bounds__(1024) void packed_kernel(PackedArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    Node16* top = reinterpret_cast<Node16*>(smem);
    float* xs = reinterpret_cast<float*>(smem + (size_t)a.top_cap * sizeof(Node16));
    int32_t* vl = reinterpret_cast<int32_t*>(xs + (FEAT_LDS ? a.R * a.Fp : 0));

    const int tid = threadIdx.x, bd = blockDim.x;
    const int r = tid % a.R, s = tid / a.R;
    const int group = blockIdx.x % a.G;
    const int blocks_per_group = gridDim.x / a.G;
    const int b_lo = group * a.bins_per_group;
    const int b_hi = min(b_lo + a.bins_per_group, a.n_bins);
    if (b_lo >= b_hi) return;  // uniform per block
    const bool single_bin = (b_hi - b_lo) == 1;

    auto stage_top = [&](int b) {
        const BinEntry be = a.bins[b];
        const int n = min(be.top_len, a.top_cap);
        const int4* src = reinterpret_cast<const int4*>(a.nodes + be.node_base);
        int4* dst = reinterpret_cast<int4*>(top);
        for (int i = tid; i < n; i += bd) dst[i] = src[i];
    };
    if (single_bin) stage_top(b_lo);

    for (int tile = blockIdx.x / a.G; tile < a.n_tiles; tile += blocks_per_group) {
        const int64_t row0 = (int64_t)tile * a.R;
        const int rows_here = (int)min<int64_t>(a.R, a.n_rows - row0);
        if (FEAT_LDS) {
            const int total = a.R * a.F;
            for (int i = tid; i < total; i += bd) {
                const int rr = i / a.F, ff = i - rr * a.F;
                xs[rr * a.Fp + ff] = rr < rows_here ? a.X[(row0 + rr) * a.ld + ff] : 0.0f;
            }
        }
        for (int i = tid; i < a.R * a.C; i += bd) vl[i] = 0;
        const bool live = r < rows_here;
        const float* xrow = a.X + (row0 + (live ? r : 0)) * a.ld;
        const float* xl = xs + r * a.Fp;
        int32_t* vrow = vl + r * a.C;

        for (int b = b_lo; b < b_hi; b++) {
            if (!single_bin) {
                __syncthreads();
                stage_top(b);
            }
            __syncthreads();
            if (!live) continue;
            const BinEntry be = a.bins[b];
            const Node16* gn = a.nodes + be.node_base;
            const int32_t* rt = a.roots + be.root_base;
            const int nt = be.n_trees;
            const int cap = min(be.top_len, a.top_cap);
            int32_t ref[K];
            int next = s + K * a.S;
#pragma unroll
            for (int k = 0; k < K; k++) {
                const int t = s + k * a.S;
                ref[k] = t < nt ? rt[t] : kDone;
            }
            while (true) {
                bool any = false;
#pragma unroll
                for (int k = 0; k < K; k++) {
                    // a class reference ends a walk: vote, then start the next tree
                    while (ref[k] < 0 && ref[k] != kDone) {
                        atomicAdd(&vrow[-ref[k] - 1], 1);
                        if (next < nt) {
                            ref[k] = rt[next];
                            next += a.S;
                        } else {
                            ref[k] = kDone;
                        }
                    }
                    any |= ref[k] != kDone;
                }
                if (!any) break;
                Node16 nd[K];
#pragma unroll
                for (int k = 0; k < K; k++) {
                    if (ref[k] >= 0) nd[k] = ref[k] < cap ? top[ref[k]] : load_node(gn + ref[k]);
                }
#pragma unroll
                for (int k = 0; k < K; k++) {
                    if (ref[k] >= 0) {
                        const float x = FEAT_LDS ? xl[nd[k].feat] : xrow[nd[k].feat];
                        ref[k] = (x <= nd[k].thr) ? nd[k].left : nd[k].right;
                    }
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < rows_here * a.C; i += bd) {
            const int rr = i / a.C, c = i - rr * a.C;
            int32_t* dst = a.votes + (row0 + rr) * a.C + c;
            if (a.atomic_votes) {
                if (vl[i]) atomicAdd(dst, vl[i]);
            } else {
                *dst = vl[i];
            }
        }
        if (!a.atomic_votes && a.cls) {
            for (int rr = tid; rr < rows_here; rr += bd) {
                int32_t best = 0, bestv = vl[rr * a.C];
                for (int c = 1; c < a.C; c++)
                    if (vl[rr * a.C + c] > bestv) { bestv = vl[rr * a.C + c]; best = c; }
                a.cls[row0 + rr] = best;
            }
        }
        __syncthreads();
    }
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void argmax_kernel(const int32_t* votes, int32_t* cls, int64_t n, int32_t C) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t* v = votes + i * C;
        int32_t best = 0, bestv = v[0];
        for (int c = 1; c < C; c++)
            if (v[c] > bestv) { bestv = v[c]; best = c; }
        cls[i] = best;
    }
}

int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fp_set_error(FP_EHIP, "%s launch: %s", what, hipGetErrorString(e));
    return FP_OK;
}

template <int K, bool FL>
void* packed_fn() {
    return reinterpret_cast<void*>(&packed_kernel<K, FL>);
}

void* pick_packed(int K, bool fl) {
    switch (K) {
        case 1: return fl ? packed_fn<1, true>() : packed_fn<1, false>();
        case 2: return fl ? packed_fn<2, true>() : packed_fn<2, false>();
        case 4: return fl ? packed_fn<4, true>() : packed_fn<4, false>();
        default: return fl ? packed_fn<8, true>() : packed_fn<8, false>();
    }
}

}  // namespace

namespace fp {

// Resolved launch configuration for the packed kernel.
struct PackedLaunch {
    int R, S, K, G, threads, top_cap, Fp, blocks;
    bool feat_lds;
    size_t lds_bytes;
};

int resolve_packed_launch(const fp_packed* p, const fp_tune* t, int64_t n_rows, const DeviceProps& dp,
                          PackedLaunch* L) {
    const Header& h = p->hdr;
    const size_t lds_max = dp.lds_per_block ? dp.lds_per_block : 65536;
    int threads = t->block_threads > 0 ? t->block_threads : 256;
    if (threads % 64 || threads < 64 || threads > 1024)
        return fp_set_error(FP_EINVAL, "block_threads %d must be a multiple of 64 in [64, 1024]", threads);
    int R = t->rows_per_block > 0 ? t->rows_per_block : 16;
    if (R > threads) R = threads;
    if (threads % R) return fp_set_error(FP_EINVAL, "rows_per_block %d must divide block_threads %d", R, threads);
    int K = t->cursors > 0 ? t->cursors : 2;
    if (K != 1 && K != 2 && K != 4 && K != 8) return fp_set_error(FP_EINVAL, "cursors must be 1, 2, 4 or 8");
    int G = t->tree_groups > 0 ? t->tree_groups : 1;
    if (G > h.n_bins) G = h.n_bins;
    const int Fp = h.n_features | 1;
    // feature_lds: 1 force LDS staging, -1 read features from memory, 0 automatic
    bool feat_lds = t->feature_lds >= 0;
    size_t votes_b = (size_t)R * h.n_classes * 4;
    size_t feat_b = feat_lds ? (size_t)R * Fp * 4 : 0;
    if (votes_b > lds_max) return fp_set_error(FP_E2BIG, "vote tile of %zu bytes exceeds LDS", votes_b);
    if (votes_b + feat_b > lds_max) {
        if (t->feature_lds == 1)
            return fp_set_error(FP_E2BIG, "observation tile of %zu bytes does not fit in LDS", feat_b);
        feat_lds = false;
        feat_b = 0;
    }
    int top_cap = t->lds_top_nodes > 0 ? t->lds_top_nodes : h.max_top_len;
    top_cap = std::min(top_cap, h.max_top_len);
    const size_t room = (lds_max - votes_b - feat_b) / sizeof(Node16);
    if ((size_t)top_cap > room) top_cap = (int)room;
    if (t->lds_top_nodes < 0) top_cap = 0;
    L->R = R;
    L->S = threads / R;
    L->K = K;
    L->G = G;
    L->threads = threads;
    L->top_cap = top_cap;
    L->Fp = Fp;
    L->feat_lds = feat_lds;
    L->lds_bytes = (size_t)top_cap * sizeof(Node16) + feat_b + votes_b;
    const int64_t n_tiles = (n_rows + R - 1) / R;
    // persistent blocks: enough to fill every CU a few times over
    int occ = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, pick_packed(K, feat_lds), threads, L->lds_bytes);
    if (e != hipSuccess || occ < 1) occ = 1;
    const int64_t per_group = std::min<int64_t>(n_tiles, (int64_t)dp.cus * occ * 2 / std::max(1, G) + 1);
    L->blocks = (int)std::max<int64_t>(1, per_group) * G;
    return FP_OK;
}

}  // namespace fp

static int predict_impl(const fp_packed* p, const fp_tune* tune, const float* X, int64_t n_rows, int64_t ld,
                        int32_t* votes, int32_t* cls, void* stream_v) {
    fp_clear_error();
    if (!p) return fp_set_error(FP_EINVAL, "packed forest is NULL");
    const fp::Header& h = p->hdr;
    if (n_rows < 0 || n_rows > INT32_MAX) return fp_set_error(FP_EINVAL, "n_rows %lld outside [0, 2^31)", (long long)n_rows);
    if (ld < h.n_features) return fp_set_error(FP_EINVAL, "ld %lld < n_features %d", (long long)ld, h.n_features);
    if (n_rows == 0) return FP_OK;
    if (!X || !votes) return fp_set_error(FP_EINVAL, "X or votes is NULL");
    if (!p->dev) return fp_set_error(FP_ENODEV, "packed forest is not uploaded");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fp_set_error(FP_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev != p->dev_id) return fp_set_error(FP_ENODEV, "forest uploaded to device %d, current device is %d", p->dev_id, dev);
    DeviceProps dp;
    int rc = device_props(dev, &dp);
    if (rc) return rc;
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    const uint8_t* base = static_cast<const uint8_t*>(p->dev);
    const Node16* nodes = reinterpret_cast<const Node16*>(base + h.nodes_offset);

    if (h.layout == FP_LAYOUT_NAIVE) {
        int threads = tune && tune->block_threads > 0 ? tune->block_threads : 256;
        if (threads % 64 || threads < 64 || threads > 1024)
            return fp_set_error(FP_EINVAL, "block_threads %d must be a multiple of 64 in [64, 1024]", threads);
        NaiveArgs a{reinterpret_cast<const int64_t*>(base + h.table_offset), nodes, X, ld, n_rows, votes, cls,
                    h.n_trees, h.n_classes};
        const size_t lds = (size_t)h.n_classes * threads * 4;
        const bool use_lds = lds <= 32768;
        const int blocks = (int)((n_rows + threads - 1) / threads);
        if (use_lds)
            hipLaunchKernelGGL(naive_kernel<true>, dim3(blocks), dim3(threads), lds, stream, a);
        else
            hipLaunchKernelGGL(naive_kernel<false>, dim3(blocks), dim3(threads), 0, stream, a);
        return check_launch("naive_kernel");
    }

    fp::PackedLaunch L;
    rc = fp::resolve_packed_launch(p, tune, n_rows, dp, &L);
    if (rc) return rc;
    PackedArgs a;
    a.bins = reinterpret_cast<const BinEntry*>(base + h.table_offset);
    a.roots = reinterpret_cast<const int32_t*>(base + h.roots_offset);
    a.nodes = nodes;
    a.X = X;
    a.ld = ld;
    a.n_rows = n_rows;
    a.votes = votes;
    a.cls = cls;
    a.F = h.n_features;
    a.C = h.n_classes;
    a.Fp = L.Fp;
    a.n_bins = h.n_bins;
    a.R = L.R;
    a.S = L.S;
    a.G = L.G;
    a.bins_per_group = (h.n_bins + L.G - 1) / L.G;
    a.top_cap = L.top_cap;
    a.n_tiles = (int32_t)((n_rows + L.R - 1) / L.R);
    a.atomic_votes = L.G > 1;
    if (a.atomic_votes) {
        const int64_t nv = n_rows * h.n_classes;
        hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)std::min<int64_t>((nv + 255) / 256, 4096)), dim3(256), 0,
                           stream, votes, nv, 0);
        rc = check_launch("fill_i32_kernel");
        if (rc) return rc;
    }
    void* fn = pick_packed(L.K, L.feat_lds);
    void* args[] = {&a};
    e = hipLaunchKernel(fn, dim3(L.blocks), dim3(L.threads), args, L.lds_bytes, stream);
    if (e != hipSuccess) return fp_set_error(FP_EHIP, "packed_kernel launch: %s", hipGetErrorString(e));
    if (a.atomic_votes && cls) {
        hipLaunchKernelGGL(argmax_kernel, dim3((unsigned)std::min<int64_t>((n_rows + 255) / 256, 4096)), dim3(256), 0,
                           stream, votes, cls, n_rows, h.n_classes);
        return check_launch("argmax_kernel");
    }
    return FP_OK;
}

extern "C" int fp_predict(const fp_packed* p, const float* X_dev, int64_t n_rows, int64_t ld, int32_t* votes_dev,
                          int32_t* class_dev, void* stream) {
    if (!p) return fp_set_error(FP_EINVAL, "packed forest is NULL");
    return predict_impl(p, &p->tune, X_dev, n_rows, ld, votes_dev, class_dev, stream);
}

extern "C" int fp_predict_tuned(const fp_packed* p, const fp_tune* tune, const float* X_dev, int64_t n_rows,
                                int64_t ld, int32_t* votes_dev, int32_t* class_dev, void* stream) {
    if (!p) return fp_set_error(FP_EINVAL, "packed forest is NULL");
    return predict_impl(p, tune ? tune : &p->tune, X_dev, n_rows, ld, votes_dev, class_dev, stream);
}
