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
    size_t lds_per_cu = 0;
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
        g_props[dev].lds_per_cu = pr.maxSharedMemoryPerMultiProcessor;
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
//
// Work unit = one (observation, tree) walk.  A workgroup owns a tile of R
// observations (compacted feature columns staged in LDS) and the trees of
// one tree group; the tile's R x trees units form a pool in LDS.  Every lane
// keeps K walks in flight (Bin+ round-robin, Sec. III-B): per step it issues
// the K node loads, then the K compares.  When walks end, the wavefront
// refills all its empty cursors at once: one lane reserves as many units as
// there are empty cursors with a single LDS atomic, and each empty cursor
// takes base + (number of empty cursors on lower lanes) -- a ballot/mbcnt
// prefix, no per-lane atomics.  Lanes therefore never idle behind a long
// walk while units remain, which is the GPU answer to the longest-path skew
// of Sec. IV-D.  The interleaved top levels of every bin of the group stay in
// LDS for the whole kernel (persistent workgroups).
// ---------------------------------------------------------------------------
struct PackedArgs {
    const BinEntry* bins;
    const int32_t* roots;
    const int32_t* fmap;
    const Node16* nodes;
    const float* X;
    int64_t ld;
    int64_t n_rows;
    int32_t* votes;
    int32_t* cls;
    int32_t Fc, Fcp, C;      // used features, LDS row stride (floats), classes
    int32_t n_bins, bin_size;
    int32_t R;               // observations per tile
    int32_t G, bins_per_group, trees_per_group;
    int32_t cap;             // LDS nodes reserved per bin of the group
    int32_t n_tiles;
    int32_t atomic_votes;    // 1: add into global votes (several groups)
};

struct PackedLds {
    size_t top, ttab, fmap, xs, votes, pool, total;
};

__host__ __device__ inline PackedLds packed_lds_layout(int cap, int bins_per_group, int trees_per_group, int Fc, int Fcp,
                                                       int R, int C, bool feat_lds) {
    PackedLds L;
    size_t o = 0;
    L.top = o;   o += (size_t)cap * bins_per_group * sizeof(Node16);
    L.ttab = o;  o += (size_t)trees_per_group * 16;
    L.fmap = o;  o += feat_lds ? 0 : ((size_t)Fc * 4 + 15) / 16 * 16;
    L.xs = o;    o += feat_lds ? ((size_t)R * Fcp * 4 + 15) / 16 * 16 : 0;
    L.votes = o; o += ((size_t)R * C * 4 + 15) / 16 * 16;
    L.pool = o;  o += 16;
    L.total = o;
    return L;
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }
__device__ __forceinline__ int bits_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <int K, bool FEAT_LDS>
__global__ __launch_bounds__(1024) void packed_kernel(PackedArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const PackedLds L = packed_lds_layout(a.cap, a.bins_per_group, a.trees_per_group, a.Fc, a.Fcp, a.R, a.C, FEAT_LDS);
    Node16* top = reinterpret_cast<Node16*>(smem + L.top);
    int4* ttab = reinterpret_cast<int4*>(smem + L.ttab);
    int32_t* fmap_l = reinterpret_cast<int32_t*>(smem + L.fmap);
    float* xs = reinterpret_cast<float*>(smem + L.xs);
    int32_t* vl = reinterpret_cast<int32_t*>(smem + L.votes);
    int32_t* pool = reinterpret_cast<int32_t*>(smem + L.pool);

    const int tid = threadIdx.x, bd = blockDim.x;
    const int group = blockIdx.x % a.G;
    const int blocks_per_group = gridDim.x / a.G;
    const int b_lo = group * a.bins_per_group;
    const int b_hi = min(b_lo + a.bins_per_group, a.n_bins);
    if (b_lo >= b_hi) return;  // uniform per block
    const int t_lo = a.bins[b_lo].first_tree;
    const int nt = a.bins[b_hi - 1].first_tree + a.bins[b_hi - 1].n_trees - t_lo;

    // once per workgroup: bin tops, tree table, feature map
    for (int i = tid; i < (b_hi - b_lo) * a.cap; i += bd) {
        const int bl = i / a.cap, k = i - bl * a.cap;
        const BinEntry& be = a.bins[b_lo + bl];
        if (k < be.top_len) top[i] = a.nodes[be.node_base + k];
    }
    for (int tl = tid; tl < nt; tl += bd) {
        const int t = t_lo + tl;
        const int b = t / a.bin_size;
        const BinEntry& be = a.bins[b];
        ttab[tl] = make_int4(a.roots[t], (int32_t)be.node_base, (b - b_lo) * a.cap, min(be.top_len, a.cap));
    }
    if (!FEAT_LDS)
        for (int j = tid; j < a.Fc; j += bd) fmap_l[j] = a.fmap[j];

    const int lane = lane_id();
    for (int tile = blockIdx.x / a.G; tile < a.n_tiles; tile += blocks_per_group) {
        const int64_t row0 = (int64_t)tile * a.R;
        const int rows_here = (int)min<int64_t>(a.R, a.n_rows - row0);
        if (FEAT_LDS) {
            const int total = rows_here * a.Fc;
            for (int i = tid; i < total; i += bd) {
                const int rr = i / a.Fc, j = i - rr * a.Fc;
                xs[rr * a.Fcp + j] = a.X[(row0 + rr) * a.ld + a.fmap[j]];
            }
        }
        for (int i = tid; i < rows_here * a.C; i += bd) vl[i] = 0;
        if (tid == 0) *pool = 0;
        __syncthreads();

        const int U = rows_here * nt;
        int32_t ref[K], rowk[K], gb[K], lb[K], cp[K];
#pragma unroll
        for (int k = 0; k < K; k++) { ref[k] = kDone; rowk[k] = 0; gb[k] = 0; lb[k] = 0; cp[k] = 0; }
        bool drained = false;  // wave-uniform: the pool has no units left
        while (true) {
            if (!drained) {
#pragma unroll
                for (int k = 0; k < K; k++) {
                    while (!drained) {
                        const uint64_t m = __ballot(ref[k] == kDone);
                        if (m == 0) break;
                        int base = 0;
                        if (lane == 0) base = atomicAdd(pool, (int)__popcll(m));
                        base = __builtin_amdgcn_readfirstlane(base);
                        if (base >= U) { drained = true; break; }
                        if (ref[k] == kDone) {
                            const int u = base + bits_below(m);
                            if (u < U) {
                                const int r = u % rows_here;
                                const int4 e = ttab[u / rows_here];
                                rowk[k] = r; gb[k] = e.y; lb[k] = e.z; cp[k] = e.w;
                                if (e.x < 0) atomicAdd(&vl[r * a.C - e.x - 1], 1);  // the root is a leaf
                                else ref[k] = e.x;
                            }
                        }
                        if (base + (int)__popcll(m) >= U) drained = true;
                    }
                }
            }
            bool live = false;
#pragma unroll
            for (int k = 0; k < K; k++) live |= ref[k] >= 0;
            if (__ballot(live) == 0) break;
            Node16 nd[K];
#pragma unroll
            for (int k = 0; k < K; k++)
                if (ref[k] >= 0) nd[k] = ref[k] < cp[k] ? top[lb[k] + ref[k]] : a.nodes[gb[k] + ref[k]];
#pragma unroll
            for (int k = 0; k < K; k++) {
                if (ref[k] >= 0) {
                    const float x = FEAT_LDS ? xs[rowk[k] * a.Fcp + nd[k].feat]
                                             : a.X[(row0 + rowk[k]) * a.ld + fmap_l[nd[k].feat]];
                    int32_t nr = (x <= nd[k].thr) ? nd[k].left : nd[k].right;
                    if (nr < 0) {
                        atomicAdd(&vl[rowk[k] * a.C - nr - 1], 1);
                        nr = kDone;
                    }
                    ref[k] = nr;
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < rows_here * a.C; i += bd) {
            int32_t* dst = a.votes + row0 * a.C + i;
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
    int R, K, G, threads, cap, Fcp, blocks, bins_per_group, trees_per_group;
    bool feat_lds;
    size_t lds_bytes;
};

int resolve_packed_launch(const fp_packed* p, const fp_tune* t, int64_t n_rows, const DeviceProps& dp,
                          PackedLaunch* L) {
    const Header& h = p->hdr;
    const size_t lds_max = dp.lds_per_block ? dp.lds_per_block : 65536;
    const size_t lds_cu = dp.lds_per_cu ? dp.lds_per_cu : lds_max;
    if (h.n_nodes >= INT32_MAX) return fp_set_error(FP_E2BIG, "packed forest has %lld nodes (limit 2^31-1)", (long long)h.n_nodes);
    const int threads = t->block_threads > 0 ? t->block_threads : 256;
    if (threads % 64 || threads < 64 || threads > 1024)
        return fp_set_error(FP_EINVAL, "block_threads %d must be a multiple of 64 in [64, 1024]", threads);
    const int R = t->rows_per_block > 0 ? t->rows_per_block : 16;
    if (R > 4096) return fp_set_error(FP_EINVAL, "rows_per_block %d exceeds 4096", R);
    const int K = t->cursors > 0 ? t->cursors : 2;
    if (K != 1 && K != 2 && K != 4 && K != 8) return fp_set_error(FP_EINVAL, "cursors must be 1, 2, 4 or 8");
    int G = t->tree_groups > 0 ? t->tree_groups : 1;
    if (G > h.n_bins) G = h.n_bins;
    const int bpg = (h.n_bins + G - 1) / G;
    const int Fc = h.n_used_features;
    const int Fcp = Fc | 1;
    // trees of the largest group
    const int tpg = std::min<int64_t>((int64_t)bpg * h.bin_size, h.n_trees);
    // feature_lds: 1 force LDS staging, -1 read features from memory, 0 automatic
    bool feat_lds = t->feature_lds >= 0;
    PackedLds base = packed_lds_layout(0, bpg, tpg, Fc, Fcp, R, h.n_classes, feat_lds);
    if (base.total > lds_max) {
        if (t->feature_lds == 1)
            return fp_set_error(FP_E2BIG, "observation tile of %d rows x %d columns does not fit in LDS", R, Fc);
        feat_lds = false;
        base = packed_lds_layout(0, bpg, tpg, Fc, Fcp, R, h.n_classes, false);
        if (base.total > lds_max)
            return fp_set_error(FP_E2BIG, "per-workgroup tables of %zu bytes exceed LDS", base.total);
    }
    // LDS for bin tops: an explicit node budget, or by default what keeps two
    // workgroups resident per CU
    size_t top_budget_nodes;
    if (t->lds_top_nodes < 0) {
        top_budget_nodes = 0;
    } else if (t->lds_top_nodes > 0) {
        top_budget_nodes = (size_t)t->lds_top_nodes;
    } else {
        const size_t per_block = std::min(lds_max, lds_cu / 2);
        top_budget_nodes = per_block > base.total ? (per_block - base.total) / sizeof(Node16) : 0;
    }
    const size_t room = (lds_max - base.total) / sizeof(Node16);
    top_budget_nodes = std::min(top_budget_nodes, room);
    int cap = (int)std::min<size_t>(top_budget_nodes / bpg, (size_t)h.max_top_len);
    L->R = R;
    L->K = K;
    L->G = G;
    L->threads = threads;
    L->cap = cap;
    L->Fcp = Fcp;
    L->feat_lds = feat_lds;
    L->bins_per_group = bpg;
    L->trees_per_group = tpg;
    L->lds_bytes = packed_lds_layout(cap, bpg, tpg, Fc, Fcp, R, h.n_classes, feat_lds).total;
    const int64_t n_tiles = (n_rows + R - 1) / R;
    int occ = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, pick_packed(K, feat_lds), threads, L->lds_bytes);
    if (e != hipSuccess || occ < 1) occ = 1;
    const int64_t per_group = std::min<int64_t>(n_tiles, std::max<int64_t>(1, (int64_t)dp.cus * occ / G));
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
    a.fmap = reinterpret_cast<const int32_t*>(base + h.fmap_offset);
    a.nodes = nodes;
    a.X = X;
    a.ld = ld;
    a.n_rows = n_rows;
    a.votes = votes;
    a.cls = cls;
    a.Fc = h.n_used_features;
    a.Fcp = L.Fcp;
    a.C = h.n_classes;
    a.n_bins = h.n_bins;
    a.bin_size = h.bin_size;
    a.R = L.R;
    a.G = L.G;
    a.bins_per_group = L.bins_per_group;
    a.trees_per_group = L.trees_per_group;
    a.cap = L.cap;
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
