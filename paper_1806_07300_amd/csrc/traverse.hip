// Traversal kernels for gfx950 and the fp_predict entry points.
//
//  naive_kernel    the baseline: one lane per observation, trees one after the
//                  other, every node (leaves included) fetched from memory in
//                  breadth-first order, features read from memory.  This is the
//                  GPU form of the BF layout the paper measures against.
//
//  packed_kernel   Forest Packing (Sec. III) on CDNA4, one forest:
//  batched_kernel  the same walk for many forests in one persistent launch.
//
// Packed walk.  A work unit is one (observation, tree) walk.  A workgroup owns
// a tile of R observations -- the feature columns some split tests are staged
// in LDS -- and the trees of one tree group, whose bins keep their interleaved
// top levels (Sec. III-A, Bin) in LDS.  The tile's R x trees units form a pool.
// Every lane keeps K walks in flight (Bin+, Sec. III-B): per step it issues
// its K node loads, then its K compares, so K independent fetches per lane
// overlap, as the paper's prefetch plus out-of-order execution does on a CPU.
// When walks end the wavefront refills all its empty cursors at once: lane 0
// reserves as many units as there are empty cursors with one LDS atomic, and
// every empty cursor takes base + (empty cursors on lower lanes), a
// ballot/mbcnt prefix.  No lane idles behind a long walk while units remain
// (the longest-path skew noted in Sec. IV-D).  Leaves are class references
// (DF-), so a walk ends without fetching a leaf; nodes below the interleaved
// levels follow the Stat order.  Votes are LDS atomics per (observation,
// class), then stored, or added into global memory with integer atomics when
// several tree groups share the rows (order-independent: still exact).
//
// Split test everywhere: x <= threshold in fp32 (v_cmp_le_f32; NaN -> right).
// The CLUSTERED 48-byte form, whose thresholds are all exact in fp16, stages
// the tile as fp16 values rounded toward +infinity and compares in fp16
// (v_cmp_le_f16), which decides every test exactly as the fp32 compare: for
// t exact in fp16, x <= t exactly when the smallest fp16 value >= x is <= t.
// Built without fast-math and without denormal flushing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "fp_internal.h"

using fp::BinEntry;
using fp::JobDesc;
using fp::Node16;
using fp::WorkItem;

namespace {

constexpr int32_t kDone = INT32_MIN;
constexpr int kDefaultRefillLanes = 16;
constexpr int kStageBatch = 4;  // row loads a thread issues before scattering them (tile staging)

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

// Leaf statistics from observations (Sec. III-A: the access statistics Stat
// orders by may be inferred after training from a set of observations): one
// lane per observation walks every tree of a NAIVE-layout forest and adds one
// to the counter of the leaf it reaches (position in the layout).  Grid-stride
// over rows; integer atomics, so the counts are exact and order-independent.
__global__ __launch_bounds__(256) void leaf_count_kernel(const Node16* __restrict__ nodes,
                                                         const int64_t* __restrict__ tree_off, int32_t n_trees,
                                                         const float* __restrict__ X, int64_t n_rows, int64_t ld,
                                                         int32_t* __restrict__ counts) {
    for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n_rows;
         row += (int64_t)gridDim.x * blockDim.x) {
        const float* x = X + row * ld;
        for (int32_t t = 0; t < n_trees; t++) {
            const Node16* tn = nodes + tree_off[t];
            int32_t n = 0;
            while (true) {  // a verified buffer's children come after their parent: the walk ends
                const Node16 nd = tn[n];
                if (nd.feat < 0) break;
                n = x[nd.feat] <= nd.thr ? nd.left : nd.right;
            }
            atomicAdd(&counts[tree_off[t] + n], 1);
        }
    }
}

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
// packed walk: device pieces shared by the single-forest and batched kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }
__device__ __forceinline__ int bits_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Unit u of a tile is (tree u / rows, row u % rows).  The division uses a
// 32-bit reciprocal m = floor((2^32 - 1) / rows): umulhi(u, m) is the
// quotient or one less for any u < 2^32, so one correction step is exact.
__device__ __forceinline__ uint32_t div_rows(uint32_t u, uint32_t rows, uint32_t m, uint32_t& rem) {
    uint32_t q = __umulhi(u, m);
    uint32_t r = u - q * rows;
    if (r >= rows) {
        q += 1;
        r -= rows;
    }
    rem = r;
    return q;
}

// Hands the idle cursors of a wavefront new units from the workgroup pool:
// per cursor slot one LDS atomic by lane 0 reserves as many units as there
// are idle lanes, and each idle lane takes base + (idle lanes below it).  A
// slot is refilled only once at least `min_idle` lanes have it idle, or when
// nothing in the wavefront is live, so most steps skip the refill's
// instructions.  take(k, row, ttab entry) sets cursor k up and returns its
// first reference, or kDone after voting when the tree's root is a leaf (the
// lane then stays idle and takes another unit).
template <int K, typename Take>
__device__ __forceinline__ void refill(int32_t (&ref)[K], int32_t* pool, int U, uint32_t rows, uint32_t rmagic,
                                       const int4* ttab, int min_idle, int lane, bool& drained, Take&& take) {
    uint64_t live = 0;
#pragma unroll
    for (int k = 0; k < K; k++) live |= __ballot(ref[k] >= 0);
#pragma unroll
    for (int k = 0; k < K; k++) {
        while (!drained) {
            const uint64_t m = __ballot(ref[k] < 0);
            const int cnt = (int)__popcll(m);
            if (cnt == 0 || (cnt < min_idle && live != 0)) break;
            int base = 0;
            if (lane == 0) base = atomicAdd(pool, cnt);
            base = __builtin_amdgcn_readfirstlane(base);
            if (base >= U) {
                drained = true;
                break;
            }
            if (ref[k] < 0) {
                const uint32_t u = (uint32_t)(base + bits_below(m));
                if (u < (uint32_t)U) {
                    uint32_t r;
                    const uint32_t t = div_rows(u, rows, rmagic, r);
                    ref[k] = take(k, (int)r, ttab[t]);
                }
            }
            if (base + cnt >= U) drained = true;
        }
    }
}

// fp16 bits (low half of each result) of the smallest fp16 values >= a, b,
// c, d (round toward +infinity; NaN stays NaN, beyond the fp16 range +inf
// or -65504): the wave's round mode for fp16 results (MODE bits 3:2) is set
// to +infinity for the four conversions and back to nearest-even, the
// kernel's mode, after them, inside one block so that no other instruction
// runs in between.
__device__ __forceinline__ void half_up4(float a, float b, float c, float d, uint32_t (&h)[4]) {
    asm volatile(
        "s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 1\n\t"
        "s_nop 1\n\t"
        "v_cvt_f16_f32 %0, %4\n\t"
        "v_cvt_f16_f32 %1, %5\n\t"
        "v_cvt_f16_f32 %2, %6\n\t"
        "v_cvt_f16_f32 %3, %7\n\t"
        "s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 0"
        : "=&v"(h[0]), "=&v"(h[1]), "=&v"(h[2]), "=&v"(h[3])
        : "v"(a), "v"(b), "v"(c), "v"(d));
}
// The same for one value without touching the round mode (the column-wise
// staging path): the nearest-even conversion, moved up one step when it fell
// below x.  Stepping the bits up a positive value, or down a negative one,
// gives the next larger value, and -0 steps to the smallest subnormal.
__device__ __forceinline__ uint16_t half_up(float x) {
    const _Float16 h = (_Float16)x;
    uint32_t b = __builtin_bit_cast(uint16_t, h);
    if ((float)h < x) b = (b & 0x8000u) ? (b == 0x8000u ? 1u : b - 1u) : b + 1u;
    return (uint16_t)b;
}

// Stores one staged feature: fp32, or fp16 bits already rounded up.
template <bool X16>
__device__ __forceinline__ void put_feature(void* row, int c, float v, uint32_t h) {
    if constexpr (X16) static_cast<uint16_t*>(row)[c] = (uint16_t)h;
    else static_cast<float*>(row)[c] = v;
}

// Copies the used feature columns of tile rows [row0, row0 + rows) into LDS
// (fp32 row-major, row stride Fcp; or, when X16, fp16 feature-major, feature
// stride Fcp, so that lanes reading one feature of consecutive rows share
// LDS words), clears
// the tile's vote counters and the unit pool, then synchronises.  Element
// i = r * Fc + c goes to thread i mod blockDim, which steps (r, c) and the
// row pointer incrementally.
template <bool X16 = false>
__device__ __forceinline__ void stage_tile(const JobDesc& j, float* xs, int32_t* vl, int32_t* pool, int64_t row0,
                                           int rows, bool feat_lds) {
    const int tid = threadIdx.x, bd = blockDim.x;
    if (feat_lds && j.stage_rows) {
        // whole rows in 16-byte loads; each used column goes to its compacted
        // slot (imap, 4 entries per 8-byte LDS read; -1 = unused)
        const int Q = (j.F + 3) / 4;
        const int16_t* imap = reinterpret_cast<const int16_t*>(reinterpret_cast<const unsigned char*>(xs) - j.off_xs +
                                                               j.off_imap);
        const int dq = bd / Q, dc = bd - dq * Q;
        int r = tid / Q, qd = tid - r * Q;
        const float4* xrow = reinterpret_cast<const float4*>(j.X + (row0 + r) * j.ld);
        const int64_t ld4 = j.ld / 4, dld4 = (int64_t)dq * ld4;
        // kStageBatch independent 16-byte loads in flight per thread, then
        // their scatter into the compacted columns
        while (r < rows) {
            float4 v[kStageBatch];
            int rr[kStageBatch], qq[kStageBatch];
#pragma unroll
            for (int u = 0; u < kStageBatch; u++) {
                rr[u] = r;
                qq[u] = qd;
                if (r < rows) v[u] = xrow[qd];
                r += dq;
                xrow += dld4;
                qd += dc;
                if (qd >= Q) {
                    qd -= Q;
                    r += 1;
                    xrow += ld4;
                }
            }
#pragma unroll
            for (int u = 0; u < kStageBatch; u++) {
                if (rr[u] >= rows) break;
                const int2 m2 = *reinterpret_cast<const int2*>(imap + 4 * qq[u]);
                const int m0 = (int16_t)(m2.x & 0xFFFF), m1 = m2.x >> 16, m2v = (int16_t)(m2.y & 0xFFFF),
                          m3 = m2.y >> 16;
                // fp32: row rr, element m; fp16: element m * Fcp of row rr
                void* dst = X16 ? static_cast<void*>(reinterpret_cast<uint16_t*>(xs) + rr[u])
                                : static_cast<void*>(xs + rr[u] * j.Fcp);
                const int es = X16 ? j.Fcp : 1;
                uint32_t h[4] = {0, 0, 0, 0};
                if constexpr (X16) half_up4(v[u].x, v[u].y, v[u].z, v[u].w, h);
                if (m0 >= 0) put_feature<X16>(dst, m0 * es, v[u].x, h[0]);
                if (m1 >= 0) put_feature<X16>(dst, m1 * es, v[u].y, h[1]);
                if (m2v >= 0) put_feature<X16>(dst, m2v * es, v[u].z, h[2]);
                if (m3 >= 0) put_feature<X16>(dst, m3 * es, v[u].w, h[3]);
            }
        }
    } else if (feat_lds) {
        const int Fc = j.Fc;
        const int dq = bd / Fc, dc = bd - dq * Fc;
        int r = tid / Fc, c = tid - r * Fc;
        const float* xrow = j.X + (row0 + r) * j.ld;
        const int64_t dld = (int64_t)dq * j.ld;
#pragma unroll 4
        while (r < rows) {
            if constexpr (X16) reinterpret_cast<uint16_t*>(xs)[c * j.Fcp + r] = half_up(xrow[j.fmap[c]]);
            else xs[r * j.Fcp + c] = xrow[j.fmap[c]];
            r += dq;
            xrow += dld;
            c += dc;
            if (c >= Fc) {
                c -= Fc;
                r += 1;
                xrow += j.ld;
            }
        }
    }
    for (int i = tid; i < rows * j.C; i += bd) vl[i] = 0;
    if (tid == 0) *pool = 0;
    __syncthreads();
}

// After the walks of a tile: stores its vote counters (or adds them into the
// global votes when several tree groups share the rows), then the class of
// each row (lowest class on ties) when this workgroup saw every tree.  In a
// later pass (accumulate) each thread owns whole rows: it adds the tile's
// counters to the stored votes and, in the last pass (cls set), takes the
// class from the sums; no other workgroup touches these rows in the launch.
__device__ __forceinline__ void write_tile(const JobDesc& j, const int32_t* vl, int64_t row0, int rows) {
    const int tid = threadIdx.x, bd = blockDim.x;
    __syncthreads();
    if (j.accumulate) {
        for (int rr = tid; rr < rows; rr += bd) {
            int32_t* dst = j.votes + (row0 + rr) * j.C;
            int32_t best = 0, bestv = INT_MIN;
            for (int c = 0; c < j.C; c++) {
                const int32_t v = dst[c] + vl[rr * j.C + c];
                dst[c] = v;
                if (v > bestv) {
                    bestv = v;
                    best = c;
                }
            }
            if (j.cls) j.cls[row0 + rr] = best;
        }
        __syncthreads();
        return;
    }
    for (int i = tid; i < rows * j.C; i += bd) {
        int32_t* dst = j.votes + row0 * j.C + i;
        if (j.atomic_votes) {
            if (vl[i]) atomicAdd(dst, vl[i]);
        } else {
            *dst = vl[i];
        }
    }
    if (!j.atomic_votes && j.cls) {
        for (int rr = tid; rr < rows; rr += bd) {
            int32_t best = 0, bestv = vl[rr * j.C];
            for (int c = 1; c < j.C; c++)
                if (vl[rr * j.C + c] > bestv) {
                    bestv = vl[rr * j.C + c];
                    best = c;
                }
            j.cls[row0 + rr] = best;
        }
    }
    __syncthreads();
}

// A tile's observations as the walks see them: feature f of tile row r
// (staged in LDS, or read from memory through the feature map) and the LDS
// vote counters of row r.  Row offsets use 24-bit multiplies (full rate;
// rows < 4096 and columns, classes < 2^24).
struct TileRows {
    const JobDesc& j;
    const float* xs;
    int32_t* vl;
    const int32_t* fmap_l;
    int64_t row0;
    bool feat_lds;
    __device__ __forceinline__ float x(int r, uint32_t f) const {
        return feat_lds ? xs[__umul24((uint32_t)r, (uint32_t)j.Fcp) + f] : j.X[(row0 + r) * j.ld + fmap_l[f]];
    }
    __device__ __forceinline__ void vote(int r, int32_t cls) const {
        atomicAdd(&vl[__umul24((uint32_t)r, (uint32_t)j.C) + (uint32_t)cls], 1);
    }
};

// Stage the bin tops, the tree table and (when features are read from memory)
// the feature map of tree group `group`; returns the group's tree count.
// The caller must have synchronised since the previous use of LDS.
__device__ int stage_group(const JobDesc& j, int group, unsigned char* smem) {
    const int tid = threadIdx.x, bd = blockDim.x;
    const int b_lo = group * j.bins_per_group;
    const int b_hi = min(b_lo + j.bins_per_group, j.n_bins);
    if (b_lo >= b_hi) return 0;
    Node16* top = reinterpret_cast<Node16*>(smem + j.off_top);
    int4* ttab = reinterpret_cast<int4*>(smem + j.off_ttab);
    const int t_lo = j.bins[b_lo].first_tree;
    const int nt = j.bins[b_hi - 1].first_tree + j.bins[b_hi - 1].n_trees - t_lo;
    // PACKED: the bin's top nodes; BLOCKED: its first blocks (roots first), as
    // 16-byte pieces; cap pieces per bin
    const int bw = j.block_bytes / 16;
    for (int i = tid; i < (b_hi - b_lo) * j.cap; i += bd) {
        const int bl = i / j.cap, k = i - bl * j.cap;
        const BinEntry& be = j.bins[b_lo + bl];
        const bool blk = j.layout >= FP_LAYOUT_BLOCKED;
        const int32_t have = blk ? be.deep_len * bw : be.top_len;
        if (k < have) top[i] = j.nodes[(blk ? be.node_base / 2 : be.node_base) + k];
    }
    for (int tl = tid; tl < nt; tl += bd) {
        const int t = t_lo + tl;
        const int b = t / j.bin_size;
        const BinEntry& be = j.bins[b];
        const int32_t nb = (int32_t)be.node_base;
        ttab[tl] = j.layout == FP_LAYOUT_COMPACT   ? make_int4(j.roots[t], nb, be.top_len, 0)
                   : j.layout >= FP_LAYOUT_BLOCKED ? make_int4(j.roots[t], nb, (b - b_lo) * j.cap,
                                                               min(be.deep_len, j.cap / max(bw, 1)))
                                                   : make_int4(j.roots[t], nb, (b - b_lo) * j.cap, min(be.top_len, j.cap));
    }
    if (!j.feat_lds) {
        int32_t* fmap_l = reinterpret_cast<int32_t*>(smem + j.off_fmap);
        for (int c = tid; c < j.Fc; c += bd) fmap_l[c] = j.fmap[c];
    }
    if (j.stage_rows) {
        int16_t* imap = reinterpret_cast<int16_t*>(smem + j.off_imap);
        const int n_imap = (j.F + 3) / 4 * 4;
        for (int c = tid; c < n_imap; c += bd) imap[c] = -1;
        __syncthreads();
        for (int i = tid; i < j.Fc; i += bd) imap[j.fmap[i]] = (int16_t)i;
        __syncthreads();  // the first tile's staging reads imap
    }
    return nt;
}

// FMODE: 0 features from memory, 1 features in LDS, 2 decided by j.feat_lds.
template <int K, int FMODE>
__device__ void run_tile(const JobDesc& j, int nt, int tile, unsigned char* smem) {
    const bool feat_lds = FMODE == 2 ? (j.feat_lds != 0) : (FMODE == 1);
    const Node16* top = reinterpret_cast<const Node16*>(smem + j.off_top);
    const int4* ttab = reinterpret_cast<const int4*>(smem + j.off_ttab);
    const int32_t* fmap_l = reinterpret_cast<const int32_t*>(smem + j.off_fmap);
    float* xs = reinterpret_cast<float*>(smem + j.off_xs);
    int32_t* vl = reinterpret_cast<int32_t*>(smem + j.off_votes);
    int32_t* pool = reinterpret_cast<int32_t*>(smem + j.off_pool);
    const int lane = lane_id();

    const int64_t row0 = (int64_t)tile * j.R;
    const int rows_here = (int)min<int64_t>(j.R, j.n_rows - row0);
    stage_tile(j, xs, vl, pool, row0, rows_here, feat_lds);

    const int U = rows_here * nt;
    const uint32_t rmagic = 0xFFFFFFFFu / (uint32_t)rows_here;
    TileRows tr{j, xs, vl, fmap_l, row0, feat_lds};
    // per cursor: row in the tile, gb = bin base in the node array, lb = the
    // bin's first top node in LDS, cp = top nodes staged in LDS
    int32_t ref[K], rowk[K], gb[K], lb[K], cp[K];
#pragma unroll
    for (int k = 0; k < K; k++) { ref[k] = kDone; rowk[k] = 0; gb[k] = 0; lb[k] = 0; cp[k] = 0; }
    auto take = [&](int k, int r, int4 e) -> int32_t {
        rowk[k] = r; gb[k] = e.y; lb[k] = e.z; cp[k] = e.w;
        if (e.x < 0) {  // the root is a leaf
            tr.vote(r, -e.x - 1);
            return kDone;
        }
        return e.x;
    };
    bool drained = false;
    while (true) {
        if (!drained) refill<K>(ref, pool, U, (uint32_t)rows_here, rmagic, ttab, j.refill_min, lane, drained, take);
        bool live = false;
#pragma unroll
        for (int k = 0; k < K; k++) live |= ref[k] >= 0;
        if (__ballot(live) == 0) {
            if (drained) break;
            continue;
        }
        Node16 nd[K];
#pragma unroll
        for (int k = 0; k < K; k++)
            if (ref[k] >= 0) nd[k] = ref[k] < cp[k] ? top[lb[k] + ref[k]] : j.nodes[gb[k] + ref[k]];
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (ref[k] >= 0) {
                int32_t nr = (tr.x(rowk[k], nd[k].feat) <= nd[k].thr) ? nd[k].left : nd[k].right;
                if (nr < 0) {
                    tr.vote(rowk[k], -nr - 1);
                    nr = kDone;
                }
                ref[k] = nr;
            }
        }
    }
    write_tile(j, vl, row0, rows_here);
}

// COMPACT layout walk.  Top nodes (Node16) come from memory (L1/L2); a deep
// node is fetched with one 16-byte load that also brings its successor, the
// Stat hot child.  When the walk moves to that successor the lane uses the
// copy it already holds and issues no load at all.  Each cursor keeps the
// LDS byte addresses of its row's features and votes, set once per walk.
typedef uint32_t u32x4_a8 __attribute__((ext_vector_type(4), aligned(8)));

template <int K, int FMODE>
__device__ void run_tile_compact(const JobDesc& j, int nt, int tile, unsigned char* smem) {
    const bool feat_lds = FMODE == 2 ? (j.feat_lds != 0) : (FMODE == 1);
    const int4* ttab = reinterpret_cast<const int4*>(smem + j.off_ttab);
    const int32_t* fmap_l = reinterpret_cast<const int32_t*>(smem + j.off_fmap);
    float* xs = reinterpret_cast<float*>(smem + j.off_xs);
    int32_t* vl = reinterpret_cast<int32_t*>(smem + j.off_votes);
    int32_t* pool = reinterpret_cast<int32_t*>(smem + j.off_pool);
    const uint2* words = reinterpret_cast<const uint2*>(j.nodes);
    const int lane = lane_id();
    const int fb = j.fbits, cb = j.cbits;
    const uint32_t fmask = (1u << fb) - 1u, cmask = (1u << cb) - 1u;

    const int64_t row0 = (int64_t)tile * j.R;
    const int rows_here = (int)min<int64_t>(j.R, j.n_rows - row0);
    stage_tile(j, xs, vl, pool, row0, rows_here, feat_lds);

    const int U = rows_here * nt;
    const uint32_t rmagic = 0xFFFFFFFFu / (uint32_t)rows_here;
    TileRows tr{j, xs, vl, fmap_l, row0, feat_lds};
    // per cursor: row in the tile, nb = bin base (words), topl = top_len,
    // the successor copy (sref, sthr, sw)
    int32_t ref[K], rowk[K], nb[K], topl[K], sref[K];
    float sthr[K];
    uint32_t sw[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        ref[k] = kDone; rowk[k] = 0; nb[k] = 0; topl[k] = 0; sref[k] = -1; sthr[k] = 0.0f; sw[k] = 0;
    }
    auto take = [&](int k, int r, int4 e) -> int32_t {
        rowk[k] = r; nb[k] = e.y; topl[k] = e.z; sref[k] = -1;
        if (e.x < 0) {  // the root is a leaf
            tr.vote(r, -e.x - 1);
            return kDone;
        }
        return e.x;
    };
    bool drained = false;
    while (true) {
        if (!drained) refill<K>(ref, pool, U, (uint32_t)rows_here, rmagic, ttab, j.refill_min, lane, drained, take);
        bool live = false;
#pragma unroll
        for (int k = 0; k < K; k++) live |= ref[k] >= 0;
        if (__ballot(live) == 0) {
            if (drained) break;
            continue;
        }
        // loads: a top node (16 B), or a deep node with its successor (16 B), or nothing
        float thr[K];
        uint32_t a0[K], a1[K], a2[K];
        bool deep[K];
#pragma unroll
        for (int k = 0; k < K; k++) {
            deep[k] = false;
            if (ref[k] < 0) continue;
            if (ref[k] < topl[k]) {
                const int4 v = *reinterpret_cast<const int4*>(words + nb[k] + 2 * ref[k]);
                thr[k] = __int_as_float(v.x); a0[k] = (uint32_t)v.y; a1[k] = (uint32_t)v.z; a2[k] = (uint32_t)v.w;
            } else if (ref[k] == sref[k]) {
                deep[k] = true;
                thr[k] = sthr[k]; a0[k] = sw[k];
            } else {
                deep[k] = true;
                const u32x4_a8 v = *reinterpret_cast<const u32x4_a8*>(words + nb[k] + topl[k] + ref[k]);
                thr[k] = __uint_as_float(v.x); a0[k] = v.y;
                sthr[k] = __uint_as_float(v.z); sw[k] = v.w; sref[k] = ref[k] + 1;
            }
        }
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (ref[k] < 0) continue;
            const uint32_t f = deep[k] ? (a0[k] & fmask) : a0[k];
            const bool go_left = tr.x(rowk[k], f) <= thr[k];
            int32_t nr;
            if (!deep[k]) {
                nr = go_left ? (int32_t)a1[k] : (int32_t)a2[k];
            } else {
                const uint32_t w = a0[k];
                const uint32_t pay = w >> (fb + 3);
                if ((w >> fb) & 1u) {
                    const bool adj_left = (w >> (fb + 1)) & 1u;
                    if (go_left == adj_left) nr = ref[k] + 1;
                    else if ((w >> (fb + 2)) & 1u) nr = -(int32_t)pay - 1;
                    else nr = ref[k] + (int32_t)pay;
                } else {
                    nr = -(int32_t)(go_left ? (pay & cmask) : (pay >> cb)) - 1;
                }
            }
            if (nr < 0) {
                tr.vote(rowk[k], -nr - 1);
                nr = kDone;
            }
            ref[k] = nr;
        }
    }
    write_tile(j, vl, row0, rows_here);
}

// A fetched block as the walk sees it: the word and threshold of each slot,
// the first child block, and how to read a child code.
struct BlockView {
    uint32_t w[7], t[7];
    uint32_t child_base, ranks;
};

// Fetches block `ref` of the bin starting at word bb: three (48-byte form) or
// four (64-byte form) 16-byte loads of one line, issued back to back; the
// bin's first `ns` blocks come from their LDS copy at piece lb instead.
// The two sources are typed with their address spaces so that the compiler
// keeps an LDS read and a global load rather than merging them into one flat
// load through a selected pointer.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const u32x4 lds_u32x4;
typedef __attribute__((address_space(1))) const u32x4 global_u32x4;

__device__ __forceinline__ uint4 as_uint4(u32x4 v) { return make_uint4(v.x, v.y, v.z, v.w); }

// LDS byte address of a pointer into the workgroup's shared memory, and back.
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
    return (uint32_t)(size_t)(__attribute__((address_space(3))) const void*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(3))) const T* lds_ptr(uint32_t a) {
    return (__attribute__((address_space(3))) const T*)(size_t)a;
}

// bp = the bin's first block in memory, la = LDS byte address of its copy
// (blocks below ns).
template <bool B48>
__device__ __forceinline__ void fetch_block(const global_u32x4* bp, uint32_t la, int32_t ns, int32_t ref,
                                            uint4 (&q)[4]) {
    constexpr int bw = B48 ? 3 : 4;  // 16-byte pieces per block
    if (ref < ns) {
        const lds_u32x4* lp = lds_ptr<u32x4>(la + (B48 ? __umul24((uint32_t)ref, 48u) : (uint32_t)ref << 6));
        q[0] = as_uint4(lp[0]);
        q[1] = as_uint4(lp[1]);
        q[2] = as_uint4(lp[2]);
        if (!B48) q[3] = as_uint4(lp[3]);
    } else {
        const global_u32x4* gp = bp + bw * ref;
        q[0] = as_uint4(gp[0]);
        q[1] = as_uint4(gp[1]);
        q[2] = as_uint4(gp[2]);
        if (!B48) q[3] = as_uint4(gp[3]);
    }
}

// Unpacks a fetched block (Block48: 19-bit words at fixed offsets of the first
// 136 bits; Block64: (thr, word) pairs after the header).
template <bool B48>
__device__ __forceinline__ BlockView view_block(const uint4 (&q)[4]) {
    BlockView b;
    if (B48) {
        const uint32_t r[5] = {q[0].x, q[0].y, q[0].z, q[0].w, q[1].x};
        constexpr uint32_t M = (1u << fp::kBlock48WordBits) - 1u;
#pragma unroll
        for (int sl = 0; sl < 7; sl++) {
            const int o = fp::kBlock48WordBits * sl;
            b.w[sl] = __builtin_amdgcn_alignbit(r[o / 32 + 1 < 5 ? o / 32 + 1 : 4], r[o / 32], o % 32) & M;
        }
        b.t[0] = q[1].y; b.t[1] = q[1].z; b.t[2] = q[1].w;
        b.t[3] = q[2].x; b.t[4] = q[2].y; b.t[5] = q[2].z; b.t[6] = q[2].w;
        b.child_base = r[4] >> 8;
        b.ranks = 0;
    } else {
        b.child_base = q[0].x; b.ranks = q[0].y;
        b.t[0] = q[0].z; b.w[0] = q[0].w;
        b.t[1] = q[1].x; b.w[1] = q[1].y; b.t[2] = q[1].z; b.w[2] = q[1].w;
        b.t[3] = q[2].x; b.w[3] = q[2].y; b.t[4] = q[2].z; b.w[4] = q[2].w;
        b.t[5] = q[3].x; b.w[5] = q[3].y; b.t[6] = q[3].z; b.w[6] = q[3].w;
    }
    return b;
}

// Field [pos, pos + width) of the 160 bits r[0..4] of a CLUSTERED block
// (positions are compile-time constants, so this is one or two ALU ops).
template <int pos, int width>
__device__ __forceinline__ uint32_t cfield(const uint32_t (&r)[5]) {
    constexpr uint32_t mask = (1u << width) - 1u;
    if constexpr (pos % 32 + width <= 32) return (r[pos / 32] >> (pos % 32)) & mask;
    else return __builtin_amdgcn_alignbit(r[pos / 32 + 1], r[pos / 32], pos % 32) & mask;
}

// Bytes of x that are zero get bit 7 set, the others clear (bytes < 0x80
// or with bit 7 set; no carry crosses a byte).
__device__ __forceinline__ uint32_t zero_bytes(uint32_t x) {
    return ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
}

// Bits [OFF, OFF + W) of x as one v_bfe_u32 the compiler cannot fold into the
// address arithmetic that follows (which would cost a shift and a mask).
template <int OFF, int W>
__device__ __forceinline__ uint32_t bfe_u32(uint32_t x) {
    uint32_t r;
    asm("v_bfe_u32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "i"(OFF), "i"(W));
    return r;
}

// Low / high fp16 half of a word widened to fp32 (exact).
__device__ __forceinline__ float half_lo(uint32_t v) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(v & 0xFFFFu));
}
__device__ __forceinline__ float half_hi(uint32_t v) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(v >> 16));
}
// The same halves as fp16 values.
__device__ __forceinline__ _Float16 bits_lo16(uint32_t v) {
    return __builtin_bit_cast(_Float16, (unsigned short)(v & 0xFFFFu));
}
__device__ __forceinline__ _Float16 bits_hi16(uint32_t v) {
    return __builtin_bit_cast(_Float16, (unsigned short)(v >> 16));
}

// CLUSTERED block: reads the seven split outcomes (one LDS round trip, as in
// the BLOCKED walk), tests four exits per 32-bit operation against the
// outcome mask replicated into every byte, and returns the next reference:
// the child block or the class of the one exit whose pattern matches.
// C48: the 48-byte form (fp16 thresholds and 9-bit features); otherwise the
// 64-byte form.  H16 (48-byte form only): `le` loads a feature of an fp16
// tile, compared with the fp16 thresholds; else `le` compares with the
// thresholds widened to fp32.
template <bool C48, bool H16, typename Le>
__device__ __forceinline__ int32_t cluster_step(const uint4 (&q)[4], int32_t xrow, Le&& le) {
    static_assert(C48 || !H16, "fp16 compares need fp16 thresholds");
    using Thr = std::conditional_t<H16, _Float16, float>;
    Thr thr[7];
    uint32_t care_lo, care_hi, val_lo, val_hi, r[5], f[7], child_base, n_child;
    if constexpr (H16) {
        thr[0] = bits_lo16(q[0].x); thr[1] = bits_hi16(q[0].x); thr[2] = bits_lo16(q[0].y);
        thr[3] = bits_hi16(q[0].y); thr[4] = bits_lo16(q[0].z); thr[5] = bits_hi16(q[0].z);
        thr[6] = bits_lo16(q[0].w);
    }
    if constexpr (C48) {
        if constexpr (!H16) {
            thr[0] = half_lo(q[0].x); thr[1] = half_hi(q[0].x); thr[2] = half_lo(q[0].y); thr[3] = half_hi(q[0].y);
            thr[4] = half_lo(q[0].z); thr[5] = half_hi(q[0].z); thr[6] = half_lo(q[0].w);
        }
        care_lo = q[1].x; care_hi = q[1].y; val_lo = q[1].z; val_hi = q[1].w;
        r[0] = q[2].x; r[1] = q[2].y; r[2] = q[2].z; r[3] = q[2].w;
        static_assert(fp::kC48FeatPos[0] == 48 && fp::kC48FeatPos[1] == 64 && fp::kC48FeatPos[2] == 73 &&
                          fp::kC48FeatPos[3] == 82 && fp::kC48FeatPos[4] == 96 && fp::kC48FeatPos[5] == 105 &&
                          fp::kC48FeatPos[6] == 114 && fp::kC48NChildPos == 57 && fp::kC48BasePos == 123,
                      "field positions below follow the 48-byte block");
        f[0] = bfe_u32<16, 9>(r[1]);
        f[1] = bfe_u32<0, 9>(r[2]); f[2] = bfe_u32<9, 9>(r[2]); f[3] = bfe_u32<18, 9>(r[2]);
        f[4] = bfe_u32<0, 9>(r[3]); f[5] = bfe_u32<9, 9>(r[3]); f[6] = bfe_u32<18, 9>(r[3]);
        n_child = (r[1] >> 25) & 15u;
        child_base = __builtin_amdgcn_alignbit(q[0].w >> 16, r[3], 27);  // rest bits [123, 144)
    } else {
        thr[0] = __uint_as_float(q[0].x); thr[1] = __uint_as_float(q[0].y); thr[2] = __uint_as_float(q[0].z);
        thr[3] = __uint_as_float(q[0].w); thr[4] = __uint_as_float(q[1].x); thr[5] = __uint_as_float(q[1].y);
        thr[6] = __uint_as_float(q[1].z);
        care_lo = q[1].w; care_hi = q[2].x; val_lo = q[2].y; val_hi = q[2].z;
        r[0] = q[2].w; r[1] = q[3].x; r[2] = q[3].y; r[3] = q[3].z; r[4] = q[3].w;
        constexpr int FW = fp::kClusterFeatBits;
        f[0] = cfield<48, FW>(r); f[1] = cfield<48 + FW, FW>(r); f[2] = cfield<48 + 2 * FW, FW>(r);
        f[3] = cfield<48 + 3 * FW, FW>(r); f[4] = cfield<48 + 4 * FW, FW>(r); f[5] = cfield<48 + 5 * FW, FW>(r);
        f[6] = cfield<48 + 6 * FW, FW>(r);
        n_child = cfield<156, 4>(r);
        child_base = cfield<132, 24>(r);
    }
    uint32_t g = 0;
    if constexpr (H16) {
        // all seven features loaded before any compare: one LDS round trip
        _Float16 x[7];
#pragma unroll
        for (int sl = 0; sl < 7; sl++) x[sl] = le(xrow, f[sl]);
#pragma unroll
        for (int sl = 0; sl < 7; sl++) g |= (x[sl] <= thr[sl] ? 0u : 1u) << sl;
    } else {
#pragma unroll
        for (int sl = 0; sl < 7; sl++) g |= (le(xrow, f[sl], thr[sl]) ? 0u : 1u) << sl;
    }
    const uint32_t g4 = __builtin_amdgcn_perm(g, g, 0u);  // byte 0 of g copied into every byte
    const uint32_t z_lo = zero_bytes((g4 ^ val_lo) & care_lo), z_hi = zero_bytes((g4 ^ val_hi) & care_hi);
    // a verified block's used exits partition the outcomes: exactly one byte
    // is zero (the top bit keeps e <= 7 for any bytes); both outcomes of the
    // exit are formed and selected, without a branch
    const uint64_t z = ((uint64_t)(z_hi | 0x80000000u) << 32) | z_lo;
    const uint32_t e = (uint32_t)__builtin_ctzll(z) >> 3;
    const uint64_t targets = ((uint64_t)r[1] << 32) | r[0];
    const uint32_t t = (uint32_t)(targets >> __umul24(e, 6u)) & 63u;
    const int32_t child = (int32_t)(child_base + min(t & 7u, n_child - 1u));
    const int32_t leaf = ~(int32_t)(t & 31u);
    const int32_t m = -(int32_t)(t >> 5);  // all ones when the exit leads to a child block
    return (child & m) | (leaf & ~m);
}

// BLOCKED layout walk.  Every reference is a block of the bin (or a class).
// A block is fetched whole and walked for up to three levels from registers:
// slot 0, then slot 1 or 2, then one of slots 3..6, ending in a class or an
// exit to a child block, which the next iteration fetches.  With the row's
// features in LDS all seven split tests are read in one LDS round trip and
// the path is resolved from a mask of sides by selects (no divergence inside
// a block).
// FMT: 0 BLOCKED 48-byte blocks, 1 BLOCKED 64-byte blocks, 2 CLUSTERED
// 64-byte blocks, 3 CLUSTERED 48-byte blocks, 4 CLUSTERED 48-byte blocks
// over an fp16 tile (features in LDS only).
template <int K, int FMODE, int FMT>
__device__ void run_tile_blocked(const JobDesc& j, int nt, int tile, unsigned char* smem) {
    constexpr bool B48 = FMT == 0 || FMT >= 3;
    constexpr bool X16 = FMT == 4;
    static_assert(!X16 || FMODE != 0, "an fp16 tile lives in LDS (x16 is set only with feat_lds)");
    const bool feat_lds = FMODE == 2 ? (j.feat_lds != 0) : (FMODE == 1);
    const int4* ttab = reinterpret_cast<const int4*>(smem + j.off_ttab);
    const int32_t* fmap_l = reinterpret_cast<const int32_t*>(smem + j.off_fmap);
    float* xs = reinterpret_cast<float*>(smem + j.off_xs);
    int32_t* vl = reinterpret_cast<int32_t*>(smem + j.off_votes);
    int32_t* pool = reinterpret_cast<int32_t*>(smem + j.off_pool);
    const uint2* words = reinterpret_cast<const uint2*>(j.nodes);
    const int lane = lane_id();
    const int fb = j.fbits;
    const int cw = 1 + (B48 ? max(j.cbits, 3) : j.cbits);  // bits of one child code
    const uint32_t fmask = (1u << fb) - 1u, code_mask = (1u << cw) - 1u;
    const uint32_t sh_l = (uint32_t)fb, sh_r = (uint32_t)(fb + cw);  // where the left / right codes start

    const int64_t row0 = (int64_t)tile * j.R;
    const int rows_here = (int)min<int64_t>(j.R, j.n_rows - row0);
    stage_tile<X16>(j, xs, vl, pool, row0, rows_here, feat_lds);

    const int U = rows_here * nt;
    const uint32_t rmagic = 0xFFFFFFFFu / (uint32_t)rows_here;
    // x <= thr for compacted feature f; xrow = LDS byte address of the row's
    // first feature in the tile (or its row in the tile when features stay
    // in memory)
    auto le = [&](int32_t xrow, uint32_t f, float thr) {
        const float x = feat_lds ? lds_ptr<float>((uint32_t)xrow)[f] : j.X[(row0 + xrow) * j.ld + fmap_l[f]];
        return x <= thr;
    };
    // the same over an fp16 tile (feature-major, feature stride Fcp): exact
    // for thresholds exact in fp16, since the tile holds each x rounded
    // toward +infinity
    const uint32_t fstride = 2u * (uint32_t)j.Fcp;
    auto le16 = [&](int32_t xrow, uint32_t f) -> _Float16 {
        return *lds_ptr<_Float16>((uint32_t)xrow + __umul24(f, fstride));
    };
    const uint32_t xs_addr = lds_addr(xs), blocks_addr = lds_addr(smem + j.off_top);
    // the block an exit leaves to: rank from the code (48-byte form) or the table
    auto exit_to = [&](const BlockView& b, uint32_t e, uint32_t code) -> int32_t {
        const uint32_t rank = B48 ? (code >> 1) : ((b.ranks >> (4 * e)) & 7u);
        return (int32_t)(b.child_base + rank);
    };
    // per cursor: xrow, vrow = the row's first vote counter, bp = the bin's
    // first block, la / ns = its LDS copy (byte address, blocks held)
    int32_t ref[K], xrow[K], vrow[K], ns[K];
    uint32_t la[K];
    const global_u32x4* bp[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        ref[k] = kDone; xrow[k] = 0; vrow[k] = 0; ns[k] = 0; la[k] = 0; bp[k] = nullptr;
    }
    auto take = [&](int k, int r, int4 e) -> int32_t {
        xrow[k] = !feat_lds ? r
                  : X16     ? (int32_t)(xs_addr + 2u * (uint32_t)r)
                            : (int32_t)(xs_addr + 4u * __umul24((uint32_t)r, (uint32_t)j.Fcp));
        vrow[k] = (int32_t)__umul24((uint32_t)r, (uint32_t)j.C);
        bp[k] = (const global_u32x4*)(words + e.y);
        la[k] = blocks_addr + 16u * (uint32_t)e.z;
        ns[k] = e.w;
        if (e.x < 0) {  // the root is a leaf
            atomicAdd(&vl[vrow[k] - e.x - 1], 1);
            return kDone;
        }
        return e.x;
    };
    bool drained = false;
    while (true) {
        if (!drained) refill<K>(ref, pool, U, (uint32_t)rows_here, rmagic, ttab, j.refill_min, lane, drained, take);
        bool live = false;
#pragma unroll
        for (int k = 0; k < K; k++) live |= ref[k] >= 0;
        if (__ballot(live) == 0) {
            if (drained) break;
            continue;
        }
        uint4 q[K][4];
#pragma unroll
        for (int k = 0; k < K; k++)
            if (ref[k] >= 0) fetch_block<B48>(bp[k], la[k], ns[k], ref[k], q[k]);
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (ref[k] < 0) continue;
            int32_t nr;
            if constexpr (X16) {
                nr = cluster_step<true, true>(q[k], xrow[k], le16);
            } else if constexpr (FMT >= 2) {
                nr = cluster_step<FMT == 3, false>(q[k], xrow[k], le);
            } else if (const BlockView b = view_block<B48>(q[k]); feat_lds) {
                // all seven split tests (absent slots are zero words: feature
                // 0, harmless) packed into a mask of sides, bit s set = slot s
                // goes right; the path reads the mask, so the seven LDS reads
                // issue together, ahead of any branch
                uint32_t gm = 0;
#pragma unroll
                for (int sl = 0; sl < 7; sl++)
                    gm |= (lds_ptr<float>((uint32_t)xrow[k])[b.w[sl] & fmask] <= __uint_as_float(b.t[sl]) ? 0u : 1u) << sl;
                const uint32_t side0 = gm & 1u;
                const uint32_t c0 = (b.w[0] >> (side0 ? sh_r : sh_l)) & code_mask;
                const uint32_t side1 = (gm >> (1 + side0)) & 1u;
                const uint32_t w1 = side0 ? b.w[2] : b.w[1];
                const uint32_t c1 = (w1 >> (side1 ? sh_r : sh_l)) & code_mask;
                const uint32_t idx = 2 * side0 + side1;
                const uint32_t side2 = (gm >> (3 + idx)) & 1u;
                const uint32_t w2 = side0 ? (side1 ? b.w[6] : b.w[5]) : (side1 ? b.w[4] : b.w[3]);
                const uint32_t c2 = (w2 >> (side2 ? sh_r : sh_l)) & code_mask;
                int32_t r = exit_to(b, 2 * idx + side2, c2);
                r = (c2 & 1u) ? ~(int32_t)(c2 >> 1) : r;
                r = (c1 & 1u) ? ~(int32_t)(c1 >> 1) : r;
                nr = (c0 & 1u) ? ~(int32_t)(c0 >> 1) : r;
            } else {
                // features from memory: one level at a time
                uint32_t side = le(xrow[k], b.w[0] & fmask, __uint_as_float(b.t[0])) ? 0u : 1u;
                uint32_t c = (b.w[0] >> (side ? sh_r : sh_l)) & code_mask;
                if (c & 1u) {
                    nr = ~(int32_t)(c >> 1);
                } else {
                    const uint32_t s1 = side;
                    const uint32_t w1 = s1 ? b.w[2] : b.w[1];
                    side = le(xrow[k], w1 & fmask, __uint_as_float(s1 ? b.t[2] : b.t[1])) ? 0u : 1u;
                    c = (w1 >> (side ? sh_r : sh_l)) & code_mask;
                    if (c & 1u) {
                        nr = ~(int32_t)(c >> 1);
                    } else {
                        const uint32_t idx = 2 * s1 + side;
                        const uint32_t w2 = s1 ? (side ? b.w[6] : b.w[5]) : (side ? b.w[4] : b.w[3]);
                        const uint32_t t2 = s1 ? (side ? b.t[6] : b.t[5]) : (side ? b.t[4] : b.t[3]);
                        side = le(xrow[k], w2 & fmask, __uint_as_float(t2)) ? 0u : 1u;
                        c = (w2 >> (side ? sh_r : sh_l)) & code_mask;
                        nr = (c & 1u) ? ~(int32_t)(c >> 1) : exit_to(b, 2 * idx + side, c);
                    }
                }
            }
            if (nr < 0) {
                atomicAdd(&vl[vrow[k] - nr - 1], 1);
                nr = kDone;
            }
            ref[k] = nr;
        }
    }
    write_tile(j, vl, row0, rows_here);
}

// One forest: persistent workgroups, group = blockIdx % G (consecutive
// workgroups land on different XCDs, so G = 8 gives each XCD its own trees).
// Waves per SIMD the kernel must allow: two 1024-thread workgroups per CU
// (8 waves per SIMD, at most 64 VGPRs) while the cursors fit in that budget.
// COMPACT and BLOCKED cursors carry more state (a BLOCKED one holds a
// 64-byte block in 16 registers while it walks it).  A 1024-thread workgroup
// needs 4 waves per SIMD, so no variant gets more than 128 VGPRs.
template <int K, int LAYOUT>
struct MinWaves {
    static constexpr int value = LAYOUT == FP_LAYOUT_PACKED    ? (K <= 4 ? 8 : 4)
                                 : LAYOUT == FP_LAYOUT_COMPACT ? (K <= 2 ? 8 : 4)
                                                               : (K == 1 ? 8 : 4);
};

template <int K, int FMODE, int LAYOUT>
__global__ __launch_bounds__(1024, (MinWaves<K, LAYOUT>::value)) void packed_kernel(JobDesc j) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int group = j.group_base + (int)(blockIdx.x % j.G);
    const int blocks_per_group = gridDim.x / j.G;
    const int nt = stage_group(j, group, smem);
    if (nt == 0) return;  // uniform per block
    for (int tile = blockIdx.x / j.G; tile < j.n_tiles; tile += blocks_per_group) {
        if (LAYOUT == FP_LAYOUT_COMPACT) run_tile_compact<K, FMODE>(j, nt, tile, smem);
        else if (LAYOUT == FP_LAYOUT_BLOCKED && j.block_bytes == 48) run_tile_blocked<K, FMODE, 0>(j, nt, tile, smem);
        else if (LAYOUT == FP_LAYOUT_BLOCKED) run_tile_blocked<K, FMODE, 1>(j, nt, tile, smem);
        else if (LAYOUT == FP_LAYOUT_CLUSTERED && j.block_bytes == 48) {
            if constexpr (FMODE == 1) {
                if (j.x16) run_tile_blocked<K, 1, 4>(j, nt, tile, smem);
                else run_tile_blocked<K, 1, 3>(j, nt, tile, smem);
            } else {
                run_tile_blocked<K, FMODE, 3>(j, nt, tile, smem);
            }
        } else if (LAYOUT == FP_LAYOUT_CLUSTERED) run_tile_blocked<K, FMODE, 2>(j, nt, tile, smem);
        else run_tile<K, FMODE>(j, nt, tile, smem);
    }
}

// Many forests: persistent workgroups pull work items from a global counter
// (items are ordered largest first) and restage LDS when the (job, group)
// changes.  Every workgroup exits once the counter passes n_items.
// Tiles [tile_begin, tile_end) of one work item, features in LDS (FM 1) or
// read from memory (FM 0).  Block layouts walk one block per lane.
// BLOCKS: every job of the launch is in a block layout (the host picks this
// variant only then), so the node-layout walks are not compiled in and do
// not set the kernel's register budget.
template <int K, int FM, bool BLOCKS>
__device__ __forceinline__ void item_tiles(const JobDesc& j, const WorkItem& w, int nt, unsigned char* smem) {
    for (int tile = w.tile_begin; tile < w.tile_end; tile++) {
        if (!BLOCKS && j.layout == FP_LAYOUT_COMPACT) {
            run_tile_compact<K, FM>(j, nt, tile, smem);
        } else if (j.layout == FP_LAYOUT_CLUSTERED && j.block_bytes == 48) {
            if constexpr (FM == 1) {
                if (j.x16) {
                    run_tile_blocked<1, 1, 4>(j, nt, tile, smem);
                    continue;
                }
            }
            run_tile_blocked<1, FM, 3>(j, nt, tile, smem);
        } else if (j.layout == FP_LAYOUT_CLUSTERED) {
            run_tile_blocked<1, FM, 2>(j, nt, tile, smem);
        } else if (j.layout == FP_LAYOUT_BLOCKED) {
            if (j.block_bytes == 48) run_tile_blocked<1, FM, 0>(j, nt, tile, smem);
            else run_tile_blocked<1, FM, 1>(j, nt, tile, smem);
        } else if constexpr (!BLOCKS) {
            run_tile<K, FM>(j, nt, tile, smem);
        }
    }
}

// The item number is broadcast through a slot at the end of the dynamic LDS
// (item_slot bytes in), not a static __shared__ variable: static LDS would
// add to every job's budget and leave two workgroups no longer fitting a CU.
template <int K, bool BLOCKS>
__global__ __launch_bounds__(1024, (K <= 2 ? 8 : 4)) void batched_kernel(const JobDesc* __restrict__ jobs,
                                                                         const WorkItem* __restrict__ items,
                                                                         int32_t n_items, int32_t* counter,
                                                                         int32_t item_slot) {
    extern __shared__ __align__(16) unsigned char smem[];
    int32_t* s_item = reinterpret_cast<int32_t*>(smem + item_slot);
    int staged_job = -1, staged_group = -1, nt = 0;
    while (true) {
        if (threadIdx.x == 0) *s_item = atomicAdd(counter, 1);
        __syncthreads();
        // the item is the workgroup's: readfirstlane makes that visible to the
        // compiler, so the item and its job descriptor are loaded into scalar
        // registers instead of occupying vector registers in every lane
        const int it = __builtin_amdgcn_readfirstlane(*s_item);
        __syncthreads();
        if (it >= n_items) break;
        const WorkItem w = items[it];
        const JobDesc j = jobs[w.job];
        if (w.job != staged_job || w.group != staged_group) {
            nt = stage_group(j, w.group, smem);
            staged_job = w.job;
            staged_group = w.group;
        }
        if (nt == 0) continue;
        // the feature source is fixed per job: walk with it compiled in
        if (j.feat_lds) item_tiles<K, 1, BLOCKS>(j, w, nt, smem);
        else item_tiles<K, 0, BLOCKS>(j, w, nt, smem);
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

// blockIdx.y = job: zero the votes of jobs that accumulate with atomics;
// block (0, 0) also clears the work counter.
__global__ void batched_prologue_kernel(const JobDesc* jobs, int32_t* counter) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *counter = 0;
    const JobDesc& j = jobs[blockIdx.y];
    if (!j.atomic_votes) return;
    const int64_t n = j.n_rows * j.C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        j.votes[i] = 0;
}

__global__ void batched_epilogue_kernel(const JobDesc* jobs) {
    const JobDesc& j = jobs[blockIdx.y];
    if (!j.atomic_votes || !j.cls) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < j.n_rows; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t* v = j.votes + i * j.C;
        int32_t best = 0, bestv = v[0];
        for (int c = 1; c < j.C; c++)
            if (v[c] > bestv) { bestv = v[c]; best = c; }
        j.cls[i] = best;
    }
}

int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fp_set_error(FP_EHIP, "%s launch: %s", what, hipGetErrorString(e));
    return FP_OK;
}

template <int K, int FM, int L>
const void* packed_fn() {
    return reinterpret_cast<const void*>(&packed_kernel<K, FM, L>);
}

template <int K, int L>
const void* packed_fn_fm(int fmode) {
    return fmode == 0 ? packed_fn<K, 0, L>() : packed_fn<K, 1, L>();
}

// A BLOCKED walk keeps one block in flight per lane whatever `cursors` says:
// a second block's 16 registers halve the waves a SIMD holds, which costs more
// than the overlap gains.
const void* pick_packed(int K, int fmode, int layout) {
    if (K != 1 && K != 2 && K != 4 && K != 8) return nullptr;
    if (layout == FP_LAYOUT_BLOCKED) return packed_fn_fm<1, FP_LAYOUT_BLOCKED>(fmode);
    if (layout == FP_LAYOUT_CLUSTERED) return packed_fn_fm<1, FP_LAYOUT_CLUSTERED>(fmode);
#define FP_PICK(KK)                                                                     \
    if (K == KK)                                                                        \
        return layout == FP_LAYOUT_COMPACT ? packed_fn_fm<KK, FP_LAYOUT_COMPACT>(fmode) \
                                           : packed_fn_fm<KK, FP_LAYOUT_PACKED>(fmode);
    FP_PICK(1)
    FP_PICK(2)
    FP_PICK(4)
    FP_PICK(8)
#undef FP_PICK
    return nullptr;
}

// blocks_only: every job is in a block layout, which walks one block per
// lane whatever K is.
const void* pick_batched(int K, bool blocks_only) {
    if (K != 1 && K != 2 && K != 4 && K != 8) return nullptr;
    if (blocks_only) return reinterpret_cast<const void*>(&batched_kernel<1, true>);
    switch (K) {
        case 1: return reinterpret_cast<const void*>(&batched_kernel<1, false>);
        case 2: return reinterpret_cast<const void*>(&batched_kernel<2, false>);
        case 4: return reinterpret_cast<const void*>(&batched_kernel<4, false>);
        default: return reinterpret_cast<const void*>(&batched_kernel<8, false>);
    }
}

std::mutex g_props_mu;
fp::DeviceProps g_props[64];
bool g_props_ok[64];

size_t round16(size_t v) { return (v + 15) / 16 * 16; }

}  // namespace

namespace fp {

int current_device(int* dev) {
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return fp_set_error(FP_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    return FP_OK;
}

int device_props(int dev, DeviceProps* out) {
    if (dev < 0 || dev >= 64) return fp_set_error(FP_ENODEV, "device id %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_props_mu);
    if (!g_props_ok[dev]) {
        hipDeviceProp_t pr;
        hipError_t e = hipGetDeviceProperties(&pr, dev);
        if (e != hipSuccess) return fp_set_error(FP_EHIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
        g_props[dev].cus = pr.multiProcessorCount;
        g_props[dev].lds_per_block = pr.sharedMemPerBlock;
        g_props[dev].lds_per_cu = pr.maxSharedMemoryPerMultiProcessor;
        g_props_ok[dev] = true;
    }
    *out = g_props[dev];
    return FP_OK;
}

size_t default_lds_block(const DeviceProps& dp) {
    const size_t blk = dp.lds_per_block ? dp.lds_per_block : 65536;
    const size_t cu = dp.lds_per_cu ? dp.lds_per_cu : blk;
    return std::min(blk, cu / 2);
}

size_t job_lds_layout(JobDesc* j) {
    size_t o = 0;
    j->off_top = (int32_t)o;   o += (size_t)j->cap * j->bins_per_group * sizeof(Node16);
    j->off_ttab = (int32_t)o;  o += (size_t)j->trees_per_group * 16;
    j->off_fmap = (int32_t)o;  o += j->feat_lds ? 0 : round16((size_t)j->Fc * 4);
    j->off_imap = (int32_t)o;  o += j->stage_rows ? round16((size_t)(j->F + 3) / 4 * 4 * 2) : 0;
    j->off_xs = (int32_t)o;    o += j->feat_lds ? round16(j->x16 ? (size_t)j->Fc * j->Fcp * 2 : (size_t)j->R * j->Fcp * 4) : 0;
    j->off_votes = (int32_t)o; o += round16((size_t)j->R * j->C * 4);
    j->off_pool = (int32_t)o;  o += 16;
    j->lds_bytes = (int32_t)o;
    return o;
}

const BinEntry* bins_host(const fp_packed* p) {
    return reinterpret_cast<const BinEntry*>(p->bytes.data() + p->hdr.table_offset);
}

int resolve_job(const fp_packed* p, const fp_tune* t, const float* X, int64_t n_rows, int64_t ld, int32_t* votes,
                int32_t* cls, size_t lds_block, JobDesc* j) {
    const Header& h = p->hdr;
    if (h.layout != FP_LAYOUT_PACKED && h.layout != FP_LAYOUT_COMPACT && h.layout != FP_LAYOUT_BLOCKED &&
        h.layout != FP_LAYOUT_CLUSTERED)
        return fp_set_error(FP_EINVAL, "forest is not in a packed layout");
    if (!p->dev) return fp_set_error(FP_ENODEV, "packed forest is not uploaded");
    if (h.n_nodes >= INT32_MAX)
        return fp_set_error(FP_E2BIG, "packed forest has %lld nodes (limit 2^31-1)", (long long)h.n_nodes);
    // rows_per_block 0: start at 16 and halve until the workgroup's tables fit
    const bool auto_R = t->rows_per_block <= 0;
    int R = auto_R ? 16 : t->rows_per_block;
    if (R > 4096) return fp_set_error(FP_EINVAL, "rows_per_block %d exceeds 4096", R);
    int G = t->tree_groups > 0 ? t->tree_groups : 1;
    if (G > h.n_bins) G = h.n_bins;
    int P = t->tree_passes > 0 ? t->tree_passes : 1;
    if ((int64_t)P * G > h.n_bins) P = std::max(1, h.n_bins / G);
    const int bpg = (h.n_bins + P * G - 1) / (P * G);
    // passes that would hold no bin are dropped: the last pass writes the classes
    P = ((h.n_bins + bpg - 1) / bpg + G - 1) / G;
    const int tpg = (int)std::min<int64_t>((int64_t)bpg * h.bin_size, h.n_trees);
    if ((int64_t)R * tpg >= (1 << 30)) return fp_set_error(FP_E2BIG, "rows_per_block x trees per group too large");
    const uint8_t* base = static_cast<const uint8_t*>(p->dev);
    memset(j, 0, sizeof *j);
    j->bins = reinterpret_cast<const BinEntry*>(base + h.table_offset);
    j->roots = reinterpret_cast<const int32_t*>(base + h.roots_offset);
    j->fmap = reinterpret_cast<const int32_t*>(base + h.fmap_offset);
    j->nodes = reinterpret_cast<const Node16*>(base + h.nodes_offset);
    j->X = X;
    j->ld = ld;
    j->n_rows = n_rows;
    j->votes = votes;
    j->cls = cls;
    j->Fc = h.n_used_features;
    j->Fcp = h.n_used_features | 1;
    j->C = h.n_classes;
    j->n_bins = h.n_bins;
    j->bin_size = h.bin_size;
    j->R = R;
    j->G = G;
    j->passes = P;
    j->bins_per_group = bpg;
    j->trees_per_group = tpg;
    j->n_tiles = (int32_t)((n_rows + R - 1) / R);
    j->atomic_votes = G > 1;
    j->layout = h.layout;
    j->fbits = h.compact_fbits;
    j->cbits = h.compact_cbits;
    j->block_bytes = h.block_bytes;
    if (t->refill_lanes < 0 || t->refill_lanes > 64) return fp_set_error(FP_EINVAL, "refill_lanes %d outside [0, 64]", t->refill_lanes);
    j->refill_min = t->refill_lanes > 0 ? t->refill_lanes : kDefaultRefillLanes;
    // feature_lds: 1 force LDS staging, 2 force it in fp32, -1 read features
    // from memory, 0 automatic
    if (t->feature_lds < -1 || t->feature_lds > 2) return fp_set_error(FP_EINVAL, "feature_lds %d outside [-1, 2]", t->feature_lds);
    // fp16 tile: exact where every threshold is exact in fp16 (the CLUSTERED
    // 48-byte form)
    const bool x16_ok = t->feature_lds != 2 && h.layout == FP_LAYOUT_CLUSTERED && h.block_bytes == 48;
    j->F = h.n_features;
    j->cap = 0;
    // LDS need of a tile of r rows, with or without the row tile in LDS
    auto size_for = [&](int r, bool feat) {
        j->R = r;
        j->n_tiles = (int32_t)((n_rows + r - 1) / r);
        j->feat_lds = feat;
        j->x16 = feat && x16_ok;
        // fp16 tile: feature-major, the feature stride an odd number of
        // 4-byte words (rows rounded up to 2 mod 4) so that strided writes
        // and reads spread over the banks; fp32 tile: row-major, odd stride
        j->Fcp = j->x16 ? r + (6 - r % 4) % 4 : h.n_used_features | 1;
        // whole-row staging: rows start on 16 bytes and the column map fits 8 KB
        j->stage_rows = feat && ld % 4 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0 && h.n_features <= 4096;
        return job_lds_layout(j);
    };
    // fit by shrinking an automatic tile first (features in LDS matter most),
    // then by reading features from memory
    auto fit = [&](bool feat) {
        size_t need = size_for(R, feat);
        for (int r = R; need > lds_block && auto_R && r > 1;) {
            r = std::max(1, r / 2);
            need = size_for(r, feat);
        }
        return need;
    };
    size_t need = fit(t->feature_lds >= 0);
    if (need > lds_block) {
        if (t->feature_lds >= 1)
            return fp_set_error(FP_E2BIG, "observation tile of %d rows x %d columns does not fit in %zu bytes of LDS",
                                R, j->Fc, lds_block);
        need = fit(false);
        if (need > lds_block)
            return fp_set_error(FP_E2BIG, "per-workgroup tables of %zu bytes exceed %zu bytes of LDS", need, lds_block);
    }
    // LDS left over holds the hottest nodes: PACKED bin tops, or the first
    // blocks of each BLOCKED bin (its trees' root blocks come first), counted
    // in 16-byte pieces per bin
    size_t top_nodes = (lds_block - need) / sizeof(Node16);
    if (t->lds_top_nodes < 0 || h.layout == FP_LAYOUT_COMPACT) top_nodes = 0;  // COMPACT: tops from memory
    else if (t->lds_top_nodes > 0) top_nodes = std::min(top_nodes, (size_t)t->lds_top_nodes);
    if (h.layout >= FP_LAYOUT_BLOCKED) {
        const size_t bw = (size_t)h.block_bytes / 16;
        int64_t max_blocks = 0;
        for (int32_t b = 0; b < h.n_bins; b++) max_blocks = std::max<int64_t>(max_blocks, bins_host(p)[b].deep_len);
        j->cap = (int32_t)(std::min<size_t>(top_nodes / bpg / bw, (size_t)max_blocks) * bw);
    } else {
        j->cap = (int32_t)std::min<size_t>(top_nodes / bpg, (size_t)h.max_top_len);
    }
    job_lds_layout(j);
    return FP_OK;
}

int packed_occupancy(int K, int fmode, int layout, int threads, size_t lds, int* blocks_per_cu) {
    const void* fn = pick_packed(K, fmode, layout);
    if (!fn) return fp_set_error(FP_EINVAL, "cursors must be 1, 2, 4 or 8");
    int occ = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, threads, lds);
    *blocks_per_cu = (e == hipSuccess && occ > 0) ? occ : 1;
    return FP_OK;
}

bool jobs_blocks_only(const JobDesc* jobs, int32_t n_jobs) {
    for (int32_t i = 0; i < n_jobs; i++)
        if (jobs[i].layout < FP_LAYOUT_BLOCKED) return false;
    return true;
}

size_t batched_job_budget(size_t lds_block) { return lds_block > kItemSlotBytes ? lds_block - kItemSlotBytes : 0; }

int batched_occupancy(int K, bool blocks_only, int threads, size_t lds, int* blocks_per_cu) {
    const void* fn = pick_batched(K, blocks_only);
    if (!fn) return fp_set_error(FP_EINVAL, "cursors must be 1, 2, 4 or 8");
    int occ = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, threads, round16(lds) + kItemSlotBytes);
    *blocks_per_cu = (e == hipSuccess && occ > 0) ? occ : 1;
    return FP_OK;
}

int launch_leaf_counts(const Node16* nodes, const int64_t* tree_off, int32_t n_trees, const float* X, int64_t n_rows,
                       int64_t ld, int32_t* counts, hipStream_t s) {
    if (n_rows <= 0 || n_trees <= 0) return FP_OK;
    const int64_t blocks = std::min<int64_t>((n_rows + 255) / 256, 65536);
    hipLaunchKernelGGL(leaf_count_kernel, dim3((unsigned)blocks), dim3(256), 0, s, nodes, tree_off, n_trees, X, n_rows,
                       ld, counts);
    return check_launch("leaf_count_kernel");
}

int device_upload(void* dev, const void* src, size_t n, void* stream_v, int* dev_id) {
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    hipError_t e = hipGetDevice(dev_id);
    if (e != hipSuccess) return fp_set_error(FP_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    e = hipMemcpyAsync(dev, src, n, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return fp_set_error(FP_EHIP, "hipMemcpyAsync: %s", hipGetErrorString(e));
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fp_set_error(FP_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return FP_OK;
}

int device_leaf_counts(const uint8_t* bytes, size_t nbytes, const Header& h, int32_t n_trees, const float* X,
                       int64_t n_rows, int64_t ld, int32_t* counts, void* stream_v) {
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    DevBuf buf, cnt;
    int rc = buf.ensure(nbytes);
    if (!rc) rc = cnt.ensure(sizeof(int32_t) * (size_t)h.n_nodes);
    if (rc) return rc;
    // once work is queued, every exit waits for the stream before the
    // buffers above (and the host arrays the copies use) go away
    struct Drain {
        hipStream_t s;
        ~Drain() { (void)hipStreamSynchronize(s); }
    } drain{stream};
    hipError_t e = hipMemcpyAsync(buf.p, bytes, nbytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * (size_t)h.n_nodes, stream);
    if (e != hipSuccess) return fp_set_error(FP_EHIP, "upload: %s", hipGetErrorString(e));
    const uint8_t* base = static_cast<const uint8_t*>(buf.p);
    rc = launch_leaf_counts(reinterpret_cast<const Node16*>(base + h.nodes_offset),
                            reinterpret_cast<const int64_t*>(base + h.table_offset), n_trees, X, n_rows, ld,
                            static_cast<int32_t*>(cnt.p), stream);
    if (rc) return rc;
    e = hipMemcpyAsync(counts, cnt.p, sizeof(int32_t) * (size_t)h.n_nodes, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fp_set_error(FP_EHIP, "counts: %s", hipGetErrorString(e));
    return FP_OK;
}

int launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return FP_OK;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s, p, n, v);
    return check_launch("fill_i32_kernel");
}

int launch_argmax(const int32_t* votes, int32_t* cls, int64_t n, int32_t C, hipStream_t s) {
    if (n <= 0) return FP_OK;
    hipLaunchKernelGGL(argmax_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s, votes,
                       cls, n, C);
    return check_launch("argmax_kernel");
}

int launch_packed(const JobDesc& j, int K, int threads, int blocks, hipStream_t s) {
    const void* fn = pick_packed(K, j.feat_lds ? 1 : 0, j.layout);
    if (!fn) return fp_set_error(FP_EINVAL, "cursors must be 1, 2, 4 or 8");
    JobDesc a = j;
    void* args[] = {&a};
    hipError_t e = hipLaunchKernel(fn, dim3(blocks), dim3(threads), args, (size_t)j.lds_bytes, s);
    if (e != hipSuccess) return fp_set_error(FP_EHIP, "packed_kernel launch: %s", hipGetErrorString(e));
    return FP_OK;
}

int launch_batched(const JobDesc* jobs, const WorkItem* items, int32_t n_items, int32_t* counter, int K,
                   bool blocks_only, int threads, size_t lds_bytes, int blocks, hipStream_t s) {
    const void* fn = pick_batched(K, blocks_only);
    if (!fn) return fp_set_error(FP_EINVAL, "cursors must be 1, 2, 4 or 8");
    int32_t item_slot = (int32_t)round16(lds_bytes);
    void* args[] = {&jobs, &items, &n_items, &counter, &item_slot};
    hipError_t e = hipLaunchKernel(fn, dim3(blocks), dim3(threads), args, (size_t)item_slot + kItemSlotBytes, s);
    if (e != hipSuccess) return fp_set_error(FP_EHIP, "batched_kernel launch: %s", hipGetErrorString(e));
    return FP_OK;
}

int launch_batched_prologue(const JobDesc* jobs_dev, int32_t n_jobs, int32_t* counter, hipStream_t s) {
    hipLaunchKernelGGL(batched_prologue_kernel, dim3(64, n_jobs), dim3(256), 0, s, jobs_dev, counter);
    return check_launch("batched_prologue_kernel");
}

int launch_batched_epilogue(const JobDesc* jobs_dev, int32_t n_jobs, hipStream_t s) {
    hipLaunchKernelGGL(batched_epilogue_kernel, dim3(64, n_jobs), dim3(256), 0, s, jobs_dev);
    return check_launch("batched_epilogue_kernel");
}

}  // namespace fp

// ---------------------------------------------------------------------------
// single-forest entry points
// ---------------------------------------------------------------------------
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
    int rc = fp::current_device(&dev);
    if (rc) return rc;
    if (dev != p->dev_id) return fp_set_error(FP_ENODEV, "forest uploaded to device %d, current device is %d", p->dev_id, dev);
    fp::DeviceProps dp;
    rc = fp::device_props(dev, &dp);
    if (rc) return rc;
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    const int threads = tune && tune->block_threads > 0 ? tune->block_threads : 256;
    if (threads % 64 || threads < 64 || threads > 1024)
        return fp_set_error(FP_EINVAL, "block_threads %d must be a multiple of 64 in [64, 1024]", threads);

    if (h.layout == FP_LAYOUT_NAIVE) {
        const uint8_t* base = static_cast<const uint8_t*>(p->dev);
        NaiveArgs a{reinterpret_cast<const int64_t*>(base + h.table_offset),
                    reinterpret_cast<const Node16*>(base + h.nodes_offset), X, ld, n_rows, votes, cls, h.n_trees,
                    h.n_classes};
        const size_t lds = (size_t)h.n_classes * threads * 4;
        const bool use_lds = lds <= 32768;
        const int blocks = (int)((n_rows + threads - 1) / threads);
        if (use_lds)
            hipLaunchKernelGGL(naive_kernel<true>, dim3(blocks), dim3(threads), lds, stream, a);
        else
            hipLaunchKernelGGL(naive_kernel<false>, dim3(blocks), dim3(threads), 0, stream, a);
        return check_launch("naive_kernel");
    }

    const int K = tune && tune->cursors > 0 ? tune->cursors : 2;
    if (K != 1 && K != 2 && K != 4 && K != 8) return fp_set_error(FP_EINVAL, "cursors must be 1, 2, 4 or 8");
    const size_t lds_max = dp.lds_per_block ? dp.lds_per_block : 65536;
    if (tune && tune->lds_bytes < 0) return fp_set_error(FP_EINVAL, "lds_bytes %d < 0", tune->lds_bytes);
    const size_t lds_block = tune && tune->lds_bytes > 0      ? std::min((size_t)tune->lds_bytes, lds_max)
                             : tune && tune->lds_top_nodes > 0 ? lds_max
                                                               : fp::default_lds_block(dp);
    fp::JobDesc j;
    rc = fp::resolve_job(p, tune, X, n_rows, ld, votes, cls, lds_block, &j);
    if (rc) return rc;
    int occ = 1;
    rc = fp::packed_occupancy(K, j.feat_lds, j.layout, threads, (size_t)j.lds_bytes, &occ);
    if (rc) return rc;
    const int64_t per_group = std::min<int64_t>(j.n_tiles, std::max<int64_t>(1, (int64_t)dp.cus * occ / j.G));
    const int blocks = (int)std::max<int64_t>(1, per_group) * j.G;
    if (j.atomic_votes) {
        rc = fp::launch_fill(votes, n_rows * h.n_classes, 0, stream);
        if (rc) return rc;
    }
    // one launch per pass; with one group per pass the first stores the votes
    // and later ones add to them (the last also writes the classes), with
    // several concurrent groups every pass adds with atomics
    for (int pass = 0; pass < j.passes; pass++) {
        fp::JobDesc jp = j;
        jp.group_base = pass * j.G;
        jp.accumulate = !j.atomic_votes && pass > 0;
        jp.cls = (!j.atomic_votes && pass == j.passes - 1) ? cls : nullptr;
        rc = fp::launch_packed(jp, K, threads, blocks, stream);
        if (rc) return rc;
    }
    if (j.atomic_votes && cls) return fp::launch_argmax(votes, cls, n_rows, h.n_classes, stream);
    return FP_OK;
}

// The launch parameters: the tune recorded for p's batch-size bucket
// (fp_tune_launch, this process or the FP_TUNE_CACHE file), else p's own.
extern "C" int fp_predict(const fp_packed* p, const float* X_dev, int64_t n_rows, int64_t ld, int32_t* votes_dev,
                          int32_t* class_dev, void* stream) {
    if (!p) return fp_set_error(FP_EINVAL, "packed forest is NULL");
    fp_tune t;
    if (p->hdr.layout != FP_LAYOUT_NAIVE && n_rows > 0 && fp::launch_tune_get(p, n_rows, 0, 0, &t))
        return predict_impl(p, &t, X_dev, n_rows, ld, votes_dev, class_dev, stream);
    return predict_impl(p, &p->tune, X_dev, n_rows, ld, votes_dev, class_dev, stream);
}

extern "C" int fp_predict_tune_get(const fp_packed* p, int64_t n_rows, fp_tune* out, int32_t* source) {
    fp_clear_error();
    if (!p || !out) return fp_set_error(FP_EINVAL, "NULL argument");
    int32_t src = p->has_tune ? 1 : 0;
    *out = p->tune;
    fp_tune t;
    if (p->hdr.layout != FP_LAYOUT_NAIVE && n_rows > 0 && fp::launch_tune_get(p, n_rows, 0, 0, &t)) {
        *out = t;
        src = 2;
    }
    if (source) *source = src;
    return FP_OK;
}

extern "C" int fp_predict_tuned(const fp_packed* p, const fp_tune* tune, const float* X_dev, int64_t n_rows,
                                int64_t ld, int32_t* votes_dev, int32_t* class_dev, void* stream) {
    if (!p) return fp_set_error(FP_EINVAL, "packed forest is NULL");
    return predict_impl(p, tune ? tune : &p->tune, X_dev, n_rows, ld, votes_dev, class_dev, stream);
}
