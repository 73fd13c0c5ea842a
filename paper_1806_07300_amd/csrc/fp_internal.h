// Internal definitions shared by the host packer and the HIP launch code.
#pragma once

#include <stdint.h>
#include <stddef.h>

#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "forestpack.h"

namespace fp {

// ---------------------------------------------------------------------------
// Packed buffer format (version kFormatVersion below).  Little-endian; every section starts on a
// 256-byte boundary so that the device copy keeps 128-byte line alignment.
//
//   [Header 256 B]
//   PACKED: [BinEntry x n_bins] [root refs int32 x n_trees]
//           [feature map int32 x n_used_features] [Node16 x n_nodes]
//   NAIVE : [tree offsets int64 x (n_trees+1)]             [Node16 x n_nodes]
//
// PACKED node references (left/right, roots) are bin-relative: r >= 0 is the
// r-th node of the bin (top region first, then the deep region); r < 0 is
// "class -r-1" (a leaf folded into its class, DF- of Sec. III-A).
// PACKED node features are compacted: a node tests observation column
// feature_map[feat]; the map lists, in increasing order, the columns that at
// least one split uses, so a kernel only stages those columns.
// NAIVE nodes keep leaves: feature < 0 marks a leaf whose class is `left`;
// internal children are tree-local ids.
// ---------------------------------------------------------------------------
constexpr uint64_t kMagic = 0x314B4341504D5046ull;  // "FPMPACK1"
constexpr uint32_t kFormatVersion = 7;
constexpr size_t kSectionAlign = 256;

struct alignas(16) Node16 {
    float thr;
    int32_t feat;
    int32_t left;
    int32_t right;
};
static_assert(sizeof(Node16) == 16, "node is 16 bytes");

// COMPACT layout: the node section is an array of 8-byte words.  A bin's
// top region holds Node16 entries (two words each); its deep region holds
// Node8 entries in Stat pre-order.  References (roots, Node16 children) live
// in one space per bin: r < top_len is top node r, r >= top_len is deep node
// r - top_len, r < 0 is class -r-1.  A Node8 at deep index i (reference
// p = top_len + i) packs in `w`:
//   bits [0, fb)        compacted feature
//   bit fb      ADJ     the child at p + 1 is internal (the hot child of Stat)
//   bit fb + 1  ADJ_L   that adjacent child is the left one
//   bit fb + 2  COLD_C  the other child is a class (else an internal node)
//   bits [fb+3, 32)     payload: ADJ & COLD_C: its class; ADJ & !COLD_C: its
//                       reference minus p (>= 2); !ADJ (both children are
//                       leaves): left class | right class << cb
struct Node8 {
    float thr;
    uint32_t w;
};
static_assert(sizeof(Node8) == 8, "compact node is 8 bytes");

// BLOCKED layout: a bin is an array of 64-byte blocks (top_len = 0, deep_len
// = block count); a reference r >= 0 names block r of the bin, entered at
// slot 0, r < 0 is class -r-1.  Slot s (0..6) of a block is the
// heap position of a complete three-level subtree (children of s at 2s+1 and
// 2s+2).  Node word w: bits [0, fb) feature; then a left code and a right
// code of (1 + cb) bits each: bit 0 set = class child (class in the other cb
// bits), clear = internal child (in the block for s < 3, else an exit).
// Exit e = 2 (s - 3) + side of a bottom slot leads to block
// child_base + rank[e], rank[e] = bits [4e, 4e + 3) of `ranks`; children of a
// block are stored together, the one with the most training samples first.
struct Block64 {
    uint32_t child_base;  // bin-relative block index of the first child block
    uint32_t ranks;       // 4 bits per exit: rank in the child group (bit 3: exit used)
    Node8 slot[7];
};
static_assert(sizeof(Block64) == 64, "block is 64 bytes");

// The 48-byte form of a BLOCKED block, used when a node word fits 19 bits.
// Bits [19 s, 19 s + 19) of words[0..4] (136 bits) are the word of slot s:
// feature in bits [0, fb), then a left and a right code of (1 + P) bits,
// P = max(cb, 3): bit 0 set = class child (class in the other P bits); clear
// = internal child, whose other P bits are 0 for s < 3 (the child is slot
// 2s+1+side) and the exit rank for s >= 3 (the child is block child_base +
// rank).  Bits [8, 32) of words[4] hold child_base; thr[s] follows.
struct Block48 {
    uint32_t words[5];
    float thr[7];
};
static_assert(sizeof(Block48) == 48, "block is 48 bytes");
constexpr int kBlock48WordBits = 19;
constexpr uint32_t kBlock48MaxChildBase = (1u << 24) - 1;

// CLUSTERED layout block (64 bytes): up to 7 internal nodes of one tree
// chosen greedily by training cardinality from the block's root (the most
// visited connected group), in slots 0..6 (slot 0 = the root), and the up to
// 8 edges that leave them ("exits": a leaf's class or a child block).  An
// exit is selected by the split outcomes of the slots on its path: with g =
// the 7-bit mask of outcomes (bit s set = slot s goes right), exit e is
// taken iff (g ^ val[e]) & care[e] == 0.  The used exits partition all 128
// masks; an unused exit has care = val = 0x80 and never matches (g < 128).
// care[] and val[] are bytes so that four exits are tested with one 32-bit
// operation.  rest[] fields (little-endian over rest[0..4]): [0, 48) target
// of exit e in 6 bits at 6 e (bit 5 set = child block child_base + bits 0..2,
// clear = class bits 0..4); [48, 132) feature of slot s in 12 bits at
// 48 + 12 s; [132, 156) child_base; [156, 160) number of child blocks.
// Absent slots and unused targets are zero.
struct BlockC64 {
    float thr[7];
    uint8_t care[8];
    uint8_t val[8];
    uint32_t rest[5];
};
static_assert(sizeof(BlockC64) == 64, "block is 64 bytes");
constexpr int kClusterFeatBits = 12, kClusterMaxClasses = 32;

// The 48-byte form of a CLUSTERED block, used when every threshold of the
// forest converts to fp16 and back unchanged (integer-valued features split
// at half-integers, for example) and at most 512 features are used: the
// same exits, with thr16[s] the fp16 bits of slot s's threshold, and rest
// fields (little-endian over rest[0..3], then rest_hi as bits [128, 144)):
// [0, 48) targets as in BlockC64; the 9-bit feature of slot s at
// kC48FeatPos[s], placed so that none crosses a 32-bit word; [57, 61) the
// number of child blocks; [123, 144) child_base (21 bits).  Bits [61, 64)
// and [91, 96) are zero.
struct BlockC48 {
    uint16_t thr16[7];
    uint16_t rest_hi;  // bits [128, 144) of rest
    uint8_t care[8];
    uint8_t val[8];
    uint32_t rest[4];
};
static_assert(sizeof(BlockC48) == 48, "block is 48 bytes");
constexpr int kCluster48FeatBits = 9;
constexpr int kC48FeatPos[7] = {48, 64, 73, 82, 96, 105, 114};
constexpr int kC48NChildPos = 57, kC48BasePos = 123, kC48BaseBits = 21;
constexpr uint32_t kC48MaxChildBase = (1u << kC48BaseBits) - 1u;

struct BinEntry {
    int64_t node_base;   // first node of the bin in the node array
    int32_t first_tree;
    int32_t n_trees;
    int32_t top_len;     // nodes of depths 0..D (interleaved region)
    int32_t deep_len;    // nodes below depth D
    int32_t root_base;   // index of the bin's first root ref
    int32_t pad;
};
static_assert(sizeof(BinEntry) == 32, "bin entry is 32 bytes");

struct Header {
    uint64_t magic;
    uint32_t version;
    int32_t layout;
    int32_t n_trees, n_features, n_classes, bin_size;
    int32_t interleave_depth, n_bins, max_top_len, max_bin_trees;
    int64_t total_bytes;
    int64_t table_offset;   // BinEntry[] (packed) or tree offsets (naive)
    int64_t roots_offset;   // root refs (packed), 0 for naive
    int64_t nodes_offset;
    int64_t n_nodes;
    int64_t n_internal, n_leaves;
    int32_t max_depth, line_align;
    uint64_t checksum;      // FNV-1a over 64-bit words of bytes [256, total_bytes)
    int32_t n_used_features, pad0;
    int64_t fmap_offset;    // feature map (packed), 0 for naive
    double expected_depth;  // mean over trees of the cardinality-weighted leaf depth
    int32_t compact_fbits;  // COMPACT, BLOCKED: feature bits fb of a node word
    int32_t compact_cbits;  // COMPACT, BLOCKED: class bits cb
    int32_t block_bytes;    // BLOCKED: 48 or 64
    int32_t pad1;
    double mean_bias;        // mean over internal nodes of max(LC, RC) / PN (cardinalities)
    double expected_fetches; // mean over trees of the cardinality-weighted fetch units per walk
    uint8_t pad[256 - 176];
};
static_assert(sizeof(Header) == 256, "header is 256 bytes");

uint64_t fnv1a64(const uint8_t* p, size_t n);

// Verifies header fields, section bounds, checksum and every reference.
int verify_buffer(const uint8_t* bytes, size_t n, std::string* why);

// Device-side limits of the packed kernel.
constexpr int kMaxClasses = 4096;
constexpr int kMaxCursors = 8;

// ---------------------------------------------------------------------------
// Launch descriptors shared by the single-forest and the batched kernels.
// ---------------------------------------------------------------------------

// Everything a workgroup needs to process one forest on one batch of rows.
// Plain data: copied to the device as a kernel argument or in a table.
struct JobDesc {
    const BinEntry* bins;
    const int32_t* roots;
    const int32_t* fmap;
    const Node16* nodes;
    const float* X;
    int64_t ld;
    int64_t n_rows;
    int32_t* votes;
    int32_t* cls;
    int32_t Fc, Fcp, C;        // used feature columns, LDS row stride (elements), classes
    int32_t n_bins, bin_size;
    int32_t R;                 // observations per tile
    int32_t G, bins_per_group, trees_per_group;
    int32_t cap;               // LDS nodes reserved per bin of a group (bin-top prefix)
    int32_t n_tiles;
    int32_t atomic_votes;      // several tree groups add into the same votes
    int32_t feat_lds;          // 1: observation tile in LDS, 0: read from memory
    int32_t off_top, off_ttab, off_fmap, off_xs, off_votes, off_pool, lds_bytes;
    int32_t layout;            // FP_LAYOUT_PACKED, FP_LAYOUT_COMPACT or FP_LAYOUT_BLOCKED
    int32_t fbits, cbits;      // COMPACT / BLOCKED field widths
    int32_t refill_min;        // idle lanes of a wavefront that trigger a refill
    int32_t block_bytes;       // BLOCKED: 48 or 64
    int32_t F;                 // feature columns of a row (the forest's n_features)
    int32_t stage_rows;        // 1: stage tiles with whole-row 16-byte loads through imap
    int32_t off_imap;          // LDS: column -> compacted feature (int16, -1 unused), 4 * ceil(F / 4) entries
    int32_t x16;               // 1: the LDS tile holds fp16 features rounded toward +inf (CLUSTERED 48-byte form)
    int32_t passes;            // consecutive launches over the groups (tree_passes), 1 in batched launches
    int32_t group_base;        // first group of this launch: workgroup b walks group group_base + b % G
    int32_t accumulate;        // 1: add the tile's votes to the stored ones (a later pass)
    int32_t pad_job;
};

// A job whose groups run in several passes, flattened for launches where all
// groups run concurrently (batched plans, the server): every group of every
// pass becomes a concurrent group, votes merged with atomics.
inline void flatten_passes(JobDesc* j) {
    if (j->passes > 1) {
        j->G *= j->passes;
        j->passes = 1;
        j->atomic_votes = j->G > 1;
    }
    j->group_base = 0;
    j->accumulate = 0;
}

// One entry of the batched work list: tiles [tile_begin, tile_end) of job
// `job`, trees of tree group `group`.
struct WorkItem {
    int32_t job, group, tile_begin, tile_end;
};

struct DeviceProps {
    int cus = 0;
    size_t lds_per_block = 0;
    size_t lds_per_cu = 0;
};

int current_device(int* dev);
int device_props(int dev, DeviceProps* out);

// LDS layout of a job (byte offsets); returns total bytes.
size_t job_lds_layout(JobDesc* j);

// Fill `j` for forest p, launch parameters t (threads and cursors decided by
// the caller), rows X.  `lds_block` caps the job's LDS footprint (bytes).
int resolve_job(const fp_packed* p, const fp_tune* t, const float* X, int64_t n_rows, int64_t ld,
                int32_t* votes, int32_t* cls, size_t lds_block, JobDesc* j);

// Default LDS footprint of one workgroup: what keeps two workgroups per CU.
size_t default_lds_block(const DeviceProps& dp);

int packed_occupancy(int K, int fmode, int layout, int threads, size_t lds, int* blocks_per_cu);
// Batched launches: `lds` is the largest job layout; the launch adds a
// 16-byte slot after it (the workgroup's item number), so jobs are resolved
// against batched_job_budget(lds_block).
constexpr size_t kItemSlotBytes = 16;
// Work items per resident workgroup a batched plan aims for.  Items are
// handed out largest estimated cost first; the estimate (rows x trees x
// expected depth) leaves out staging and cache behaviour, so finer items
// balance the end of a launch better: on the 64-forest workload 4 per
// workgroup took 19.8 ms, 8 16.7 ms, 16 14.8 ms, 64 14.4 ms.
constexpr int kDefaultItemsPerBlock = 16;
size_t batched_job_budget(size_t lds_block);
// blocks_only: every job of the launch is in a block layout (BLOCKED or
// CLUSTERED): the launch takes the kernel variant without node-layout walks.
int batched_occupancy(int K, bool blocks_only, int threads, size_t lds, int* blocks_per_cu);
bool jobs_blocks_only(const JobDesc* jobs, int32_t n_jobs);

// The packer's two device operations, kept out of the host-only packer:
// copy n bytes to device memory on `stream` and wait for it (the current
// device's id in *dev_id), and count on the GPU the rows of X that end in
// each leaf of a NAIVE-layout buffer (`bytes`, header h), node by node of
// that buffer into counts[h.n_nodes] (host), synchronising `stream`.
int device_upload(void* dev, const void* src, size_t n, void* stream, int* dev_id);
int device_leaf_counts(const uint8_t* bytes, size_t nbytes, const Header& h, int32_t n_trees, const float* X,
                       int64_t n_rows, int64_t ld, int32_t* counts, void* stream);

int launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t s);
// counts[i] += observations whose walk ends at node i of a NAIVE layout
int launch_leaf_counts(const Node16* nodes, const int64_t* tree_off, int32_t n_trees, const float* X, int64_t n_rows,
                       int64_t ld, int32_t* counts, hipStream_t s);
int launch_argmax(const int32_t* votes, int32_t* cls, int64_t n, int32_t C, hipStream_t s);
int launch_packed(const JobDesc& j, int K, int threads, int blocks, hipStream_t s);
int launch_batched(const JobDesc* jobs, const WorkItem* items, int32_t n_items, int32_t* counter, int K,
                   bool blocks_only, int threads, size_t lds_bytes, int blocks, hipStream_t s);
// Zero the work counter and the votes of every job that accumulates with atomics.
int launch_batched_prologue(const JobDesc* jobs_dev, int32_t n_jobs, int32_t* counter, hipStream_t s);
int launch_batched_epilogue(const JobDesc* jobs_dev, int32_t n_jobs, hipStream_t s);

// Launch tunes per (packed forest, batch-size bucket) and the autotuner's
// results, in a process-wide table mirrored to the FP_TUNE_CACHE file
// (tune.cpp).  threads / cursors 0 key the single-forest tunes fp_predict
// uses; a plan keys its fixed workgroup size and cursor count.
int32_t rows_bucket(int64_t n_rows);
uint64_t forest_key(const fp_packed* p);
bool launch_tune_get(const fp_packed* p, int64_t n_rows, int32_t threads, int32_t cursors, fp_tune* out);
void launch_tune_put(const fp_packed* p, int64_t n_rows, int32_t threads, int32_t cursors, const fp_tune& t);
bool autotune_cache_get(uint64_t key, fp_autotune_result* out);
void autotune_cache_put(uint64_t key, const fp_autotune_result& r);
// Times launch candidates of p on the first rows of X; fastest in *best.
int search_launch(const fp_packed* p, const float* X, int64_t n_rows, int64_t ld, int32_t threads, int32_t cursors,
                  hipStream_t stream, fp_tune* best, double* best_ms, int32_t* tried);

// Work list of a batched launch (plan.cpp): chunks of row tiles per (job,
// tree group), about `items_per_block` items per resident workgroup, largest
// estimated cost first.  `expected_depth[i]` is job i's forest cost model.
void build_items(const std::vector<JobDesc>& jobs, const std::vector<double>& expected_depth, int64_t resident,
                 int items_per_block, std::vector<WorkItem>* items, double* total_cost);
// The same into caller memory of cap items; returns the number of items
// (sorted only when it is at most cap).  Allocates nothing.
size_t build_items_into(const JobDesc* jobs, const double* expected_depth, size_t n, int64_t resident,
                        int items_per_block, WorkItem* out, size_t cap, double* total_cost);

}  // namespace fp

// ---------------------------------------------------------------------------
// Opaque object behind fp_packed*.
// ---------------------------------------------------------------------------
struct fp_packed {
    std::vector<uint8_t> bytes;  // whole buffer, header first
    fp::Header hdr;
    void* dev = nullptr;         // borrowed device copy
    size_t dev_cap = 0;
    int dev_id = -1;
    fp_tune tune{};
    bool has_tune = false;
};

// Error helpers (thread-local last error).
int fp_set_error(int code, const char* fmt, ...);
void fp_clear_error();

namespace fp {

// A device allocation owned by host code, released with the object.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    int ensure(size_t n) {
        if (n <= cap) return FP_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) return fp_set_error(FP_ENOMEM, "hipMalloc(%zu): %s", n, hipGetErrorString(e));
        cap = n;
        return FP_OK;
    }
};

}  // namespace fp
