// Internal definitions shared by the host packer and the HIP launch code.
#pragma once

#include <stdint.h>
#include <stddef.h>

#include <string>
#include <vector>

#include "forestpack.h"

namespace fp {

// ---------------------------------------------------------------------------
// Packed buffer format (version 1).  Little-endian; every section starts on a
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
constexpr uint32_t kFormatVersion = 2;
constexpr size_t kSectionAlign = 256;

struct alignas(16) Node16 {
    float thr;
    int32_t feat;
    int32_t left;
    int32_t right;
};
static_assert(sizeof(Node16) == 16, "node is 16 bytes");

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
    uint8_t pad[256 - 136];
};
static_assert(sizeof(Header) == 256, "header is 256 bytes");

uint64_t fnv1a64(const uint8_t* p, size_t n);

// Verifies header fields, section bounds, checksum and every reference.
int verify_buffer(const uint8_t* bytes, size_t n, std::string* why);

// Device-side limits of the packed kernel.
constexpr int kMaxClasses = 4096;
constexpr int kMaxCursors = 8;

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
