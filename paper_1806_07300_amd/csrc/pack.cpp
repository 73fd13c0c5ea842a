// Host packer: validates a trained forest and re-lays it (Sec. III-A).
//
//   NAIVE  : per-tree breadth-first arrays with leaves stored as nodes, the
//            BF baseline layout that the paper measures everything against.
//   PACKED : DF-  -- leaves are not stored; a child that is a leaf becomes the
//                    reference "class c" (-c-1), one shared class node per class
//                    as in DF- but needing no storage at all;
//            Stat -- below the interleaved levels, each tree is laid out depth
//                    first with the child reached by more training samples
//                    placed right after its parent (an internal child always
//                    wins over a leaf sibling, which is folded away);
//            Bin  -- trees are grouped into bins of B consecutive trees; depths
//                    0..D of all trees of a bin are interleaved level-major
//                    (all depth-0 nodes of the bin's trees, then all depth-1
//                    nodes, ...), each tree's nodes of one depth in
//                    breadth-first order, so the most used nodes of many trees
//                    share lines.  The kernels stage this top region in LDS.
//
// Every internal node index in a bin is larger than its parent's: children
// always come later (level-major top, pre-order deep region), which the
// verifier checks, so every walk terminates.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <new>

#include "fp_internal.h"

using fp::BinEntry;
using fp::Header;
using fp::Node16;
using fp::Node8;
using fp::Block48;
using fp::BlockC48;
using fp::BlockC64;
using fp::Block64;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

int fp_set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}
void fp_clear_error() { g_last_error.clear(); }

extern "C" const char* fp_last_error(void) { return g_last_error.c_str(); }
#define FP_STR2(x) #x
#define FP_STR(x) FP_STR2(x)
#define FP_FORMAT_VERSION 7
static_assert(FP_FORMAT_VERSION == fp::kFormatVersion, "version string follows the format");
extern "C" const char* fp_version(void) { return "forestpack 0.2 packed-format " FP_STR(FP_FORMAT_VERSION); }

namespace fp {

uint64_t fnv1a64(const uint8_t* p, size_t n) {
    // FNV-1a over little-endian 64-bit words (n is a multiple of 8 here).
    uint64_t h = 0xcbf29ce484222325ull;
    size_t w = n / 8;
    const uint64_t prime = 0x100000001b3ull;
    for (size_t i = 0; i < w; i++) {
        uint64_t v;
        memcpy(&v, p + 8 * i, 8);
        h = (h ^ v) * prime;
    }
    for (size_t i = 8 * w; i < n; i++) h = (h ^ p[i]) * prime;
    return h;
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

namespace {

// Per-tree structure recovered from the view.
struct TreeShape {
    int64_t base = 0, size = 0;
    std::vector<int32_t> bfs;     // reachable nodes, breadth-first, left before right
    std::vector<int32_t> depth;   // per local node (-1 unreachable)
    std::vector<int64_t> card;    // subtree cardinality per local node
    int64_t n_internal = 0, n_leaves = 0;
    int32_t max_depth = 0;
};

bool is_internal(const fp_forest_view* v, const TreeShape& t, int32_t n) {
    return v->feature[t.base + n] >= 0;
}

int validate_tree(const fp_forest_view* v, int32_t ti, TreeShape* t) {
    const int64_t base = v->tree_node_offset[ti];
    const int64_t size = v->tree_node_offset[ti + 1] - base;
    if (size < 1)
        return fp_set_error(FP_ECORRUPT, "tree %d has no nodes", ti);
    if (size > INT32_MAX / 2)
        return fp_set_error(FP_E2BIG, "tree %d has %lld nodes (limit %d)", ti, (long long)size,
                            INT32_MAX / 2);
    t->base = base;
    t->size = size;
    t->depth.assign(size, -1);
    t->bfs.clear();
    t->bfs.reserve(size);
    std::deque<int32_t> q;
    q.push_back(0);
    t->depth[0] = 0;
    while (!q.empty()) {
        int32_t n = q.front();
        q.pop_front();
        t->bfs.push_back(n);
        const int64_t g = base + n;
        const int32_t f = v->feature[g];
        if (f >= 0) {
            if (f >= v->n_features)
                return fp_set_error(FP_ECORRUPT, "tree %d node %d: feature %d >= n_features %d", ti,
                                    n, f, v->n_features);
            const int32_t ch[2] = {v->left[g], v->right[g]};
            for (int k = 0; k < 2; k++) {
                if (ch[k] < 0 || ch[k] >= size)
                    return fp_set_error(FP_ECORRUPT, "tree %d node %d: child %d out of range [0,%lld)",
                                        ti, n, ch[k], (long long)size);
                if (t->depth[ch[k]] >= 0)
                    return fp_set_error(FP_ECORRUPT,
                                        "tree %d node %d: child %d reached twice (cycle or shared node)",
                                        ti, n, ch[k]);
                t->depth[ch[k]] = t->depth[n] + 1;
                q.push_back(ch[k]);
            }
            t->n_internal++;
        } else {
            const int32_t c = v->leaf_class[g];
            if (c < 0 || c >= v->n_classes)
                return fp_set_error(FP_ECORRUPT, "tree %d leaf %d: class %d outside [0,%d)", ti, n, c,
                                    v->n_classes);
            t->n_leaves++;
            t->max_depth = std::max(t->max_depth, t->depth[n]);
        }
    }
    // subtree cardinalities, children before parents (reverse breadth-first)
    t->card.assign(size, 0);
    for (auto it = t->bfs.rbegin(); it != t->bfs.rend(); ++it) {
        const int32_t n = *it;
        const int64_t g = base + n;
        if (v->feature[g] >= 0) {
            t->card[n] = v->cardinality ? v->cardinality[g]
                                        : t->card[v->left[g]] + t->card[v->right[g]];
        } else {
            t->card[n] = v->cardinality ? v->cardinality[g] : 1;
        }
        if (t->card[n] < 0)
            return fp_set_error(FP_ECORRUPT, "tree %d node %d: negative cardinality", ti, n);
    }
    return FP_OK;
}

int validate_view(const fp_forest_view* v, std::vector<TreeShape>* shapes) {
    if (!v) return fp_set_error(FP_EINVAL, "forest view is NULL");
    if (v->n_trees < 1 || v->n_features < 1 || v->n_classes < 1)
        return fp_set_error(FP_EINVAL, "need n_trees, n_features, n_classes >= 1 (got %d, %d, %d)",
                            v->n_trees, v->n_features, v->n_classes);
    if (v->n_classes > kMaxClasses)
        return fp_set_error(FP_E2BIG, "n_classes %d exceeds %d", v->n_classes, kMaxClasses);
    if (!v->tree_node_offset || !v->feature || !v->threshold || !v->left || !v->right ||
        !v->leaf_class)
        return fp_set_error(FP_EINVAL, "forest view has a NULL array");
    if (v->tree_node_offset[0] != 0)
        return fp_set_error(FP_ECORRUPT, "tree_node_offset[0] must be 0");
    for (int32_t t = 0; t < v->n_trees; t++)
        if (v->tree_node_offset[t + 1] < v->tree_node_offset[t])
            return fp_set_error(FP_ECORRUPT, "tree_node_offset decreases at tree %d", t);
    shapes->resize(v->n_trees);
    for (int32_t t = 0; t < v->n_trees; t++) {
        int rc = validate_tree(v, t, &(*shapes)[t]);
        if (rc) return rc;
    }
    return FP_OK;
}

void fill_header_common(Header* h, const fp_forest_view* v, const std::vector<TreeShape>& s,
                        int32_t layout) {
    memset(h, 0, sizeof *h);
    h->magic = kMagic;
    h->version = kFormatVersion;
    h->layout = layout;
    h->n_trees = v->n_trees;
    h->n_features = v->n_features;
    h->n_classes = v->n_classes;
    double depth_sum = 0.0, bias_sum = 0.0;
    int64_t bias_n = 0;
    for (const auto& t : s) {
        h->n_internal += t.n_internal;
        h->n_leaves += t.n_leaves;
        h->max_depth = std::max(h->max_depth, t.max_depth);
        // expected internal nodes visited by a training-distributed observation
        // (the average depth of Eq. 1): leaf depths weighted by leaf cardinality
        double num = 0.0, den = 0.0;
        for (int32_t n : t.bfs) {
            const int64_t g = t.base + n;
            if (v->feature[g] < 0) {
                num += (double)t.card[n] * t.depth[n];
                den += (double)t.card[n];
            } else if (t.card[n] > 0) {
                // the bias of a split (Sec. III-A): max(LC, RC) / PN
                bias_sum += (double)std::max(t.card[v->left[g]], t.card[v->right[g]]) / (double)t.card[n];
                bias_n++;
            }
        }
        depth_sum += den > 0 ? num / den : 0.0;
    }
    h->expected_depth = depth_sum / (double)s.size();
    h->mean_bias = bias_n ? bias_sum / (double)bias_n : 0.0;
    // node layouts fetch one node per internal node visited; the naive layout
    // also fetches the leaf; block layouts overwrite this with blocks per walk
    h->expected_fetches = h->expected_depth + (layout == FP_LAYOUT_NAIVE ? 1.0 : 0.0);
}

void finish(std::vector<uint8_t>* bytes, Header* h) {
    h->total_bytes = (int64_t)bytes->size();
    h->checksum = fnv1a64(bytes->data() + sizeof(Header), bytes->size() - sizeof(Header));
    memcpy(bytes->data(), h, sizeof *h);
}

// Depth-first pre-order of a tree's nodes, left child first (the DF layout).
void depth_first(const fp_forest_view* v, const TreeShape& t, std::vector<int32_t>* order) {
    order->clear();
    std::vector<int32_t> stack{0};
    while (!stack.empty()) {
        const int32_t n = stack.back();
        stack.pop_back();
        order->push_back(n);
        const int64_t g = t.base + n;
        if (v->feature[g] < 0) continue;
        stack.push_back(v->right[g]);
        stack.push_back(v->left[g]);
    }
}

int pack_naive(const fp_forest_view* v, const std::vector<TreeShape>& s, const fp_pack_opts* opts,
               std::vector<uint8_t>* out, Header* h) {
    fill_header_common(h, v, s, FP_LAYOUT_NAIVE);
    const bool df = opts->node_order == FP_ORDER_DF;
    int64_t n_nodes = 0;
    for (const auto& t : s) n_nodes += (int64_t)t.bfs.size();
    const size_t table_off = sizeof(Header);
    const size_t nodes_off = align_up(table_off + sizeof(int64_t) * (v->n_trees + 1), kSectionAlign);
    const size_t total = align_up(nodes_off + sizeof(Node16) * (size_t)n_nodes, kSectionAlign);
    out->assign(total, 0);
    int64_t* offs = reinterpret_cast<int64_t*>(out->data() + table_off);
    Node16* nodes = reinterpret_cast<Node16*>(out->data() + nodes_off);
    int64_t o = 0;
    std::vector<int32_t> pos, dfo;
    for (int32_t ti = 0; ti < v->n_trees; ti++) {
        const TreeShape& t = s[ti];
        offs[ti] = o;
        if (df) depth_first(v, t, &dfo);
        const std::vector<int32_t>& order = df ? dfo : t.bfs;  // both hold every reachable node once
        pos.assign(t.size, -1);
        for (size_t k = 0; k < order.size(); k++) pos[order[k]] = (int32_t)k;
        for (size_t k = 0; k < order.size(); k++) {
            const int64_t g = t.base + order[k];
            Node16& nd = nodes[o + (int64_t)k];
            if (v->feature[g] >= 0) {
                nd.thr = v->threshold[g];
                nd.feat = v->feature[g];
                nd.left = pos[v->left[g]];
                nd.right = pos[v->right[g]];
            } else {
                nd.thr = 0.0f;
                nd.feat = -1;
                nd.left = v->leaf_class[g];
                nd.right = v->leaf_class[g];
            }
        }
        o += (int64_t)t.bfs.size();
    }
    offs[v->n_trees] = o;
    h->bin_size = 1;
    h->interleave_depth = 0;
    h->n_bins = v->n_trees;
    h->n_used_features = v->n_features;
    h->fmap_offset = 0;
    h->table_offset = (int64_t)table_off;
    h->roots_offset = 0;
    h->nodes_offset = (int64_t)nodes_off;
    h->n_nodes = n_nodes;
    finish(out, h);
    return FP_OK;
}

// Compacted feature numbering: the columns some split tests, in increasing order.
void feature_map(const fp_forest_view* v, const std::vector<TreeShape>& s, std::vector<int32_t>* remap,
                 std::vector<int32_t>* fmap) {
    remap->assign(v->n_features, -1);
    fmap->clear();
    for (int32_t ti = 0; ti < v->n_trees; ti++)
        for (int32_t n : s[ti].bfs)
            if (is_internal(v, s[ti], n)) (*remap)[v->feature[s[ti].base + n]] = 0;
    for (int32_t f = 0; f < v->n_features; f++)
        if ((*remap)[f] == 0) {
            (*remap)[f] = (int32_t)fmap->size();
            fmap->push_back(f);
        }
    if (fmap->empty()) fmap->push_back(0);  // forest of lone leaves: keep one column
}

int bits_for(int64_t n_values) {  // bits to write 0 .. n_values-1 (at least 1)
    int b = 1;
    while ((int64_t)1 << b < n_values) b++;
    return b;
}

int pack_packed(const fp_forest_view* v, const std::vector<TreeShape>& s, const fp_pack_opts* o,
                std::vector<uint8_t>* out, Header* h) {
    const int32_t T = v->n_trees;
    const int32_t B = (o->bin_size <= 0 || o->bin_size > T) ? T : o->bin_size;
    const int32_t D = o->interleave_depth;
    const bool compact = o->layout == FP_LAYOUT_COMPACT;
    const bool align_lines = o->line_align != 0 && !compact;
    const bool stat = o->node_order != FP_ORDER_DF;  // DF-: plain depth-first, left child first
    const int32_t n_bins = (T + B - 1) / B;
    fill_header_common(h, v, s, compact ? FP_LAYOUT_COMPACT : FP_LAYOUT_PACKED);

    // 1) positions of every internal node, bin by bin
    std::vector<std::vector<int32_t>> pos(T);
    std::vector<BinEntry> bins(n_bins);
    int64_t node_cursor = 0;
    int32_t max_top = 0;
    std::vector<int32_t> stack;
    for (int32_t b = 0; b < n_bins; b++) {
        BinEntry& be = bins[b];
        be.first_tree = b * B;
        be.n_trees = std::min(B, T - b * B);
        be.root_base = be.first_tree;
        // bins start on a 128 B line (8 Node16 units, or 16 words of 8 bytes)
        node_cursor = (int64_t)align_up((size_t)node_cursor, compact ? 16 : 8);
        be.node_base = node_cursor;
        int64_t next = 0;
        for (int32_t j = 0; j < be.n_trees; j++) pos[be.first_tree + j].assign(s[be.first_tree + j].size, -1);
        // top region: level-major, tree-minor, breadth-first inside a (depth, tree)
        for (int32_t d = 0; d <= D; d++)
            for (int32_t j = 0; j < be.n_trees; j++) {
                const int32_t ti = be.first_tree + j;
                const TreeShape& t = s[ti];
                for (int32_t n : t.bfs) {
                    if (t.depth[n] > d) break;  // bfs is sorted by depth
                    if (t.depth[n] == d && is_internal(v, t, n)) pos[ti][n] = (int32_t)next++;
                }
            }
        be.top_len = (int32_t)next;
        max_top = std::max(max_top, be.top_len);
        // deep region: per tree, each subtree hanging below depth D in Stat order
        for (int32_t j = 0; j < be.n_trees; j++) {
            const int32_t ti = be.first_tree + j;
            const TreeShape& t = s[ti];
            auto emit_subtree = [&](int32_t root) {
                if (align_lines) next = (int64_t)align_up((size_t)next, 8);
                stack.clear();
                stack.push_back(root);
                while (!stack.empty()) {
                    const int32_t n = stack.back();
                    stack.pop_back();
                    pos[ti][n] = (int32_t)next++;
                    const int64_t g = t.base + n;
                    const int32_t l = v->left[g], r = v->right[g];
                    const bool li = is_internal(v, t, l), ri = is_internal(v, t, r);
                    if (li && ri) {
                        // hot child (more training samples; ties -> left) goes right after
                        // n; without Stat the left child does
                        const bool left_hot = !stat || t.card[l] >= t.card[r];
                        stack.push_back(left_hot ? r : l);
                        stack.push_back(left_hot ? l : r);
                    } else if (li) {
                        stack.push_back(l);
                    } else if (ri) {
                        stack.push_back(r);
                    }
                }
            };
            for (int32_t n : t.bfs) {
                if (t.depth[n] > D) break;
                if (t.depth[n] != D || !is_internal(v, t, n)) continue;
                const int64_t g = t.base + n;
                if (is_internal(v, t, v->left[g])) emit_subtree(v->left[g]);
                if (is_internal(v, t, v->right[g])) emit_subtree(v->right[g]);
            }
        }
        if (next > INT32_MAX)
            return fp_set_error(FP_E2BIG, "bin %d holds %lld nodes (limit %d)", b, (long long)next,
                                INT32_MAX);
        be.deep_len = (int32_t)(next - be.top_len);
        node_cursor += compact ? 2 * (int64_t)be.top_len + be.deep_len : next;
    }
    const int64_t n_nodes = node_cursor;  // Node16 units, or 8-byte words (COMPACT)

    // 2) compacted feature numbering: the columns some split tests, in increasing order
    std::vector<int32_t> remap(v->n_features, -1), fmap;
    for (int32_t ti = 0; ti < T; ti++)
        for (int32_t n : s[ti].bfs)
            if (is_internal(v, s[ti], n)) remap[v->feature[s[ti].base + n]] = 0;
    for (int32_t f = 0; f < v->n_features; f++)
        if (remap[f] == 0) {
            remap[f] = (int32_t)fmap.size();
            fmap.push_back(f);
        }
    if (fmap.empty()) fmap.push_back(0);  // forest of lone leaves: keep one column

    // 3) buffer
    const size_t table_off = sizeof(Header);
    const size_t roots_off = align_up(table_off + sizeof(BinEntry) * (size_t)n_bins, kSectionAlign);
    const size_t fmap_off = align_up(roots_off + sizeof(int32_t) * (size_t)T, kSectionAlign);
    const size_t nodes_off = align_up(fmap_off + sizeof(int32_t) * fmap.size(), kSectionAlign);
    // COMPACT keeps 16 bytes of slack after the last word: a kernel reads every
    // deep node together with its successor in one 16-byte load
    const size_t node_bytes = compact ? 8 * (size_t)n_nodes + 16 : sizeof(Node16) * (size_t)n_nodes;
    const size_t total = align_up(nodes_off + node_bytes, kSectionAlign);
    int fb = 0, cb = 0;
    if (compact) {
        fb = bits_for((int64_t)fmap.size());
        cb = bits_for(v->n_classes);
        const int pb = 29 - fb;
        if (pb < 2 * cb || pb < bits_for(v->n_classes))
            return fp_set_error(FP_E2BIG, "compact layout: %d feature bits and %d classes do not fit a 32-bit node word",
                                fb, v->n_classes);
    }
    try {
        out->assign(total, 0);
    } catch (const std::bad_alloc&) {
        return fp_set_error(FP_ENOMEM, "cannot allocate %zu bytes for the packed forest", total);
    }
    memcpy(out->data() + table_off, bins.data(), sizeof(BinEntry) * (size_t)n_bins);
    memcpy(out->data() + fmap_off, fmap.data(), sizeof(int32_t) * fmap.size());
    int32_t* roots = reinterpret_cast<int32_t*>(out->data() + roots_off);
    Node16* nodes = reinterpret_cast<Node16*>(out->data() + nodes_off);
    Node8* words = reinterpret_cast<Node8*>(out->data() + nodes_off);
    const int pb = 29 - fb;
    for (int32_t b = 0; b < n_bins; b++) {
        const BinEntry& be = bins[b];
        Node16* bn = compact ? reinterpret_cast<Node16*>(words + be.node_base) : nodes + be.node_base;
        Node8* deep = words + be.node_base + 2 * (int64_t)be.top_len;
        for (int32_t j = 0; j < be.n_trees; j++) {
            const int32_t ti = be.first_tree + j;
            const TreeShape& t = s[ti];
            const std::vector<int32_t>& p = pos[ti];
            auto ref = [&](int32_t child) -> int32_t {
                const int64_t g = t.base + child;
                return v->feature[g] >= 0 ? p[child] : -v->leaf_class[g] - 1;
            };
            roots[ti] = ref(0);
            for (int32_t n : t.bfs) {
                if (!is_internal(v, t, n)) continue;
                const int64_t g = t.base + n;
                const int32_t self = p[n];
                if (!compact || self < be.top_len) {
                    Node16& nd = bn[self];
                    nd.thr = v->threshold[g];
                    nd.feat = remap[v->feature[g]];
                    nd.left = ref(v->left[g]);
                    nd.right = ref(v->right[g]);
                    continue;
                }
                // compact deep node: the internal child Stat placed at self + 1
                const int32_t l = v->left[g], r = v->right[g];
                const bool li = is_internal(v, t, l), ri = is_internal(v, t, r);
                uint32_t w = (uint32_t)remap[v->feature[g]];
                uint32_t payload;
                if (li || ri) {
                    const int32_t adj = (li && p[l] == self + 1) ? l : r;
                    const int32_t other = adj == l ? r : l;
                    if (!is_internal(v, t, adj) || p[adj] != self + 1)
                        return fp_set_error(FP_ECORRUPT, "internal error: hot child not adjacent in tree %d", ti);
                    w |= 1u << fb;
                    if (adj == l) w |= 1u << (fb + 1);
                    if (is_internal(v, t, other)) {
                        const int64_t delta = (int64_t)p[other] - self;
                        if (delta < 2 || delta >= ((int64_t)1 << pb))
                            return fp_set_error(FP_E2BIG, "compact layout: subtree distance %lld needs more than %d bits",
                                                (long long)delta, pb);
                        payload = (uint32_t)delta;
                    } else {
                        w |= 1u << (fb + 2);
                        payload = (uint32_t)v->leaf_class[t.base + other];
                    }
                } else {
                    payload = (uint32_t)v->leaf_class[t.base + l] | ((uint32_t)v->leaf_class[t.base + r] << cb);
                }
                w |= payload << (fb + 3);
                deep[self - be.top_len] = Node8{v->threshold[g], w};
            }
        }
    }
    h->bin_size = B;
    h->interleave_depth = D;
    h->n_bins = n_bins;
    h->max_top_len = max_top;
    h->max_bin_trees = B;
    h->line_align = align_lines ? 1 : 0;
    h->n_used_features = (int32_t)fmap.size();
    h->fmap_offset = (int64_t)fmap_off;
    h->compact_fbits = fb;
    h->compact_cbits = cb;
    h->table_offset = (int64_t)table_off;
    h->roots_offset = (int64_t)roots_off;
    h->nodes_offset = (int64_t)nodes_off;
    h->n_nodes = n_nodes;
    finish(out, h);
    return FP_OK;
}


// BLOCKED layout: every internal node lives in a block holding a complete
// three-level subtree (Block48 when a node word fits 19 bits, else Block64);
// there is no Node16 region.
// Each tree's blocks form a tree of their own, built breadth-first; a block's
// child blocks are one contiguous group ordered by training cardinality
// (most samples first, ties in exit order).  Bin interleaving works on
// blocks: the blocks whose root node has depth <= D (block levels
// 0 .. D / 3) of all the bin's trees come first, level-major and tree-minor;
// then each tree's remaining blocks, tree by tree, breadth-first.  Both
// orders keep every child group contiguous and after its parent.
int pack_blocked(const fp_forest_view* v, const std::vector<TreeShape>& s, const fp_pack_opts* o,
                 std::vector<uint8_t>* out, Header* h) {
    const int32_t T = v->n_trees;
    const int32_t B = (o->bin_size <= 0 || o->bin_size > T) ? T : o->bin_size;
    const int32_t D = o->interleave_depth;
    const int32_t n_bins = (T + B - 1) / B;
    const bool clustered = o->layout == FP_LAYOUT_CLUSTERED;
    fill_header_common(h, v, s, o->layout);
    std::vector<int32_t> remap, fmap;
    feature_map(v, s, &remap, &fmap);
    const int fb = bits_for((int64_t)fmap.size());
    const int cb = bits_for(v->n_classes);
    if (!clustered && fb + 2 * (1 + cb) > 32)
        return fp_set_error(FP_E2BIG, "blocked layout: %d feature bits and %d classes do not fit a 32-bit node word",
                            fb, v->n_classes);
    if (clustered && (fb > kClusterFeatBits || v->n_classes > kClusterMaxClasses))
        return fp_set_error(FP_E2BIG, "clustered layout: %zu used features (max %d) or %d classes (max %d)",
                            fmap.size(), 1 << kClusterFeatBits, v->n_classes, kClusterMaxClasses);
    const int32_t last_interleaved_level = D / 3;
    const int P = std::max(cb, 3);
    // 48-byte blocks when a node word fits 19 bits and every bin has fewer
    // than 2^24 blocks (checked below; the packing restarts in 64-byte form)
    bool use48 = !clustered && fb + 2 * (1 + P) <= kBlock48WordBits;
    if (clustered) {  // 48-byte clustered blocks: 9-bit features, thresholds exact in fp16
        use48 = fb <= kCluster48FeatBits;
        for (int64_t i = 0; use48 && i < v->tree_node_offset[T]; i++)
            if (v->feature[i] >= 0) {
                const float t = v->threshold[i];
                use48 = (float)(_Float16)t == t && !std::isnan(t);
            }
    }

    // One tree's blocks in breadth-first order: the subtree root node of each
    // block, its level, and its slots; child blocks are found by bfs index.
    struct Slot {
        bool present = false;
        float thr = 0.0f;
        uint32_t feat = 0;
        uint32_t kind[2] = {0, 0};  // 0 internal, 1 class
        uint32_t pay[2] = {0, 0};   // class, or exit rank of a bottom slot
    };
    struct BlockIR {
        Slot slot[7];
        uint32_t first_child = 0;  // bfs index of the first child block
        uint32_t n_children = 0;
        // CLUSTERED: exits with the outcomes that select them
        uint32_t n_exits = 0;
        uint32_t care[8] = {0}, val[8] = {0}, target[8] = {0};
    };
    struct TreeBlocks {
        std::vector<int32_t> root, level;
        std::vector<BlockIR> body;
    };
    auto build_tree = [&](const TreeShape& t, TreeBlocks* tb) {
        tb->root.assign(1, 0);
        tb->level.assign(1, 0);
        for (size_t q = 0; q < tb->root.size(); q++) {
            int32_t slot_node[7];
            for (int k = 0; k < 7; k++) slot_node[k] = -1;
            slot_node[0] = tb->root[q];
            struct Exit {
                int slot, side;
                int32_t node;
                int64_t card;
            };
            std::vector<Exit> exits;
            BlockIR bk;
            for (int k = 0; k < 7; k++) {
                const int32_t n = slot_node[k];
                if (n < 0) continue;
                const int64_t g = t.base + n;
                const int32_t ch[2] = {v->left[g], v->right[g]};
                Slot& sl = bk.slot[k];
                sl.present = true;
                sl.thr = v->threshold[g];
                sl.feat = (uint32_t)remap[v->feature[g]];
                for (int side = 0; side < 2; side++) {
                    const int64_t gc = t.base + ch[side];
                    if (v->feature[gc] < 0) {
                        sl.kind[side] = 1;
                        sl.pay[side] = (uint32_t)v->leaf_class[gc];
                    } else if (k < 3) {
                        slot_node[2 * k + 1 + side] = ch[side];
                    } else {
                        exits.push_back(Exit{k, side, ch[side], t.card[ch[side]]});
                    }
                }
            }
            std::stable_sort(exits.begin(), exits.end(), [](const Exit& a, const Exit& c) { return a.card > c.card; });
            bk.first_child = (uint32_t)tb->root.size();
            bk.n_children = (uint32_t)exits.size();
            for (size_t r = 0; r < exits.size(); r++) {
                bk.slot[exits[r].slot].pay[exits[r].side] = (uint32_t)r;
                tb->root.push_back(exits[r].node);
                tb->level.push_back(tb->level[q] + 1);
            }
            tb->body.push_back(bk);
        }
    };
    // CLUSTERED: greedy groups of up to 7 nodes, most samples first
    auto build_clusters = [&](const TreeShape& t, TreeBlocks* tb) {
        tb->root.assign(1, 0);
        tb->level.assign(1, 0);
        for (size_t q = 0; q < tb->root.size(); q++) {
            // members in the order they join; parent slot and side of each
            int32_t node[7], par[7], pside[7];
            int m = 0;
            struct Cand {
                int64_t card;
                int32_t node, par, side;
            };
            auto hotter = [](const Cand& a, const Cand& c) {  // max-heap by cardinality, then lower node id
                return a.card != c.card ? a.card < c.card : a.node > c.node;
            };
            std::vector<Cand> front{Cand{t.card[tb->root[q]], tb->root[q], -1, 0}};
            while (!front.empty() && m < 7) {
                std::pop_heap(front.begin(), front.end(), hotter);
                const Cand c = front.back();
                front.pop_back();
                node[m] = c.node;
                par[m] = c.par;
                pside[m] = c.side;
                const int64_t g = t.base + c.node;
                const int32_t ch[2] = {v->left[g], v->right[g]};
                for (int side = 0; side < 2; side++)
                    if (v->feature[t.base + ch[side]] >= 0) {
                        front.push_back(Cand{t.card[ch[side]], ch[side], m, side});
                        std::push_heap(front.begin(), front.end(), hotter);
                    }
                m++;
            }
            BlockIR bk;
            auto path = [&](int slot, uint32_t* care, uint32_t* val) {  // outcomes that lead to slot
                *care = 0;
                *val = 0;
                for (int x = slot; par[x] >= 0; x = par[x]) {
                    *care |= 1u << par[x];
                    *val |= (uint32_t)pside[x] << par[x];
                }
            };
            struct Exit {
                int e;
                int32_t node;
                int64_t card;
            };
            std::vector<Exit> ext;  // exits to child blocks
            for (int k = 0; k < m; k++) {
                const int64_t g = t.base + node[k];
                Slot& sl = bk.slot[k];
                sl.present = true;
                sl.thr = v->threshold[g];
                sl.feat = (uint32_t)remap[v->feature[g]];
                const int32_t ch[2] = {v->left[g], v->right[g]};
                for (int side = 0; side < 2; side++) {
                    bool inside = false;
                    for (int x = 0; x < m; x++) inside |= (par[x] == k && pside[x] == side);
                    if (inside) continue;
                    const int e = (int)bk.n_exits++;
                    uint32_t care, val;
                    path(k, &care, &val);
                    bk.care[e] = care | (1u << k);
                    bk.val[e] = val | ((uint32_t)side << k);
                    const int64_t gc = t.base + ch[side];
                    if (v->feature[gc] < 0) bk.target[e] = (uint32_t)v->leaf_class[gc];
                    else ext.push_back(Exit{e, ch[side], t.card[ch[side]]});
                }
            }
            std::stable_sort(ext.begin(), ext.end(), [](const Exit& a, const Exit& c) { return a.card > c.card; });
            bk.first_child = (uint32_t)tb->root.size();
            bk.n_children = (uint32_t)ext.size();
            for (size_t r = 0; r < ext.size(); r++) {
                bk.target[ext[r].e] = 32u | (uint32_t)r;
                tb->root.push_back(ext[r].node);
                tb->level.push_back(tb->level[q] + 1);
            }
            tb->body.push_back(bk);
        }
    };
    auto encodeC48 = [&](const BlockIR& bk, uint32_t child_base, BlockC48* out) {
        *out = BlockC48{};
        uint32_t r[5] = {0, 0, 0, 0, 0};
        auto put = [&](int pos, int width, uint32_t value) {
            for (int i = 0; i < width; i++)
                if (value >> i & 1u) r[(pos + i) / 32] |= 1u << ((pos + i) % 32);
        };
        for (int k = 0; k < 7; k++) {
            if (!bk.slot[k].present) continue;
            const _Float16 h16 = (_Float16)bk.slot[k].thr;
            memcpy(&out->thr16[k], &h16, 2);
            put(fp::kC48FeatPos[k], kCluster48FeatBits, bk.slot[k].feat);
        }
        for (uint32_t e = 0; e < 8; e++) {
            if (e < bk.n_exits) {
                out->care[e] = (uint8_t)bk.care[e];
                out->val[e] = (uint8_t)bk.val[e];
                put(6 * (int)e, 6, bk.target[e]);
            } else {
                out->care[e] = 0x80;
                out->val[e] = 0x80;
            }
        }
        put(fp::kC48BasePos, fp::kC48BaseBits, bk.n_children ? child_base : 0u);
        put(fp::kC48NChildPos, 4, bk.n_children);
        for (int i = 0; i < 4; i++) out->rest[i] = r[i];
        out->rest_hi = (uint16_t)r[4];
    };
    auto encodeC = [&](const BlockIR& bk, uint32_t child_base, BlockC64* out) {
        *out = BlockC64{};
        auto put = [&](int pos, int width, uint32_t value) {
            for (int i = 0; i < width; i++)
                if (value >> i & 1u) out->rest[(pos + i) / 32] |= 1u << ((pos + i) % 32);
        };
        for (int k = 0; k < 7; k++) {
            if (!bk.slot[k].present) continue;
            out->thr[k] = bk.slot[k].thr;
            put(48 + kClusterFeatBits * k, kClusterFeatBits, bk.slot[k].feat);
        }
        for (uint32_t e = 0; e < 8; e++) {
            if (e < bk.n_exits) {
                out->care[e] = (uint8_t)bk.care[e];
                out->val[e] = (uint8_t)bk.val[e];
                put(6 * (int)e, 6, bk.target[e]);
            } else {
                out->care[e] = 0x80;
                out->val[e] = 0x80;
            }
        }
        put(132, 24, bk.n_children ? child_base : 0u);
        put(156, 4, bk.n_children);
    };
    // encoders: child_base is the final index of the block's first child
    auto encode64 = [&](const BlockIR& bk, uint32_t child_base, Block64* out) {
        *out = Block64{};
        out->child_base = bk.n_children ? child_base : 0u;
        for (int k = 0; k < 7; k++) {
            const Slot& sl = bk.slot[k];
            if (!sl.present) continue;
            uint32_t w = sl.feat;
            for (int side = 0; side < 2; side++) {
                const uint32_t c = sl.kind[side] ? 1u | (sl.pay[side] << 1) : 0u;
                w |= c << (fb + side * (1 + cb));
                if (!sl.kind[side] && k >= 3) out->ranks |= (8u | sl.pay[side]) << (4 * (2 * (k - 3) + side));
            }
            out->slot[k] = Node8{sl.thr, w};
        }
    };
    auto encode48 = [&](const BlockIR& bk, uint32_t child_base, Block48* out) {
        *out = Block48{};
        uint64_t bits[3] = {0, 0, 0};  // 136 bits of words, little-endian
        for (int k = 0; k < 7; k++) {
            const Slot& sl = bk.slot[k];
            if (!sl.present) continue;
            uint64_t w = sl.feat;
            for (int side = 0; side < 2; side++) {
                const uint64_t c = sl.kind[side] ? 1u | (sl.pay[side] << 1) : (uint64_t)sl.pay[side] << 1;
                w |= c << (fb + side * (1 + P));
            }
            const int o = kBlock48WordBits * k;
            bits[o / 64] |= w << (o % 64);
            if (o % 64 + kBlock48WordBits > 64) bits[o / 64 + 1] |= w >> (64 - o % 64);
            out->thr[k] = sl.thr;
        }
        out->words[0] = (uint32_t)bits[0];
        out->words[1] = (uint32_t)(bits[0] >> 32);
        out->words[2] = (uint32_t)bits[1];
        out->words[3] = (uint32_t)(bits[1] >> 32);
        out->words[4] = ((uint32_t)bits[2] & 0xFFu) | ((bk.n_children ? child_base : 0u) << 8);
    };

    std::vector<BinEntry> bins(n_bins);
    std::vector<std::vector<uint8_t>> blocks(n_bins);
    std::vector<int32_t> roots(T, 0);
    int64_t word_cursor = 0;
    double fetch_sum = 0.0;  // per tree: blocks a training-distributed walk fetches
restart:
    const int64_t block_words = use48 ? 6 : 8;  // 8-byte words per block
    word_cursor = 0;
    fetch_sum = 0.0;
    for (int32_t b = 0; b < n_bins; b++) {
        BinEntry& be = bins[b];
        be.first_tree = b * B;
        be.n_trees = std::min(B, T - b * B);
        be.root_base = be.first_tree;
        be.top_len = 0;
        std::vector<TreeBlocks> tb(be.n_trees);
        for (int32_t j = 0; j < be.n_trees; j++) {
            const TreeShape& t = s[be.first_tree + j];
            if (v->feature[t.base] < 0) continue;
            if (clustered) build_clusters(t, &tb[j]);
            else build_tree(t, &tb[j]);
            // a walk fetches block q iff it reaches q's root node
            if (t.card[0] > 0)
                for (int32_t r : tb[j].root) fetch_sum += (double)t.card[r] / (double)t.card[0];
        }
        // final position of every (tree, bfs index)
        std::vector<std::vector<int64_t>> pos(be.n_trees);
        int64_t next = 0;
        for (int32_t j = 0; j < be.n_trees; j++) pos[j].assign(tb[j].root.size(), -1);
        for (int32_t L = 0; L <= last_interleaved_level; L++)
            for (int32_t j = 0; j < be.n_trees; j++)
                for (size_t q = 0; q < tb[j].root.size(); q++)
                    if (tb[j].level[q] == L) pos[j][q] = next++;
        for (int32_t j = 0; j < be.n_trees; j++)
            for (size_t q = 0; q < tb[j].root.size(); q++)
                if (pos[j][q] < 0) pos[j][q] = next++;
        if (next > INT32_MAX) return fp_set_error(FP_E2BIG, "bin %d holds too many blocks", b);
        if (use48 && next > (int64_t)(clustered ? fp::kC48MaxChildBase : kBlock48MaxChildBase)) {
            use48 = false;
            goto restart;
        }
        if (clustered && next > (int64_t)kBlock48MaxChildBase)
            return fp_set_error(FP_E2BIG, "bin %d holds %lld blocks (clustered layout addresses 2^24)", b, (long long)next);
        std::vector<uint8_t>& bl = blocks[b];
        bl.assign((size_t)next * 8 * block_words, 0);
        for (int32_t j = 0; j < be.n_trees; j++) {
            const int32_t ti = be.first_tree + j;
            const TreeShape& t = s[ti];
            if (v->feature[t.base] < 0) {
                roots[ti] = -v->leaf_class[t.base] - 1;
                continue;
            }
            roots[ti] = (int32_t)pos[j][0];
            for (size_t q = 0; q < tb[j].root.size(); q++) {
                const BlockIR& bk = tb[j].body[q];
                const uint32_t child_base = bk.n_children ? (uint32_t)pos[j][bk.first_child] : 0u;
                uint8_t* dst = bl.data() + (size_t)pos[j][q] * 8 * block_words;
                if (clustered && use48) encodeC48(bk, child_base, reinterpret_cast<BlockC48*>(dst));
                else if (clustered) encodeC(bk, child_base, reinterpret_cast<BlockC64*>(dst));
                else if (use48) encode48(bk, child_base, reinterpret_cast<Block48*>(dst));
                else encode64(bk, child_base, reinterpret_cast<Block64*>(dst));
            }
        }
        word_cursor = (int64_t)align_up((size_t)word_cursor, 16);
        be.node_base = word_cursor;
        be.deep_len = (int32_t)next;
        word_cursor += block_words * next;
    }
    const int64_t n_words = word_cursor;
    const size_t table_off = sizeof(Header);
    const size_t roots_off = align_up(table_off + sizeof(BinEntry) * (size_t)n_bins, kSectionAlign);
    const size_t fmap_off = align_up(roots_off + sizeof(int32_t) * (size_t)T, kSectionAlign);
    const size_t nodes_off = align_up(fmap_off + sizeof(int32_t) * fmap.size(), kSectionAlign);
    const size_t total = align_up(nodes_off + 8 * (size_t)n_words, kSectionAlign);
    try {
        out->assign(total, 0);
    } catch (const std::bad_alloc&) {
        return fp_set_error(FP_ENOMEM, "cannot allocate %zu bytes for the packed forest", total);
    }
    memcpy(out->data() + table_off, bins.data(), sizeof(BinEntry) * (size_t)n_bins);
    memcpy(out->data() + roots_off, roots.data(), sizeof(int32_t) * (size_t)T);
    memcpy(out->data() + fmap_off, fmap.data(), sizeof(int32_t) * fmap.size());
    uint8_t* words = out->data() + nodes_off;
    for (int32_t b = 0; b < n_bins; b++)
        if (!blocks[b].empty()) memcpy(words + 8 * bins[b].node_base, blocks[b].data(), blocks[b].size());
    h->bin_size = B;
    h->interleave_depth = D;
    h->n_bins = n_bins;
    h->max_top_len = 0;
    h->max_bin_trees = B;
    h->n_used_features = (int32_t)fmap.size();
    h->fmap_offset = (int64_t)fmap_off;
    h->compact_fbits = fb;
    h->compact_cbits = cb;
    h->block_bytes = use48 ? 48 : 64;
    h->expected_fetches = fetch_sum / (double)T;
    h->table_offset = (int64_t)table_off;
    h->roots_offset = (int64_t)roots_off;
    h->nodes_offset = (int64_t)nodes_off;
    h->n_nodes = n_words;
    finish(out, h);
    return FP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// verification of a packed buffer (used on every buffer built from bytes)
// ---------------------------------------------------------------------------
int verify_buffer(const uint8_t* bytes, size_t n, std::string* why) {
    char buf[256];
#define bad(...) (snprintf(buf, sizeof buf, __VA_ARGS__), *why = buf, FP_ECORRUPT)
    if (n < sizeof(Header)) return bad("buffer of %zu bytes is shorter than the header", n);
    Header h;
    memcpy(&h, bytes, sizeof h);
    if (h.magic != kMagic) return bad("bad magic");
    if (h.version != kFormatVersion) return bad("format version %u, expected %u", h.version, kFormatVersion);
    if (h.total_bytes != (int64_t)n) return bad("size %zu != header size %lld", n, (long long)h.total_bytes);
    // sizes bounded by the buffer first, so that no offset arithmetic below overflows
    if (h.n_trees < 1 || h.n_trees > (int64_t)(n / 4) || h.n_features < 1 || h.n_classes < 1 ||
        h.n_classes > kMaxClasses || h.n_bins < 0 || h.n_bins > h.n_trees || h.n_used_features < 0 ||
        h.n_used_features > (int64_t)(n / 4))
        return bad("bad forest dimensions");
    if (h.n_nodes < 0 || h.n_nodes > (int64_t)n || h.nodes_offset < 0 || h.nodes_offset > (int64_t)n ||
        h.table_offset < 0 || h.table_offset > (int64_t)n || h.roots_offset < 0 || h.roots_offset > (int64_t)n ||
        h.fmap_offset < 0 || h.fmap_offset > (int64_t)n)
        return bad("section offsets or node count beyond the buffer");
    if (fnv1a64(bytes + sizeof(Header), n - sizeof(Header)) != h.checksum) return bad("checksum mismatch");
    const int64_t N = h.n_nodes;
    const int64_t unit = h.layout == FP_LAYOUT_COMPACT || h.layout == FP_LAYOUT_BLOCKED || h.layout == FP_LAYOUT_CLUSTERED
                             ? 8
                             : (int64_t)sizeof(Node16);
    if (N < 0 || h.nodes_offset < (int64_t)sizeof(Header) || h.nodes_offset % 256 ||
        N > ((int64_t)n - h.nodes_offset) / unit)
        return bad("node section out of bounds");
    const Node16* nodes = reinterpret_cast<const Node16*>(bytes + h.nodes_offset);
    const int32_t C = h.n_classes;
    int32_t F = h.n_features;
    // every table starts on a section boundary after the header (the packer
    // writes them so), which also keeps the typed reads below aligned
    auto section_ok = [&](int64_t off) {
        return off >= (int64_t)sizeof(Header) && off % (int64_t)kSectionAlign == 0 && off <= h.nodes_offset;
    };
    if (h.layout == FP_LAYOUT_NAIVE) {
        if (!section_ok(h.table_offset) || h.table_offset + (int64_t)sizeof(int64_t) * (h.n_trees + 1) > h.nodes_offset)
            return bad("tree table out of bounds");
        const int64_t* offs = reinterpret_cast<const int64_t*>(bytes + h.table_offset);
        if (offs[0] != 0 || offs[h.n_trees] != N) return bad("tree table endpoints");
        for (int32_t t = 0; t < h.n_trees; t++) {
            const int64_t lo = offs[t], hi = offs[t + 1];
            if (hi <= lo) return bad("tree %d empty or reversed", t);
            for (int64_t i = lo; i < hi; i++) {
                const Node16& nd = nodes[i];
                const int64_t self = i - lo;
                if (nd.feat < 0) {
                    if (nd.left < 0 || nd.left >= C) return bad("tree %d leaf %lld class", t, (long long)self);
                } else {
                    if (nd.feat >= F) return bad("tree %d node %lld feature", t, (long long)self);
                    if (nd.left <= self || nd.left >= hi - lo || nd.right <= self || nd.right >= hi - lo)
                        return bad("tree %d node %lld child not after it", t, (long long)self);
                }
            }
        }
        return FP_OK;
    }
    if (h.layout != FP_LAYOUT_PACKED && h.layout != FP_LAYOUT_COMPACT && h.layout != FP_LAYOUT_BLOCKED &&
        h.layout != FP_LAYOUT_CLUSTERED)
        return bad("unknown layout %d", h.layout);
    const bool compact = h.layout == FP_LAYOUT_COMPACT;
    const bool clustered = h.layout == FP_LAYOUT_CLUSTERED;
    const bool blocked = h.layout == FP_LAYOUT_BLOCKED || clustered;
    if (h.compact_fbits < 0 || h.compact_fbits > 32 || h.compact_cbits < 0 || h.compact_cbits > 32)
        return bad("field widths");
    if (compact && (h.nodes_offset + 8 * N + 16 > (int64_t)n || h.compact_fbits < 1 || h.compact_fbits > 26 ||
                    h.compact_cbits < 1 || 2 * h.compact_cbits > 29 - h.compact_fbits))
        return bad("compact node section or field widths");
    if (blocked && !clustered &&
        (h.nodes_offset + 8 * N > (int64_t)n || h.compact_fbits < 1 || h.compact_cbits < 1 ||
         h.compact_fbits + 2 * (1 + h.compact_cbits) > 32 || (h.block_bytes != 48 && h.block_bytes != 64) ||
         (h.block_bytes == 48 && h.compact_fbits + 2 * (1 + std::max(h.compact_cbits, 3)) > fp::kBlock48WordBits)))
        return bad("blocked node section or field widths");
    if (clustered && (h.nodes_offset + 8 * N > (int64_t)n || (h.block_bytes != 64 && h.block_bytes != 48) ||
                      h.compact_fbits < 1 || C > fp::kClusterMaxClasses ||
                      h.compact_fbits > (h.block_bytes == 48 ? fp::kCluster48FeatBits : fp::kClusterFeatBits)))
        return bad("clustered node section or field widths");
    const int64_t block_words = h.block_bytes == 48 ? 6 : 8;
    if (!section_ok(h.table_offset) || !section_ok(h.roots_offset) || !section_ok(h.fmap_offset))
        return bad("bin/root/feature tables misplaced");
    if (h.n_bins < 1 || h.table_offset + (int64_t)sizeof(BinEntry) * h.n_bins > h.roots_offset ||
        h.roots_offset + (int64_t)sizeof(int32_t) * h.n_trees > h.fmap_offset ||
        h.n_used_features < 1 || h.n_used_features > h.n_features ||
        h.fmap_offset + (int64_t)sizeof(int32_t) * h.n_used_features > h.nodes_offset)
        return bad("bin/root/feature tables out of bounds");
    const int32_t* fmap = reinterpret_cast<const int32_t*>(bytes + h.fmap_offset);
    for (int32_t j = 0; j < h.n_used_features; j++)
        if (fmap[j] < 0 || fmap[j] >= h.n_features || (j && fmap[j] <= fmap[j - 1]))
            return bad("feature map entry %d", j);
    F = h.n_used_features;  // packed nodes index the compacted feature map
    const BinEntry* bins = reinterpret_cast<const BinEntry*>(bytes + h.table_offset);
    const int32_t* roots = reinterpret_cast<const int32_t*>(bytes + h.roots_offset);
    int32_t tree_cursor = 0;
    int32_t max_top = 0, max_trees = 0;
    for (int32_t b = 0; b < h.n_bins; b++) {
        const BinEntry& be = bins[b];
        if (be.first_tree != tree_cursor || be.n_trees < 1 || be.root_base != be.first_tree)
            return bad("bin %d tree range", b);
        tree_cursor += be.n_trees;
        const int64_t units = compact   ? 2 * (int64_t)be.top_len + be.deep_len
                              : blocked ? block_words * (int64_t)be.deep_len
                                        : (int64_t)be.top_len + be.deep_len;
        if (be.top_len < 0 || be.deep_len < 0 || be.node_base < 0 || be.node_base % (compact || blocked ? 16 : 8) ||
            be.node_base + units > N)
            return bad("bin %d node range", b);
        const int64_t len = (int64_t)be.top_len + be.deep_len;
        max_top = std::max(max_top, be.top_len);
        max_trees = std::max(max_trees, be.n_trees);
        auto ref_ok = [&](int32_t r, int64_t self) { return r < 0 ? (-(int64_t)r - 1) < C : (r > self && r < len); };
        for (int32_t j = 0; j < be.n_trees; j++)
            if (!ref_ok(roots[be.first_tree + j], -1)) return bad("bin %d root %d", b, j);
        if (blocked) {
            if (be.top_len != 0) return bad("bin %d: blocked layout with a top region", b);
            for (int32_t j = 0; j < be.n_trees; j++) {
                const int32_t r = roots[be.first_tree + j];
                if (r < 0 ? (-(int64_t)r - 1) >= C : r >= be.deep_len) return bad("bin %d root %d", b, j);
            }
            const Node8* words = reinterpret_cast<const Node8*>(bytes + h.nodes_offset) + be.node_base;
            const int fb = h.compact_fbits, cb = h.compact_cbits;
            if (clustered) {
                const bool c48 = h.block_bytes == 48;
                const int fw = c48 ? fp::kCluster48FeatBits : fp::kClusterFeatBits;
                const int p_base = c48 ? fp::kC48BasePos : 132, w_base = c48 ? fp::kC48BaseBits : 24;
                const int p_nchild = c48 ? fp::kC48NChildPos : 156;
                for (int64_t k = 0; k < be.deep_len; k++) {
                    const uint8_t* raw = reinterpret_cast<const uint8_t*>(words) + k * h.block_bytes;
                    uint32_t rest[5];
                    float thr[7];
                    const uint8_t *care_b, *val_b;
                    if (c48) {
                        const fp::BlockC48& b48 = *reinterpret_cast<const fp::BlockC48*>(raw);
                        for (int i = 0; i < 4; i++) rest[i] = b48.rest[i];
                        rest[4] = b48.rest_hi;
                        for (int sl = 0; sl < 7; sl++) {
                            _Float16 t16;
                            memcpy(&t16, &b48.thr16[sl], 2);
                            thr[sl] = (float)t16;
                            if (std::isnan(thr[sl])) return bad("bin %d block %lld: NaN threshold", b, (long long)k);
                        }
                        care_b = b48.care;
                        val_b = b48.val;
                    } else {
                        const BlockC64& b64 = *reinterpret_cast<const BlockC64*>(raw);
                        for (int i = 0; i < 5; i++) rest[i] = b64.rest[i];
                        for (int sl = 0; sl < 7; sl++) thr[sl] = b64.thr[sl];
                        care_b = b64.care;
                        val_b = b64.val;
                    }
                    struct View {
                        const float* thr;
                        const uint8_t *care, *val;
                    } bk{thr, care_b, val_b};
                    auto get = [&](int pos, int width) -> uint32_t {
                        uint32_t v = 0;
                        for (int i = 0; i < width; i++) v |= ((rest[(pos + i) / 32] >> ((pos + i) % 32)) & 1u) << i;
                        return v;
                    };
                    if (c48 ? (get(61, 3) | get(91, 5) | (rest[4] >> 16)) != 0 : false)
                        return bad("bin %d block %lld: stray bits", b, (long long)k);
                    const uint32_t n_child = get(p_nchild, 4);
                    const int64_t child_base = get(p_base, w_base);
                    uint32_t n_exit = 0;
                    while (n_exit < 8 && bk.care[n_exit] != 0x80) n_exit++;
                    if (n_exit < 2 || n_child > n_exit)
                        return bad("bin %d block %lld: exit counts", b, (long long)k);
                    if (n_child ? (child_base <= k || child_base + n_child > be.deep_len) : child_base != 0)
                        return bad("bin %d block %lld: child blocks", b, (long long)k);
                    const uint32_t n_slot = n_exit - 1;  // a binary tree of m nodes has m + 1 exits
                    for (uint32_t sl = 0; sl < 7; sl++) {
                        const uint32_t f = get(c48 ? fp::kC48FeatPos[sl] : 48 + fw * (int)sl, fw);
                        if (sl < n_slot ? (int64_t)f >= F : (f != 0 || bk.thr[sl] != 0.0f))
                            return bad("bin %d block %lld slot %u", b, (long long)k, sl);
                    }
                    // used exits: targets in range, and their outcome patterns
                    // partition the 2^n_slot masks (pairwise disjoint, sizes sum)
                    uint32_t child_used = 0;
                    int64_t covered = 0;
                    for (uint32_t e = 0; e < 8; e++) {
                        const uint32_t care = bk.care[e], val = bk.val[e];
                        const uint32_t tgt = get(6 * (int)e, 6);
                        if (e >= n_exit) {
                            if (care != 0x80 || val != 0x80 || tgt)
                                return bad("bin %d block %lld: stray exit %u", b, (long long)k, e);
                            continue;
                        }
                        if ((val & ~care) || (care >> n_slot) || care == 0)
                            return bad("bin %d block %lld exit %u pattern", b, (long long)k, e);
                        if (tgt & 32u) {
                            if ((tgt & 31u) >= n_child) return bad("bin %d block %lld exit %u child", b, (long long)k, e);
                            child_used |= 1u << (tgt & 31u);
                        } else if ((int64_t)tgt >= C) {
                            return bad("bin %d block %lld exit %u class", b, (long long)k, e);
                        }
                        covered += (int64_t)1 << (n_slot - __builtin_popcount(care));
                        for (uint32_t d = 0; d < e; d++)
                            if (((val ^ bk.val[d]) & care & bk.care[d]) == 0)
                                return bad("bin %d block %lld exits %u and %u overlap", b, (long long)k, d, e);
                    }
                    if (covered != ((int64_t)1 << n_slot) || child_used != (n_child ? (1u << n_child) - 1u : 0u))
                        return bad("bin %d block %lld: exits do not cover every outcome once", b, (long long)k);
                }
                continue;
            }
            if (h.block_bytes == 48) {
                const int P = std::max(cb, 3);
                const Block48* blk = reinterpret_cast<const Block48*>(words);
                for (int64_t k = 0; k < be.deep_len; k++) {
                    const Block48& bk = blk[k];
                    const uint64_t lo = (uint64_t)bk.words[0] | (uint64_t)bk.words[1] << 32;
                    const uint64_t mid = (uint64_t)bk.words[2] | (uint64_t)bk.words[3] << 32;
                    const uint64_t hi = bk.words[4] & 0xFFu;
                    auto word_of = [&](int sl) -> uint32_t {
                        const int o = fp::kBlock48WordBits * sl;
                        const uint64_t a = o < 64 ? lo : o < 128 ? mid : hi;
                        const uint64_t c = o < 64 ? mid : hi;
                        uint64_t w = a >> (o % 64);
                        if (o % 64 + fp::kBlock48WordBits > 64) w |= c << (64 - o % 64);
                        return (uint32_t)(w & ((1u << fp::kBlock48WordBits) - 1));
                    };
                    const int64_t child_base = bk.words[4] >> 8;
                    if ((hi >> (7 * fp::kBlock48WordBits - 128)) != 0) return bad("bin %d block %lld: stray bits", b, (long long)k);
                    bool present[7] = {true, false, false, false, false, false, false};
                    int64_t n_exits = 0;
                    for (int sl = 0; sl < 7; sl++) {
                        const uint32_t w = word_of(sl);
                        if (!present[sl]) {
                            if (w != 0 || bk.thr[sl] != 0.0f) return bad("bin %d block %lld: stray slot %d", b, (long long)k, sl);
                            continue;
                        }
                        if ((int64_t)(w & ((1u << fb) - 1)) >= F) return bad("bin %d block %lld slot %d feature", b, (long long)k, sl);
                        if ((w >> (fb + 2 * (1 + P))) != 0) return bad("bin %d block %lld slot %d: stray bits", b, (long long)k, sl);
                        for (int side = 0; side < 2; side++) {
                            const uint32_t c = (w >> (fb + side * (1 + P))) & ((2u << P) - 1);
                            if (c & 1) {
                                if ((int64_t)(c >> 1) >= C) return bad("bin %d block %lld slot %d class", b, (long long)k, sl);
                            } else if (sl < 3) {
                                if (c != 0) return bad("bin %d block %lld slot %d: internal code with payload", b, (long long)k, sl);
                                present[2 * sl + 1 + side] = true;
                            } else {
                                const int64_t rank = c >> 1;
                                if (rank > 7 || child_base + rank <= k || child_base + rank >= be.deep_len)
                                    return bad("bin %d block %lld exit of slot %d", b, (long long)k, sl);
                                n_exits++;
                            }
                        }
                    }
                    if (n_exits == 0 && child_base != 0) return bad("bin %d block %lld: child base without exits", b, (long long)k);
                }
                continue;
            }
            const Block64* blk = reinterpret_cast<const Block64*>(words);
            for (int64_t k = 0; k < be.deep_len; k++) {
                const Block64& bk = blk[k];
                bool present[7] = {true, false, false, false, false, false, false};
                uint32_t used_exits = 0;
                for (int s = 0; s < 7; s++) {
                    const uint32_t w = bk.slot[s].w;
                    if (!present[s]) {
                        if (w != 0 || bk.slot[s].thr != 0.0f) return bad("bin %d block %lld: stray slot %d", b, (long long)k, s);
                        continue;
                    }
                    if ((int64_t)(w & ((1u << fb) - 1)) >= F) return bad("bin %d block %lld slot %d feature", b, (long long)k, s);
                    if (fb + 2 * (1 + cb) < 32 && (w >> (fb + 2 * (1 + cb))) != 0)
                        return bad("bin %d block %lld slot %d: stray bits", b, (long long)k, s);
                    for (int side = 0; side < 2; side++) {
                        const uint32_t c = (w >> (fb + side * (1 + cb))) & ((2u << cb) - 1);
                        if (c & 1) {
                            if ((int64_t)(c >> 1) >= C) return bad("bin %d block %lld slot %d class", b, (long long)k, s);
                        } else if (c != 0) {
                            return bad("bin %d block %lld slot %d: internal code with payload", b, (long long)k, s);
                        } else if (s < 3) {
                            present[2 * s + 1 + side] = true;
                        } else {
                            const int e = 2 * (s - 3) + side;
                            const uint32_t rk = (bk.ranks >> (4 * e)) & 15;
                            const int64_t child = (int64_t)bk.child_base + (rk & 7);
                            if (!(rk & 8) || child <= k || child >= be.deep_len)
                                return bad("bin %d block %lld exit %d", b, (long long)k, e);
                            used_exits |= 1u << e;
                        }
                    }
                }
                for (int e = 0; e < 8; e++)
                    if (!(used_exits >> e & 1) && ((bk.ranks >> (4 * e)) & 15))
                        return bad("bin %d block %lld: rank of unused exit %d", b, (long long)k, e);
            }
            continue;
        }
        if (compact) {
            const Node8* words = reinterpret_cast<const Node8*>(bytes + h.nodes_offset) + be.node_base;
            const Node16* top = reinterpret_cast<const Node16*>(words);
            for (int64_t i = 0; i < be.top_len; i++) {
                const Node16& nd = top[i];
                if (nd.feat < 0 || nd.feat >= F || !ref_ok(nd.left, i) || !ref_ok(nd.right, i))
                    return bad("bin %d top node %lld", b, (long long)i);
            }
            const int fb = h.compact_fbits, cb = h.compact_cbits;
            const Node8* deep = words + 2 * (int64_t)be.top_len;
            for (int64_t i = 0; i < be.deep_len; i++) {
                const uint32_t w = deep[i].w;
                const int64_t self = be.top_len + i;
                const uint32_t pay = w >> (fb + 3);
                if ((int64_t)(w & ((1u << fb) - 1)) >= F) return bad("bin %d deep node %lld feature", b, (long long)i);
                if ((w >> fb) & 1) {
                    if (self + 1 >= len) return bad("bin %d deep node %lld: adjacent child past the bin", b, (long long)i);
                    if ((w >> (fb + 2)) & 1) {
                        if ((int64_t)pay >= C) return bad("bin %d deep node %lld class", b, (long long)i);
                    } else if (pay < 2 || self + (int64_t)pay >= len) {
                        return bad("bin %d deep node %lld distance", b, (long long)i);
                    }
                } else if ((int64_t)(pay & ((1u << cb) - 1)) >= C || (int64_t)(pay >> cb) >= C) {
                    return bad("bin %d deep node %lld leaf classes", b, (long long)i);
                }
            }
            continue;
        }
        const Node16* bn = nodes + be.node_base;
        for (int64_t i = 0; i < len; i++) {
            const Node16& nd = bn[i];
            if (nd.feat < 0 || nd.feat >= F) {
                // padding slots between aligned subtrees are all-zero and unreferenced;
                // a real node must have a valid feature
                if (!(nd.feat == 0 && nd.left == 0 && nd.right == 0)) return bad("bin %d node %lld feature", b, (long long)i);
                continue;
            }
            if (!(nd.feat == 0 && nd.left == 0 && nd.right == 0) && (!ref_ok(nd.left, i) || !ref_ok(nd.right, i)))
                return bad("bin %d node %lld reference", b, (long long)i);
        }
    }
    if (tree_cursor != h.n_trees) return bad("bins cover %d of %d trees", tree_cursor, h.n_trees);
    if (max_top != h.max_top_len || max_trees > h.max_bin_trees) return bad("bin maxima");
    return FP_OK;
#undef bad
}

}  // namespace fp

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int fp_pack_forest(const fp_forest_view* forest, const fp_pack_opts* opts, fp_packed** out) {
    fp_clear_error();
    if (!out) return fp_set_error(FP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!opts) return fp_set_error(FP_EINVAL, "opts is NULL");
    if (opts->layout < FP_LAYOUT_NAIVE || opts->layout > FP_LAYOUT_CLUSTERED)
        return fp_set_error(FP_EINVAL, "unknown layout %d", opts->layout);
    if (opts->layout != FP_LAYOUT_NAIVE && (opts->interleave_depth < 0 || opts->interleave_depth > 30))
        return fp_set_error(FP_EINVAL, "interleave_depth %d outside [0, 30]", opts->interleave_depth);
    if (opts->node_order != FP_ORDER_DEFAULT && opts->node_order != FP_ORDER_DF)
        return fp_set_error(FP_EINVAL, "unknown node_order %d", opts->node_order);
    if (opts->node_order == FP_ORDER_DF && opts->layout != FP_LAYOUT_NAIVE && opts->layout != FP_LAYOUT_PACKED)
        return fp_set_error(FP_EINVAL, "node_order DF needs the NAIVE or PACKED layout");
    try {
        std::vector<fp::TreeShape> shapes;
        int rc = fp::validate_view(forest, &shapes);
        if (rc) return rc;
        std::unique_ptr<fp_packed> p(new fp_packed());
        rc = opts->layout == FP_LAYOUT_NAIVE     ? fp::pack_naive(forest, shapes, opts, &p->bytes, &p->hdr)
             : opts->layout >= FP_LAYOUT_BLOCKED ? fp::pack_blocked(forest, shapes, opts, &p->bytes, &p->hdr)
                                                 : fp::pack_packed(forest, shapes, opts, &p->bytes, &p->hdr);
        if (rc) return rc;
        *out = p.release();
        return FP_OK;
    } catch (const std::bad_alloc&) {
        return fp_set_error(FP_ENOMEM, "out of host memory while packing");
    }
}

extern "C" int fp_packed_info_get(const fp_packed* p, fp_packed_info* out) {
    fp_clear_error();
    if (!p || !out) return fp_set_error(FP_EINVAL, "NULL argument");
    const fp::Header& h = p->hdr;
    memset(out, 0, sizeof *out);
    out->layout = h.layout;
    out->n_trees = h.n_trees;
    out->n_features = h.n_features;
    out->n_classes = h.n_classes;
    out->bin_size = h.bin_size;
    out->interleave_depth = h.interleave_depth;
    out->n_bins = h.n_bins;
    out->max_top_nodes = h.max_top_len;
    out->n_nodes = h.n_nodes;
    out->n_internal = h.n_internal;
    out->n_leaves = h.n_leaves;
    out->bytes = h.total_bytes;
    out->uploaded = p->dev != nullptr;
    out->max_depth = h.max_depth;
    out->n_used_features = h.n_used_features;
    out->expected_depth = h.expected_depth;
    out->mean_bias = h.mean_bias;
    out->expected_fetches = h.expected_fetches;
    return FP_OK;
}

extern "C" int fp_packed_host_bytes(const fp_packed* p, const void** bytes, size_t* nbytes) {
    fp_clear_error();
    if (!p || !bytes || !nbytes) return fp_set_error(FP_EINVAL, "NULL argument");
    *bytes = p->bytes.data();
    *nbytes = p->bytes.size();
    return FP_OK;
}

extern "C" int fp_packed_from_bytes(const void* bytes, size_t nbytes, fp_packed** out) {
    fp_clear_error();
    if (!out) return fp_set_error(FP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!bytes) return fp_set_error(FP_EINVAL, "bytes is NULL");
    std::string why;
    const uint8_t* b = static_cast<const uint8_t*>(bytes);
    if (fp::verify_buffer(b, nbytes, &why)) return fp_set_error(FP_ECORRUPT, "packed buffer: %s", why.c_str());
    try {
        std::unique_ptr<fp_packed> p(new fp_packed());
        p->bytes.assign(b, b + nbytes);
        memcpy(&p->hdr, b, sizeof(fp::Header));
        *out = p.release();
    } catch (const std::bad_alloc&) {
        return fp_set_error(FP_ENOMEM, "out of host memory");
    }
    return FP_OK;
}

extern "C" int fp_packed_save(const fp_packed* p, const char* path) {
    fp_clear_error();
    if (!p || !path) return fp_set_error(FP_EINVAL, "NULL argument");
    FILE* f = fopen(path, "wb");
    if (!f) return fp_set_error(FP_EINVAL, "cannot open %s for writing", path);
    size_t w = fwrite(p->bytes.data(), 1, p->bytes.size(), f);
    int rc = fclose(f);
    if (w != p->bytes.size() || rc != 0) return fp_set_error(FP_EINVAL, "short write to %s", path);
    return FP_OK;
}

extern "C" int fp_packed_load(const char* path, fp_packed** out) {
    fp_clear_error();
    if (!path || !out) return fp_set_error(FP_EINVAL, "NULL argument");
    *out = nullptr;
    FILE* f = fopen(path, "rb");
    if (!f) return fp_set_error(FP_EINVAL, "cannot open %s", path);
    std::vector<uint8_t> buf;
    if (fseek(f, 0, SEEK_END) == 0) {
        long n = ftell(f);
        if (n > 0) {
            buf.resize((size_t)n);
            fseek(f, 0, SEEK_SET);
            if (fread(buf.data(), 1, buf.size(), f) != buf.size()) buf.clear();
        }
    }
    fclose(f);
    if (buf.empty()) return fp_set_error(FP_ECORRUPT, "%s is empty or unreadable", path);
    return fp_packed_from_bytes(buf.data(), buf.size(), out);
}

extern "C" int fp_packed_upload(fp_packed* p, void* dev, size_t cap, void* stream) {
    fp_clear_error();
    if (!p || !dev) return fp_set_error(FP_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(dev) % 256) return fp_set_error(FP_EINVAL, "device buffer not 256-byte aligned");
    if (cap < p->bytes.size())
        return fp_set_error(FP_E2BIG, "device buffer of %zu bytes < packed size %zu", cap, p->bytes.size());
    int dev_id = -1;
    // waits for the copy: the host vector must outlive it
    const int rc = fp::device_upload(dev, p->bytes.data(), p->bytes.size(), stream, &dev_id);
    if (rc) return rc;
    p->dev = dev;
    p->dev_cap = cap;
    p->dev_id = dev_id;
    return FP_OK;
}

extern "C" int fp_infer_cardinality(const fp_forest_view* forest, const float* X_dev, int64_t n_rows, int64_t ld,
                                    int64_t* card_out, void* stream_v) {
    fp_clear_error();
    if (!forest || !card_out) return fp_set_error(FP_EINVAL, "NULL argument");
    if (n_rows < 0 || n_rows > INT32_MAX) return fp_set_error(FP_EINVAL, "n_rows %lld outside [0, 2^31-1]", (long long)n_rows);
    if (n_rows > 0 && !X_dev) return fp_set_error(FP_EINVAL, "X is NULL");
    if (ld < forest->n_features) return fp_set_error(FP_EINVAL, "ld %lld < n_features %d", (long long)ld, forest->n_features);
    try {
        std::vector<fp::TreeShape> shapes;
        int rc = fp::validate_view(forest, &shapes);
        if (rc) return rc;
        // the forest in the breadth-first NAIVE layout (leaves stored), walked on the GPU
        std::vector<uint8_t> bytes;
        fp::Header h;
        const fp_pack_opts opts{FP_LAYOUT_NAIVE, 0, 0, 0, FP_ORDER_DEFAULT};
        rc = fp::pack_naive(forest, shapes, &opts, &bytes, &h);
        if (rc) return rc;
        std::vector<int32_t> counts((size_t)h.n_nodes, 0);
        if (n_rows > 0) {
            rc = fp::device_leaf_counts(bytes.data(), bytes.size(), h, forest->n_trees, X_dev, n_rows, ld,
                                        counts.data(), stream_v);
            if (rc) return rc;
        }
        // leaf counts back to the caller's node ids, summed up to the roots
        const int64_t* offs = reinterpret_cast<const int64_t*>(bytes.data() + h.table_offset);
        for (int32_t ti = 0; ti < forest->n_trees; ti++) {
            const fp::TreeShape& t = shapes[ti];
            std::vector<int64_t> card((size_t)t.size, 0);
            for (size_t k = t.bfs.size(); k-- > 0;) {  // children before parents
                const int32_t n = t.bfs[k];
                const int64_t g = t.base + n;
                card[n] = forest->feature[g] < 0 ? counts[(size_t)(offs[ti] + (int64_t)k)]
                                                 : card[forest->left[g]] + card[forest->right[g]];
            }
            memcpy(card_out + t.base, card.data(), sizeof(int64_t) * card.size());
        }
        return FP_OK;
    } catch (const std::bad_alloc&) {
        return fp_set_error(FP_ENOMEM, "out of host memory");
    }
}

extern "C" void fp_packed_free(fp_packed* p) { delete p; }

extern "C" int fp_packed_set_tune(fp_packed* p, const fp_tune* tune) {
    fp_clear_error();
    if (!p) return fp_set_error(FP_EINVAL, "NULL packed forest");
    if (tune) {
        p->tune = *tune;
        p->has_tune = true;
    } else {
        p->tune = fp_tune{};
        p->has_tune = false;
    }
    return FP_OK;
}

extern "C" int fp_packed_get_tune(const fp_packed* p, fp_tune* out) {
    fp_clear_error();
    if (!p || !out) return fp_set_error(FP_EINVAL, "NULL argument");
    *out = p->tune;
    return FP_OK;
}
