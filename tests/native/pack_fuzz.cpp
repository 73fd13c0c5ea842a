// Packer under AddressSanitizer and UndefinedBehaviorSanitizer (host only).
//
// For the forest in argv[1]: every layout and several (bin size, interleave
// depth) pairs are packed, verified, rebuilt from their bytes and saved and
// loaded again; then every packed buffer is mutated many times (random bytes
// of the header, bin table, roots, feature map and node section, with the
// checksum recomputed so that the reference checks run, and truncations) and
// handed to fp_packed_from_bytes, which must refuse or accept it without a
// single out-of-bounds access.  Malformed forest views (cycles, shared
// children, out-of-range features, children and classes) must be refused.
// Prints a summary line; exits 1 on a wrong status, the sanitizers abort on
// memory or undefined-behaviour errors.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "forest_file.h"
#include "fp_internal.h"

static int fail(const char* what) {
    fprintf(stderr, "pack_fuzz: %s: %s\n", what, fp_last_error());
    return 1;
}

int main(int argc, char** argv) {
    if (argc < 3) {
        fprintf(stderr, "usage: pack_fuzz forest.bin tmpdir [mutations]\n");
        return 2;
    }
    ForestFile ff;
    if (!ff.read(argv[1])) return fail("reading the forest file");
    const int mutations = argc > 3 ? atoi(argv[3]) : 300;
    const fp_forest_view v = ff.view();
    std::mt19937_64 rng(12345);
    int packed = 0, refused = 0, accepted = 0;
    struct Opt {
        int layout, B, D, align, order;
    };
    const std::vector<Opt> opts = {
        {FP_LAYOUT_NAIVE, 0, 0, 0, FP_ORDER_DEFAULT},    {FP_LAYOUT_NAIVE, 0, 0, 0, FP_ORDER_DF},
        {FP_LAYOUT_PACKED, 1, 0, 0, FP_ORDER_DEFAULT},   {FP_LAYOUT_PACKED, 4, 3, 1, FP_ORDER_DEFAULT},
        {FP_LAYOUT_PACKED, 16, 6, 0, FP_ORDER_DF},       {FP_LAYOUT_COMPACT, 3, 2, 0, FP_ORDER_DEFAULT},
        {FP_LAYOUT_BLOCKED, 5, 3, 0, FP_ORDER_DEFAULT},  {FP_LAYOUT_BLOCKED, 64, 0, 0, FP_ORDER_DEFAULT},
        {FP_LAYOUT_CLUSTERED, 4, 3, 0, FP_ORDER_DEFAULT}, {FP_LAYOUT_CLUSTERED, 1, 6, 0, FP_ORDER_DEFAULT},
    };
    const std::string tmp = std::string(argv[2]) + "/fuzz.fpk";
    for (const Opt& o : opts) {
        fp_pack_opts po{o.layout, o.B, o.D, o.align, o.order};
        fp_packed* p = nullptr;
        int rc = fp_pack_forest(&v, &po, &p);
        if (rc == FP_E2BIG) continue;  // the layout's encoding does not hold this forest
        if (rc) return fail("fp_pack_forest");
        packed++;
        const void* bytes = nullptr;
        size_t n = 0;
        if (fp_packed_host_bytes(p, &bytes, &n)) return fail("fp_packed_host_bytes");
        fp_packed_info info;
        if (fp_packed_info_get(p, &info) || (size_t)info.bytes != n) return fail("fp_packed_info_get");
        fp_packed* q = nullptr;
        if (fp_packed_from_bytes(bytes, n, &q)) return fail("fp_packed_from_bytes of a good buffer");
        fp_packed_free(q);
        if (fp_packed_save(p, tmp.c_str()) || fp_packed_load(tmp.c_str(), &q)) return fail("save / load");
        fp_packed_free(q);
        std::vector<uint8_t> good(static_cast<const uint8_t*>(bytes), static_cast<const uint8_t*>(bytes) + n);
        fp::Header h;
        memcpy(&h, good.data(), sizeof h);
        const size_t body = (size_t)h.nodes_offset;
        for (int m = 0; m < mutations; m++) {
            std::vector<uint8_t> bad = good;
            const int kind = (int)(rng() % 4);
            if (kind == 0) {  // a truncated buffer
                bad.resize(rng() % n);
            } else {
                // 1: header fields, 2: tables (bins, roots, feature map), 3: nodes
                const size_t lo = kind == 1 ? 8 : kind == 2 ? sizeof(fp::Header) : body;
                const size_t hi = kind == 1 ? sizeof(fp::Header) : kind == 2 ? body : n;
                if (hi <= lo) continue;
                const int flips = 1 + (int)(rng() % 4);
                for (int k = 0; k < flips; k++) bad[lo + rng() % (hi - lo)] ^= (uint8_t)(1u << (rng() % 8));
                if (bad.size() >= sizeof(fp::Header)) {  // a consistent checksum, so the reference checks run
                    fp::Header hb;
                    memcpy(&hb, bad.data(), sizeof hb);
                    if (hb.total_bytes == (int64_t)bad.size()) {
                        hb.checksum = fp::fnv1a64(bad.data() + sizeof hb, bad.size() - sizeof hb);
                        memcpy(bad.data(), &hb, sizeof hb);
                    }
                }
            }
            fp_packed* r = nullptr;
            if (fp_packed_from_bytes(bad.data(), bad.size(), &r) == FP_OK) {
                accepted++;  // a flip that keeps the buffer well formed (a threshold, say)
                fp_packed_free(r);
            } else {
                refused++;
            }
        }
        fp_packed_free(p);
    }
    // malformed views must be refused with FP_ECORRUPT
    int bad_views = 0;
    for (int k = 0; k < 6; k++) {
        ForestFile g = ff;
        const int64_t t0 = g.off[0], t1 = g.off[1];
        int64_t inner = -1;
        for (int64_t i = t0; i < t1; i++)
            if (g.feat[i] >= 0) inner = i;
        if (inner < 0) break;
        switch (k) {
            case 0: g.left[inner] = 0; break;                                  // a cycle back to the root
            case 1: g.right[inner] = g.left[inner]; break;                     // a shared child
            case 2: g.feat[inner] = g.F; break;                                // feature out of range
            case 3: g.left[inner] = (int32_t)(t1 - t0); break;                 // child outside the tree
            case 4: for (int64_t i = t0; i < t1; i++) if (g.feat[i] < 0) g.leaf[i] = g.C; break;  // class
            case 5: g.off[1] = g.off[0] - 1; break;                            // decreasing offsets
        }
        fp_forest_view gv = g.view();
        fp_pack_opts po{FP_LAYOUT_PACKED, 4, 2, 0, FP_ORDER_DEFAULT};
        fp_packed* p = nullptr;
        const int rc = fp_pack_forest(&gv, &po, &p);
        if (rc == FP_OK) {
            fprintf(stderr, "pack_fuzz: malformed view %d was accepted\n", k);
            return 1;
        }
        bad_views++;
    }
    printf("pack_fuzz: %d packings, %d mutated buffers refused, %d accepted, %d malformed views refused\n", packed,
           refused, accepted, bad_views);
    return packed > 0 && refused > 0 ? 0 : 1;
}
