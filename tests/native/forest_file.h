// Reads a forest written by tests/test_sanitizers.py: int32 T, F, C; int64
// offsets[T + 1]; then, over the n = offsets[T] nodes, int32 feature[n],
// float threshold[n], int32 left[n], int32 right[n], int32 leaf_class[n],
// int64 cardinality[n] (little-endian).
#pragma once
#include <cstdio>
#include <cstdint>
#include <vector>

#include "forestpack.h"

struct ForestFile {
    int32_t T = 0, F = 0, C = 0;
    std::vector<int64_t> off, card;
    std::vector<int32_t> feat, left, right, leaf;
    std::vector<float> thr;

    bool read(const char* path) {
        FILE* f = fopen(path, "rb");
        if (!f) return false;
        bool ok = fread(&T, 4, 1, f) == 1 && fread(&F, 4, 1, f) == 1 && fread(&C, 4, 1, f) == 1 && T > 0;
        if (ok) {
            off.resize((size_t)T + 1);
            ok = fread(off.data(), 8, off.size(), f) == off.size();
        }
        const size_t n = ok ? (size_t)off[T] : 0;
        feat.resize(n); thr.resize(n); left.resize(n); right.resize(n); leaf.resize(n); card.resize(n);
        ok = ok && fread(feat.data(), 4, n, f) == n && fread(thr.data(), 4, n, f) == n &&
             fread(left.data(), 4, n, f) == n && fread(right.data(), 4, n, f) == n &&
             fread(leaf.data(), 4, n, f) == n && fread(card.data(), 8, n, f) == n;
        fclose(f);
        return ok;
    }
    fp_forest_view view() const {
        return fp_forest_view{T, F, C, 0, off.data(), feat.data(), thr.data(), left.data(), right.data(), leaf.data(),
                              card.data()};
    }
};
