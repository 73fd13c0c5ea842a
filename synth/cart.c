/*
 * Seeded CART random-forest trainer: the producer of the trained forests that
 * the packing method takes as its input (the method starts from a forest of T
 * trained trees whose internal nodes hold a split and whose leaves hold one
 * class label, Sec. III).  Training itself is not part of Forest Packing; this
 * file only manufactures realistic, reproducible inputs for both the CPU
 * checker and the GPU library, which share nothing else.
 *
 * Algorithm (Breiman random forest, Sec. II): every tree is grown on a
 * bootstrap sample, breadth-first, with Gini splits searched over a random
 * subset of mtry features per node.  Conventions fixed here:
 *   - split test is  x[f] <= t  -> left child, else right child;
 *   - a node id is its creation index; nodes are created breadth-first with the
 *     left child before the right one, so id order is the BF layout of Sec. III-A;
 *   - thresholds are fp32 midpoints a <= t < b between consecutive distinct
 *     training values a < b (rounded midpoint, pulled down to a if it rounds up
 *     to b), so the training partition equals the prediction partition;
 *   - split scores  sum_c L_c^2/n_L + sum_c R_c^2/n_R  (maximising it minimises
 *     weighted Gini) are compared exactly with 128-bit cross-multiplication;
 *     ties keep the earlier candidate (earlier feature in the node's shuffled
 *     order, then the lower threshold);
 *   - the first mtry features of a fresh Fisher-Yates shuffle are searched; when
 *     none of them separates the node, the search continues down the shuffled
 *     list until a feature does;
 *   - a node is a leaf when it is pure, at max_depth, holds fewer than
 *     min_samples_split samples, or no feature separates it; its class is the
 *     majority class, ties to the lowest index;
 *   - cardinality = in-bag sample count with bootstrap multiplicity
 *     (Sec. III-A uses leaf cardinalities collected during training).
 *
 * Random numbers: per tree, a SplitMix64 stream seeds xoshiro256** (Blackman &
 * Vigna, both public domain generators); bounded integers use rejection
 * sampling, so a tree depends only on (seed, tree index), never on threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t n_trees, n_features, n_classes;
    int32_t mtry;              /* features searched per node (>=1) */
    int32_t max_depth;         /* root depth 0; <0 means unlimited */
    int32_t min_samples_split; /* nodes with fewer in-bag samples become leaves (>=2) */
    int32_t bootstrap;         /* 1: n draws with replacement; 0: every row once */
    int32_t n_threads;         /* 0: OpenMP default */
    int32_t tree_offset;       /* index of the first tree: trees [off, off+n_trees) of the seeded forest */
    int32_t reserved;
    uint64_t seed;
} cart_params;

typedef struct {
    int64_t n_nodes, cap;
    int32_t *feature;  /* -1 for a leaf */
    float *threshold;
    int32_t *left, *right; /* tree-local ids, -1 for a leaf */
    int32_t *leaf_class;   /* majority class (defined for every node) */
    int64_t *cardinality;
    int32_t *depth;
    int64_t *lo, *hi; /* sample range during growth */
} cart_tree;

typedef struct {
    int32_t n_trees, n_features, n_classes;
    cart_tree *trees;
} cart_forest;

/* ---------------- random numbers ---------------- */
static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
typedef struct { uint64_t s[4]; } xoshiro;
static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static inline uint64_t xo_next(xoshiro *r) {
    uint64_t *s = r->s;
    uint64_t result = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return result;
}
static void xo_seed(xoshiro *r, uint64_t forest_seed, uint64_t tree) {
    uint64_t x = forest_seed ^ (0xD1B54A32D192ED03ULL * (tree + 1));
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64(&x);
}
/* uniform integer in [0, n), n >= 1, by rejection of the biased low range */
static inline uint64_t xo_bounded(xoshiro *r, uint64_t n) {
    uint64_t lim = (0 - n) % n; /* 2^64 mod n */
    uint64_t v;
    do { v = xo_next(r); } while (v < lim);
    return v % n;
}

/* ---------------- sorting ---------------- */
static inline uint32_t fkey(float v) {
    uint32_t u; memcpy(&u, &v, 4);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
static inline float key_to_float(uint32_t k) {
    uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    float v; memcpy(&v, &u, 4); return v;
}
/* 64-bit items ordered by their high 32 bits (stable LSD radix, 8-bit digits) */
static void sort_hi32(uint64_t *a, uint64_t *tmp, int64_t m) {
    uint64_t *src = a, *dst = tmp;
    for (int pass = 0; pass < 4; pass++) {
        int sh = 32 + 8 * pass;
        int64_t cnt[257];
        memset(cnt, 0, sizeof cnt);
        for (int64_t i = 0; i < m; i++) cnt[((src[i] >> sh) & 255) + 1]++;
        int skip = 0;
        for (int b = 0; b < 256; b++) if (cnt[b + 1] == m) skip = 1;
        if (skip) continue;
        for (int b = 0; b < 256; b++) cnt[b + 1] += cnt[b];
        for (int64_t i = 0; i < m; i++) dst[cnt[(src[i] >> sh) & 255]++] = src[i];
        uint64_t *t = src; src = dst; dst = t;
    }
    if (src != a) memcpy(a, src, (size_t)m * sizeof(uint64_t));
}

/*
 * Split keys.  Every training value of feature f is replaced once per
 * forest by its dense rank among the column's distinct fp32 bit patterns in
 * ascending order of value (-0 ranks just below +0), and key = rank << 8 |
 * class.  Ranks order as the values do, so sorting a node's keys by rank
 * orders its samples by value; vals[f][r] is the value of rank r.  A
 * boundary between neighbours of ranks ra < rb is a candidate when
 * vals[ra] < vals[rb], which rules out only -0 | +0 (ra = zneg[f], rb = ra + 1).
 */
typedef struct {
    uint32_t *key;   /* [F][n] */
    uint32_t *zneg;  /* [F]: rank of -0 when +0 follows it in the column, else UINT32_MAX */
    float *vals;     /* [F][n]: the column's distinct values, ascending, in the first ranks */
} cart_ranks;

static int ranks_build(const float *Xt, int64_t n, const int32_t *y, int32_t F, int nt, cart_ranks *rk) {
    rk->key = (uint32_t *)malloc((size_t)F * (size_t)n * sizeof(uint32_t));
    rk->vals = (float *)malloc((size_t)F * (size_t)n * sizeof(float));
    rk->zneg = (uint32_t *)malloc((size_t)F * sizeof(uint32_t));
    if (!rk->key || !rk->vals || !rk->zneg) return -1;
    int failed = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt) reduction(| : failed)
#endif
    for (int32_t f = 0; f < F; f++) {
        uint64_t *it = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
        uint64_t *tmp = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
        if (!it || !tmp) { free(it); free(tmp); failed = 1; continue; }
        const float *col = Xt + (size_t)f * (size_t)n;
        for (int64_t i = 0; i < n; i++) it[i] = ((uint64_t)fkey(col[i]) << 32) | (uint64_t)i;
        sort_hi32(it, tmp, n);
        uint32_t *key = rk->key + (size_t)f * (size_t)n;
        float *vals = rk->vals + (size_t)f * (size_t)n;
        uint32_t r = 0;
        rk->zneg[f] = UINT32_MAX;
        for (int64_t k = 0; k < n; k++) {
            const uint32_t fk = (uint32_t)(it[k] >> 32);
            if (k == 0) vals[0] = key_to_float(fk);
            else if (fk != (uint32_t)(it[k - 1] >> 32)) {
                vals[++r] = key_to_float(fk);
                if (fk == 0x80000000u && (uint32_t)(it[k - 1] >> 32) == 0x7FFFFFFFu) rk->zneg[f] = r - 1;
            }
            const int64_t i = (int64_t)(it[k] & 0xFFFFFFFFu);
            key[i] = (r << 8) | (uint32_t)y[i];
        }
        free(it); free(tmp);
    }
    (void)nt;
    return failed ? -1 : 0;
}

/* Orders m keys by rank (key >> 8), given every rank lies in [lo, lo + 2^bits):
 * insertion sort for short runs, else LSD radix over the rank offset. */
static void sort_keys(uint32_t *a, uint32_t *tmp, int64_t m, uint32_t lo, int bits) {
    if (m <= 64) {
        for (int64_t i = 1; i < m; i++) {
            uint32_t v = a[i]; int64_t j = i - 1;
            while (j >= 0 && (a[j] >> 8) > (v >> 8)) { a[j + 1] = a[j]; j--; }
            a[j + 1] = v;
        }
        return;
    }
    const int d = m < 4096 ? 8 : 11;
    const uint32_t mask = (1u << d) - 1u;
    uint32_t cnt[(1 << 11) + 1];
    uint32_t *src = a, *dst = tmp;
    for (int sh = 0; sh < bits; sh += d) {
        memset(cnt, 0, sizeof(uint32_t) * (mask + 2));
        for (int64_t i = 0; i < m; i++) cnt[((((src[i] >> 8) - lo) >> sh) & mask) + 1]++;
        for (uint32_t b = 0; b <= mask; b++) cnt[b + 1] += cnt[b];
        for (int64_t i = 0; i < m; i++) dst[cnt[(((src[i] >> 8) - lo) >> sh) & mask]++] = src[i];
        uint32_t *t = src; src = dst; dst = t;
    }
    if (src != a) memcpy(a, src, (size_t)m * sizeof(uint32_t));
}

/* score comparison: is (numA/denA) > (numB/denB) ?  all non-negative */
static inline int score_greater(uint64_t numA, uint64_t denA, uint64_t numB, uint64_t denB) {
    unsigned __int128 l = (unsigned __int128)numA * denB;
    unsigned __int128 r = (unsigned __int128)numB * denA;
    return l > r;
}

typedef struct {
    int found;
    int32_t feature;
    float threshold;
    uint64_t num, den; /* score = num/den */
} split_t;

/* Best split of one feature over the node's samples; returns 1 if any. */
static int best_split_feature(const uint32_t *key, const float *vals, uint32_t zneg, const int32_t *idx, int64_t m,
                              int32_t C, const int64_t *tot, uint32_t *items, uint32_t *tmp,
                              int64_t *L, split_t *out) {
    uint32_t lo = UINT32_MAX, hi = 0;
    for (int64_t i = 0; i < m; i++) {
        const uint32_t k = key[idx[i]];
        items[i] = k;
        const uint32_t r = k >> 8;
        lo = r < lo ? r : lo;
        hi = r > hi ? r : hi;
    }
    if (lo == hi) return 0;
    int bits = 0;
    while (bits < 32 && ((hi - lo) >> bits)) bits++;
    sort_keys(items, tmp, m, lo, bits);
    memset(L, 0, sizeof(int64_t) * (size_t)C);
    uint64_t A = 0; /* sum L_c^2 */
    uint64_t B = 0; /* sum R_c^2 */
    for (int c = 0; c < C; c++) B += (uint64_t)tot[c] * (uint64_t)tot[c];
    int any = 0;
    for (int64_t i = 0; i + 1 < m; i++) {
        const uint32_t c = items[i] & 0xFFu;
        const int64_t Rc = tot[c] - L[c];
        A += 2 * (uint64_t)L[c] + 1;
        B -= 2 * (uint64_t)Rc - 1;
        L[c]++;
        const uint32_t ra = items[i] >> 8, rb = items[i + 1] >> 8;
        if (ra == rb || (ra == zneg && rb == zneg + 1)) continue; /* equal values, or -0 | +0 */
        uint64_t nL = (uint64_t)(i + 1), nR = (uint64_t)(m - i - 1);
        uint64_t num = A * nR + B * nL, den = nL * nR;
        if (!any || score_greater(num, den, out->num, out->den)) {
            const float a = vals[ra], b = vals[rb];
            float t = (float)(((double)a + (double)b) * 0.5);
            if (t >= b) t = a;
            out->num = num; out->den = den; out->threshold = t;
            any = 1;
        }
    }
    return any;
}

static int tree_grow_cap(cart_tree *t, int64_t need) {
    if (need <= t->cap) return 0;
    int64_t nc = t->cap ? t->cap * 2 : 1024;
    while (nc < need) nc *= 2;
#define GROW(p, T) do { void *q = realloc(t->p, (size_t)nc * sizeof(T)); if (!q) return -1; t->p = (T *)q; } while (0)
    GROW(feature, int32_t); GROW(threshold, float); GROW(left, int32_t); GROW(right, int32_t);
    GROW(leaf_class, int32_t); GROW(cardinality, int64_t); GROW(depth, int32_t);
    GROW(lo, int64_t); GROW(hi, int64_t);
#undef GROW
    t->cap = nc;
    return 0;
}

/* A node is a multiset of samples: the order of idx inside a node changes
 * nothing the tree depends on.  It is kept ascending (a counting sort of the
 * bootstrap draws, then stable partitions), so that the per-node gathers
 * walk the columns forwards. */
static int train_tree(const float *Xt, const cart_ranks *rk, int64_t n, const int32_t *y, const cart_params *p,
                      int64_t tree_index, cart_tree *t) {
    const int32_t F = p->n_features, C = p->n_classes;
    xoshiro rng; xo_seed(&rng, p->seed, (uint64_t)tree_index);
    int32_t *idx = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *side = (int32_t *)malloc((size_t)n * sizeof(int32_t)); /* draw counts, then partition scratch */
    uint32_t *items = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    uint32_t *tmp = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    int32_t *perm = (int32_t *)malloc((size_t)F * sizeof(int32_t));
    int64_t *tot = (int64_t *)malloc((size_t)C * sizeof(int64_t));
    int64_t *L = (int64_t *)malloc((size_t)C * sizeof(int64_t));
    int rc = 0;
    if (!idx || !side || !items || !tmp || !perm || !tot || !L) { rc = -1; goto done; }
    if (p->bootstrap) {
        memset(side, 0, (size_t)n * sizeof(int32_t));
        for (int64_t i = 0; i < n; i++) side[xo_bounded(&rng, (uint64_t)n)]++;
        int64_t k = 0;
        for (int64_t i = 0; i < n; i++)
            for (int32_t c = 0; c < side[i]; c++) idx[k++] = (int32_t)i;
    } else {
        for (int64_t i = 0; i < n; i++) idx[i] = (int32_t)i;
    }

    memset(t, 0, sizeof *t);
    if (tree_grow_cap(t, 1)) { rc = -1; goto done; }
    t->n_nodes = 1; t->lo[0] = 0; t->hi[0] = n; t->depth[0] = 0;
    for (int64_t q = 0; q < t->n_nodes; q++) {
        int64_t lo = t->lo[q], hi = t->hi[q], m = hi - lo;
        memset(tot, 0, sizeof(int64_t) * (size_t)C);
        for (int64_t i = lo; i < hi; i++) tot[y[idx[i]]]++;
        int32_t maj = 0; int n_nonzero = 0;
        for (int c = 0; c < C; c++) { if (tot[c] > tot[maj]) maj = c; if (tot[c]) n_nonzero++; }
        t->leaf_class[q] = maj; t->cardinality[q] = m;
        t->feature[q] = -1; t->threshold[q] = 0.0f; t->left[q] = -1; t->right[q] = -1;
        if (n_nonzero <= 1 || m < p->min_samples_split ||
            (p->max_depth >= 0 && t->depth[q] >= p->max_depth))
            continue;
        for (int32_t f = 0; f < F; f++) perm[f] = f;
        for (int32_t i = F - 1; i > 0; i--) {
            int32_t j = (int32_t)xo_bounded(&rng, (uint64_t)i + 1);
            int32_t s = perm[i]; perm[i] = perm[j]; perm[j] = s;
        }
        split_t best; memset(&best, 0, sizeof best);
        for (int32_t k = 0; k < F; k++) {
            if (k >= p->mtry && best.found) break;
            int32_t f = perm[k];
            split_t cand; memset(&cand, 0, sizeof cand);
            if (!best_split_feature(rk->key + (size_t)f * (size_t)n, rk->vals + (size_t)f * (size_t)n, rk->zneg[f], idx + lo, m,
                                    C, tot, items, tmp, L, &cand))
                continue;
            if (!best.found || score_greater(cand.num, cand.den, best.num, best.den)) {
                best = cand; best.found = 1; best.feature = f;
            }
        }
        if (!best.found) continue;
        /* stable partition of idx[lo,hi) by x[f] <= thr */
        const float *col = Xt + (size_t)best.feature * (size_t)n;
        int64_t nl = 0, nr = 0;
        for (int64_t i = lo; i < hi; i++) {
            const int32_t s = idx[i];
            if (col[s] <= best.threshold) idx[lo + nl++] = s;
            else side[nr++] = s;
        }
        memcpy(idx + lo + nl, side, (size_t)nr * sizeof(int32_t));
        int64_t mid = lo + nl;
        if (tree_grow_cap(t, t->n_nodes + 2)) { rc = -1; goto done; }
        int64_t l = t->n_nodes, r = l + 1;
        t->n_nodes += 2;
        t->feature[q] = best.feature; t->threshold[q] = best.threshold;
        t->left[q] = (int32_t)l; t->right[q] = (int32_t)r;
        t->lo[l] = lo; t->hi[l] = mid; t->depth[l] = t->depth[q] + 1;
        t->lo[r] = mid; t->hi[r] = hi; t->depth[r] = t->depth[q] + 1;
    }
done:
    free(idx); free(side); free(items); free(tmp); free(perm); free(tot); free(L);
    return rc;
}

static void tree_free(cart_tree *t) {
    free(t->feature); free(t->threshold); free(t->left); free(t->right);
    free(t->leaf_class); free(t->cardinality); free(t->depth); free(t->lo); free(t->hi);
}

void cart_free(cart_forest *f) {
    if (!f) return;
    if (f->trees) for (int32_t i = 0; i < f->n_trees; i++) tree_free(&f->trees[i]);
    free(f->trees);
    free(f);
}

/* Training data prepared once for any number of cart_train_prepared calls
 * (a forest trained chunk by chunk): the feature-major copy and the split
 * keys.  The labels stay the caller's (borrowed until cart_data_free). */
typedef struct {
    int64_t n;
    int32_t F, C;
    float *Xt;
    const int32_t *y;
    cart_ranks rk;
} cart_data;

void cart_data_free(cart_data *d) {
    if (!d) return;
    free(d->Xt); free(d->rk.key); free(d->rk.zneg); free(d->rk.vals);
    free(d);
}

/* Returns 0, -1 on allocation failure, -2 on invalid arguments (including
 * NaN training values, labels outside [0, n_classes) and more than 256
 * classes). */
int cart_data_create(const float *X, int64_t n, int64_t ld, int32_t n_features, const int32_t *y,
                     int32_t n_classes, int32_t n_threads, cart_data **out) {
    *out = NULL;
    /* n <= 4e6 keeps the exact split score (at most n^3/4) inside 64 bits */
    if (!X || !y || n < 1 || n > 4000000LL || n_features < 1 || ld < n_features || n_classes < 1 ||
        n_classes > 256)
        return -2;
    for (int64_t i = 0; i < n; i++) if (y[i] < 0 || y[i] >= n_classes) return -2;
    const int32_t F = n_features;
    cart_data *d = (cart_data *)calloc(1, sizeof *d);
    if (!d) return -1;
    d->n = n; d->F = F; d->C = n_classes; d->y = y;
    /* feature-major copy so that per-node gathers stay within one column */
    d->Xt = (float *)malloc((size_t)n * (size_t)F * sizeof(float));
    if (!d->Xt) { cart_data_free(d); return -1; }
    int nan_seen = 0;
    for (int64_t i = 0; i < n; i++)
        for (int32_t f = 0; f < F; f++) {
            const float v = X[(size_t)i * (size_t)ld + f];
            nan_seen |= v != v;
            d->Xt[(size_t)f * (size_t)n + (size_t)i] = v;
        }
    if (nan_seen) { cart_data_free(d); return -2; }
#ifdef _OPENMP
    int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    int nt = 1;
    (void)n_threads;
#endif
    if (ranks_build(d->Xt, n, y, F, nt, &d->rk)) { cart_data_free(d); return -1; }
    *out = d;
    return 0;
}

/* Trees [tree_offset, tree_offset + n_trees) of the seeded forest on
 * prepared data.  Returns 0, -1 on allocation failure, -2 on invalid
 * arguments. */
int cart_train_prepared(const cart_data *d, const cart_params *p, cart_forest **out) {
    *out = NULL;
    if (!d || !p || p->n_trees < 1 || p->n_features != d->F || p->n_classes != d->C || p->mtry < 1 ||
        p->min_samples_split < 2)
        return -2;
#ifdef _OPENMP
    int nt = p->n_threads > 0 ? p->n_threads : omp_get_max_threads();
#endif
    cart_forest *fo = (cart_forest *)calloc(1, sizeof *fo);
    if (fo) fo->trees = (cart_tree *)calloc((size_t)p->n_trees, sizeof(cart_tree));
    if (!fo || !fo->trees) { free(fo); return -1; }
    fo->n_trees = p->n_trees; fo->n_features = d->F; fo->n_classes = p->n_classes;
    int failed = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt) reduction(| : failed)
#endif
    for (int32_t t = 0; t < p->n_trees; t++)
        if (train_tree(d->Xt, &d->rk, d->n, d->y, p, (int64_t)p->tree_offset + t, &fo->trees[t])) failed = 1;
    if (failed) { cart_free(fo); return -1; }
    *out = fo;
    return 0;
}

/* Prepare and train in one call.  Returns as cart_data_create /
 * cart_train_prepared. */
int cart_train(const float *X, int64_t n, int64_t ld, const int32_t *y, const cart_params *p,
               cart_forest **out) {
    *out = NULL;
    if (!p) return -2;
    cart_data *d = NULL;
    int rc = cart_data_create(X, n, ld, p->n_features, y, p->n_classes, p->n_threads, &d);
    if (rc) return rc;
    rc = cart_train_prepared(d, p, out);
    cart_data_free(d);
    return rc;
}

int64_t cart_total_nodes(const cart_forest *f) {
    int64_t s = 0;
    for (int32_t i = 0; i < f->n_trees; i++) s += f->trees[i].n_nodes;
    return s;
}

/* Concatenated structure-of-arrays export; ids stay tree-local. */
void cart_export(const cart_forest *f, int64_t *tree_node_offset, int32_t *feature, float *threshold,
                 int32_t *left, int32_t *right, int32_t *leaf_class, int64_t *cardinality,
                 int32_t *depth) {
    int64_t off = 0;
    for (int32_t i = 0; i < f->n_trees; i++) {
        const cart_tree *t = &f->trees[i];
        size_t k = (size_t)t->n_nodes;
        tree_node_offset[i] = off;
        memcpy(feature + off, t->feature, k * 4);
        memcpy(threshold + off, t->threshold, k * 4);
        memcpy(left + off, t->left, k * 4);
        memcpy(right + off, t->right, k * 4);
        memcpy(leaf_class + off, t->leaf_class, k * 4);
        memcpy(cardinality + off, t->cardinality, k * 8);
        memcpy(depth + off, t->depth, k * 4);
        off += t->n_nodes;
    }
    tree_node_offset[f->n_trees] = off;
}
