/*
 * forestpack -- packed decision-forest classification on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libforestpack.so.  Plain pointers and sizes only.
 *
 * What is computed (Forest Packing, Browne et al., arXiv 1806.07300):
 *   A trained forest of T decision trees (Sec. III) classifies an observation
 *   x in R^F: in every tree the observation walks from the root to a leaf,
 *   going to the left child when x[feature] <= threshold (fp32 compare, NaN
 *   goes right), and the leaf's single class label (Sec. III) gets one vote.
 *   votes[c] counts the trees voting c; the class is argmax_c votes[c] with
 *   ties resolved to the lowest class index.  Packing (Sec. III-A) changes the
 *   memory layout and evaluation order only, never the result (Sec. III-A,
 *   cost model discussion), so every layout and every launch configuration
 *   returns bit-identical int32 votes.
 *
 * Conventions shared by all calls:
 *   - Every call returns an int status (FP_OK = 0 or an FP_E* code); on error
 *     fp_last_error() returns a message (thread-local, valid until the next
 *     call on the same thread).  No C++ exception crosses this boundary.
 *   - Objects (fp_packed, fp_plan, fp_server) are opaque, library-owned, and
 *     released by their *_free / *_destroy call.  They are not thread-safe,
 *     except fp_server whose submit/poll may be called from any thread.
 *   - Caller arrays are borrowed for the duration of the call, except where a
 *     call says otherwise (device buffers given to fp_packed_upload and
 *     fp_plan_create; the output buffer of fp_serve_submit).
 *   - "device" pointers are HIP device memory of the current device (for
 *     example torch tensors' data_ptr()); "host" pointers are CPU memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls taking a stream are asynchronous with respect to the host and
 *     do not synchronise the device.
 */
#ifndef FORESTPACK_H
#define FORESTPACK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------------ */
/* Status codes                                                              */
/* ------------------------------------------------------------------------ */
enum {
    FP_OK = 0,
    FP_EINVAL = 1,     /* invalid argument (null pointer, bad size, ld < n_features ...) */
    FP_ENOMEM = 2,     /* host or device allocation failed */
    FP_EHIP = 3,       /* a HIP runtime call failed (message names it) */
    FP_ECORRUPT = 4,   /* malformed forest or packed buffer (range, cycle, checksum) */
    FP_E2BIG = 5,      /* request larger than a configured limit (capacity, budget) */
    FP_EAGAIN = 6,     /* bounded queue full: retry later */
    FP_ENOTREADY = 7,  /* result not ready yet (poll) */
    FP_ENODEV = 8      /* no usable gfx950 device / object not uploaded */
};

/* Message describing the last error on the calling thread ("" if none). */
const char *fp_last_error(void);

/* Library version string, "forestpack <major>.<minor> packed-format <n>". */
const char *fp_version(void);

/* ------------------------------------------------------------------------ */
/* Trained forest (input to packing)                                          */
/* ------------------------------------------------------------------------ */
/*
 * The input of packing is a trained forest of T trees (Sec. III): each
 * internal node holds a split (feature, fp32 threshold) and two children; each
 * leaf holds one class label (Sec. III); training cardinalities (in-bag sample
 * counts reaching each node) drive the statistical ordering (Sec. III-A, Stat).
 *
 * Layout: structure of arrays, trees concatenated.  Tree t owns nodes
 * [tree_node_offset[t], tree_node_offset[t+1]); ids inside left/right are
 * local to the tree; local node 0 is the root.  Nodes are expected in
 * node-creation order (breadth-first for the trainer used in the tests), but
 * any order whose links form a tree is accepted.
 *
 *   feature[i]     >= 0: split feature (< n_features); < 0: leaf
 *   threshold[i]   split threshold (fp32), ignored for leaves
 *   left[i],right[i] local child ids of an internal node, ignored for leaves
 *   leaf_class[i]  class of a leaf in [0, n_classes), ignored for internal nodes
 *   cardinality[i] in-bag training count (>= 0); NULL: every leaf counts 1 and
 *                  an internal node counts the leaves below it
 * All arrays are host memory, borrowed during fp_pack_forest only.
 */
typedef struct fp_forest_view {
    int32_t n_trees;
    int32_t n_features;
    int32_t n_classes;
    int32_t reserved;
    const int64_t *tree_node_offset; /* [n_trees + 1], [0] == 0, non-decreasing */
    const int32_t *feature;
    const float *threshold;
    const int32_t *left;
    const int32_t *right;
    const int32_t *leaf_class;
    const int64_t *cardinality; /* nullable */
} fp_forest_view;

/* ------------------------------------------------------------------------ */
/* Packing                                                                    */
/* ------------------------------------------------------------------------ */
enum {
    /* Baseline: every tree its own array in breadth-first order with leaves
     * stored as nodes (the BF layout of Sec. III-A, the paper's baseline). */
    FP_LAYOUT_NAIVE = 0,
    /* Forest packing (Sec. III-A): leaves replaced by class references (DF-),
     * per-tree statistical depth-first order with the more frequently taken
     * child adjacent to its parent (Stat), trees grouped into bins whose top
     * levels are interleaved level by level across the bin's trees (Bin). */
    FP_LAYOUT_PACKED = 1,
    /* PACKED with 8-byte nodes below the interleaved levels: the Stat hot
     * child is implicitly the next node, so a 16-byte load fetches a node and
     * its most likely successor (the prefetch of the adjacent line that the
     * paper's EU estimate credits, Sec. III-A).  Needs the feature index, the
     * classes and in-tree distances to fit 32 bits (FP_E2BIG otherwise);
     * line_align is ignored. */
    FP_LAYOUT_COMPACT = 2,
    /* Every tree cut into blocks, each a complete three-level subtree (7
     * node slots + a header): one fetch serves up to three steps of a walk.
     * A block takes 48 bytes when a node's feature and child codes fit 19
     * bits (feature bits + 2 x (1 + max(class bits, 3))), else 64 bytes.
     * A block's child blocks are stored together, most-visited first by
     * training cardinality (Stat at block granularity).  Bin interleaving
     * moves to blocks: the blocks whose root node has depth <=
     * interleave_depth, of all the bin's trees, come first, level-major.
     * Needs feature and class fields to fit 32 bits (FP_E2BIG otherwise);
     * line_align is ignored. */
    FP_LAYOUT_BLOCKED = 3,
    /* Like BLOCKED, but a block holds the up to 7 most visited nodes
     * reachable from its root (chosen greedily by training cardinality: the
     * hot paths of Stat, grouped into one fetch) instead of a fixed
     * three-level subtree, with a table that maps the 7 split outcomes to
     * the block's exit.  A block takes 48 bytes when at most 512 features
     * are used and every threshold of the forest is exactly an fp16 value
     * (stored as fp16; e.g. pixel data with half-integer thresholds), else
     * 64 bytes.  The 48-byte form compares in fp16 against a row tile
     * rounded toward +infinity, which gives the fp32 compare's result for
     * every such threshold (see feature_lds).  Needs
     * at most 4,096 used features and 32 classes (FP_E2BIG otherwise);
     * line_align is ignored. */
    FP_LAYOUT_CLUSTERED = 4
};

/* Node order inside a tree, for the layout ablation of Sec. III-A (Fig. 4). */
enum {
    /* the layout's own order: breadth-first (NAIVE), Stat (PACKED, COMPACT),
     * blocks (BLOCKED, CLUSTERED) */
    FP_ORDER_DEFAULT = 0,
    /* depth-first pre-order, left child first: with NAIVE the DF layout (leaves
     * stored), with PACKED the DF- layout (class references, no Stat); other
     * layouts reject it (FP_EINVAL) */
    FP_ORDER_DF = 1
};

/*
 * Packing parameters (Sec. III-A, "two parameters used when interleaving"):
 *   bin_size          trees per bin (stripe width); <= 0 or > T: one bin of all
 *                     trees.  Bins hold consecutive trees; the last may be short.
 *   interleave_depth  depths 0..D of every tree in a bin are interleaved
 *                     (D = 0: only the roots are contiguous, as in Fig. 2);
 *                     0 <= D <= 30.
 *   line_align        1: start each deep subtree on a 128-byte line when it
 *                     fits in the remaining part of the current line otherwise;
 *                     0: dense.  (Ignored by the naive layout.)
 *   node_order        FP_ORDER_DEFAULT or FP_ORDER_DF (see above).
 */
typedef struct fp_pack_opts {
    int32_t layout;
    int32_t bin_size;
    int32_t interleave_depth;
    int32_t line_align;
    int32_t node_order;
} fp_pack_opts;

typedef struct fp_packed fp_packed;

/* Summary of a packed forest. */
typedef struct fp_packed_info {
    int32_t layout, n_trees, n_features, n_classes;
    int32_t bin_size, interleave_depth, n_bins, max_top_nodes; /* largest bin top region */
    int64_t n_nodes;      /* stored 16-byte nodes */
    int64_t n_internal;   /* internal nodes of the forest */
    int64_t n_leaves;     /* leaves of the forest */
    int64_t bytes;        /* size of the packed buffer (host and device copy) */
    int32_t uploaded;     /* 1 once fp_packed_upload succeeded */
    int32_t max_depth;    /* deepest leaf depth (root = 0) */
    int32_t n_used_features; /* observation columns some split tests */
    int32_t reserved;
    double expected_depth;   /* internal nodes a training-distributed observation
                                visits per tree (leaf depths weighted by
                                cardinality): the average depth of Eq. 1 */
    double mean_bias;        /* mean over internal nodes of max(LC, RC) / PN,
                                the bias of the EU estimate (Sec. III-A) */
    double expected_fetches; /* fetch units such an observation loads per tree:
                                nodes (NAIVE: expected_depth + 1 for the stored
                                leaf; PACKED, COMPACT: expected_depth) or blocks
                                (BLOCKED, CLUSTERED) */
} fp_packed_info;

/*
 * Validate and re-lay a forest (Sec. III-A).  Deterministic: equal inputs give
 * byte-identical packed buffers.  Validation: tree offsets, feature < F,
 * children within the tree, class < C, every node reached at most once from
 * the root (no cycle, no shared child).  Errors: FP_EINVAL (null/size),
 * FP_ECORRUPT (malformed forest), FP_ENOMEM.  *out is set only on FP_OK.
 */
int fp_pack_forest(const fp_forest_view *forest, const fp_pack_opts *opts, fp_packed **out);

int fp_packed_info_get(const fp_packed *p, fp_packed_info *out);

/* Host copy of the packed buffer (owned by p, valid until fp_packed_free). */
int fp_packed_host_bytes(const fp_packed *p, const void **bytes, size_t *nbytes);

/* Rebuild a packed forest from bytes written by fp_packed_host_bytes or
 * fp_packed_save.  Verifies magic, version, sizes, checksum and every node
 * reference; FP_ECORRUPT on any mismatch.  The bytes are copied. */
int fp_packed_from_bytes(const void *bytes, size_t nbytes, fp_packed **out);

int fp_packed_save(const fp_packed *p, const char *path);
int fp_packed_load(const char *path, fp_packed **out);

/*
 * Copy the packed buffer to device memory `dev` (at least info.bytes bytes,
 * 256-byte aligned, owned by the caller and kept alive while p is used) on
 * `stream`.  p remembers dev and the current device; predictions read it.
 * Errors: FP_EINVAL (null, misaligned), FP_E2BIG (cap too small), FP_EHIP.
 */
int fp_packed_upload(fp_packed *p, void *dev, size_t cap, void *stream);

void fp_packed_free(fp_packed *p);

/*
 * Node cardinalities inferred from observations (Sec. III-A: the statistics
 * Stat orders by may be collected during training or inferred afterwards from
 * a suitably large set of observations).  Every row of X_dev (device fp32
 * [n_rows][ld], row-major, ld >= n_features) is walked through every tree on
 * the GPU (`stream`, synchronised before returning); card_out (host int64,
 * one entry per node of the view: tree_node_offset[T] entries, owned by the
 * caller) receives for each node the number of rows that reach it (a leaf:
 * rows ending there; an internal node: the sum of its children; unreachable
 * nodes 0).  Pass it as the view's `cardinality` to fp_pack_forest.  The
 * library allocates and frees temporary device memory (the forest in the
 * NAIVE layout and one int32 counter per node).  Errors: FP_EINVAL (NULL,
 * ld < n_features, n_rows outside [0, 2^31-1]), FP_ECORRUPT (malformed forest),
 * FP_ENOMEM, FP_EHIP.
 */
int fp_infer_cardinality(const fp_forest_view *forest, const float *X_dev, int64_t n_rows, int64_t ld,
                         int64_t *card_out, void *stream);

/* ------------------------------------------------------------------------ */
/* Single-forest prediction                                                   */
/* ------------------------------------------------------------------------ */
/*
 * Launch parameters of the traversal kernels (the GPU form of assigning bins
 * to workers, Sec. III, and of Bin+ round-robin evaluation, Sec. III-B).
 *   rows_per_block  observations per workgroup (packed layouts; 1..4096;
 *                   0: 16, halved until the workgroup's LDS tables fit, e.g.
 *                   for thousands of classes)
 *   cursors         trees a lane walks concurrently, round-robin (1, 2, 4, 8);
 *                   BLOCKED walks one block per lane and ignores it
 *   tree_groups     bins are split into this many groups, each group handled
 *                   by its own workgroups (votes then merge with atomics);
 *                   0: one group
 *   block_threads   workgroup size (64..1024, multiple of 64)
 *   lds_top_nodes   bin-top nodes staged in LDS (0: the whole top region as far
 *                   as LDS allows; -1: none)
 *   feature_lds     1: stage the observation tile in LDS (FP_E2BIG if it cannot
 *                   fit); -1: read features from memory; 0: LDS when it fits;
 *                   2: as 1, always in fp32.  Otherwise the LDS tile of a
 *                   CLUSTERED forest in its 48-byte form (every threshold
 *                   exact in fp16) holds fp16 values rounded toward
 *                   +infinity, half the bytes per row: for a threshold t
 *                   exact in fp16, x <= t holds exactly when the rounded
 *                   x <= t, so votes do not change (NaN stays NaN and goes
 *                   right); twice the rows fit a given LDS budget
 *   refill_lanes    a wavefront hands its idle cursors new walks once this many
 *                   of its lanes (1..64) are idle in a cursor slot, or when none
 *                   is walking; larger values spend fewer instructions on
 *                   refills and leave lanes idle longer
 *   lds_bytes       LDS one workgroup may use (0: half of a CU's, so that two
 *                   workgroups share a CU; capped at the device's per-block
 *                   limit); more LDS fits more observations per tile.  A
 *                   forest far larger than the caches walked in tree passes
 *                   runs faster with a CU's whole LDS in one 1024-thread
 *                   workgroup, which keeps one copy of the pass's first
 *                   blocks per CU instead of two
 *   tree_passes     the bins are split into this many consecutive groups
 *                   that run one after the other, each group walked by every
 *                   workgroup over all rows in a launch of its own, the
 *                   votes added up in place (0 or 1: one pass).  A forest
 *                   larger than the caches is then read from memory about
 *                   once per pass instead of once per row tile: only one
 *                   group's bins are in use at a time (Sec. III-A, Bin: keep
 *                   the well-used nodes of few trees cached).  Clamped so
 *                   that tree_passes x tree_groups <= the number of bins.
 *                   Batched plans run the passes' groups concurrently.
 * Zero fields mean "library default".  Naive layout uses block_threads only.
 */
typedef struct fp_tune {
    int32_t rows_per_block;
    int32_t cursors;
    int32_t tree_groups;
    int32_t block_threads;
    int32_t lds_top_nodes;
    int32_t feature_lds;
    int32_t refill_lanes;
    int32_t lds_bytes;
    int32_t tree_passes;
    int32_t reserved;
} fp_tune;

/* Store `tune` as p's own launch parameters (NULL: library defaults): the
 * ones fp_predict uses for a batch size with no tune recorded by
 * fp_tune_launch, and batched plans and the server use for p's jobs.
 * fp_packed_get_tune returns them.  Errors: FP_EINVAL (NULL p / out). */
int fp_packed_set_tune(fp_packed *p, const fp_tune *tune);
int fp_packed_get_tune(const fp_packed *p, fp_tune *out);

/*
 * Classify n_rows observations with the uploaded forest p: every row walks
 * every tree (Sec. III), its votes are counted per class and its class is
 * their argmax (Sec. III-A: packing leaves this result unchanged).
 *   X_dev     device fp32 [n_rows][ld], row-major; ld >= n_features
 *   votes_dev device int32 [n_rows][n_classes], overwritten
 *   class_dev device int32 [n_rows] (argmax, lowest index on ties) or NULL
 * Launch parameters: the tune recorded by fp_tune_launch for p's bytes and
 * the batch's size bucket ceil(log2(n_rows)) -- in this process or, with the
 * FP_TUNE_CACHE environment variable naming a file, by an earlier process --
 * else p's own (fp_packed_set_tune), else library defaults.
 * n_rows == 0 is a no-op.  Errors: FP_EINVAL (ld < F, null with n_rows > 0,
 * n_rows > 2^31-1), FP_ENODEV (not uploaded, other device), FP_EHIP.
 */
int fp_predict(const fp_packed *p, const float *X_dev, int64_t n_rows, int64_t ld,
               int32_t *votes_dev, int32_t *class_dev, void *stream);

/* The launch parameters fp_predict would use for a batch of n_rows rows of
 * p (for inspection).  *source (may be NULL): 2 a tune recorded by
 * fp_tune_launch (this process or the FP_TUNE_CACHE file), 1 p's own
 * (fp_packed_set_tune), 0 library defaults (*out all zero).  Errors:
 * FP_EINVAL (NULL p / out). */
int fp_predict_tune_get(const fp_packed *p, int64_t n_rows, fp_tune *out, int32_t *source);

/* fp_predict with explicit launch parameters (NULL: p's own, as set by
 * fp_packed_set_tune); no tune record is consulted.  Same arguments, layout,
 * ownership and errors as fp_predict, plus FP_EINVAL for launch parameters
 * outside their ranges and FP_E2BIG when the row tile or tables do not fit
 * the workgroup's LDS. */
int fp_predict_tuned(const fp_packed *p, const fp_tune *tune, const float *X_dev, int64_t n_rows,
                     int64_t ld, int32_t *votes_dev, int32_t *class_dev, void *stream);

/*
 * The design experiment of Sec. III-A (Fig. 2) for a forest already packed:
 * times candidate launch parameters of p (rows per workgroup, workgroup
 * size, cursors, refill threshold, tree groups; with block_threads 0 also a
 * CU's whole LDS for one 1024-thread workgroup and, for a forest larger than
 * the last-level cache, tree passes) on the first min(n_rows, 2^18) rows of
 * X_dev, records the fastest for p's bytes and the size bucket
 * ceil(log2(n_rows)) in the process-wide tune table (fp_predict then uses it
 * for batches of that bucket; fp_plan_create for jobs of that bucket when
 * block_threads and cursors match) and, when the FP_TUNE_CACHE environment
 * variable names a file, appends it there for later processes (a text file,
 * one record per line; a write failure only loses the record).
 *   block_threads, cursors  0: searched; > 0: kept fixed (a batched plan fixes
 *                           both for all its jobs)
 *   out                     receives the chosen parameters (may be NULL)
 * Votes never depend on the candidate.  The library allocates and frees a
 * temporary device buffer for the votes and synchronises `stream`.
 * Errors: FP_EINVAL (NULL, n_rows < 1, ld < F, naive layout, bad
 * block_threads / cursors), FP_E2BIG (no candidate fits), FP_ENOMEM, FP_EHIP.
 */
int fp_tune_launch(fp_packed *p, const float *X_dev, int64_t n_rows, int64_t ld, int32_t block_threads,
                   int32_t cursors, fp_tune *out, void *stream);


/* ------------------------------------------------------------------------ */
/* Autotuning (bin size, interleave depth, launch mapping)                    */
/* ------------------------------------------------------------------------ */
/*
 * Sec. III-A chooses the stripe width B and the interleave depth D with a
 * design experiment on the target processor (Fig. 2).  fp_autotune runs that
 * experiment on the GPU with the paper's cost model as its prior:
 *   1. it packs the forest in every candidate layout (PACKED, COMPACT,
 *      BLOCKED, CLUSTERED) and (B, D) (B in {T, 64, 16}, D in 0..7; block
 *      layouts interleave whole three-level blocks, so only D = 0, 3, 6) and
 *      scores each with Eq. 2's estimate from the packed header's statistics:
 *      (expected fetches per walk - well-used fetches) / EU, where EU =
 *      1 + b(1 + b(1 + b)) for node layouts (b the mean split bias), the
 *      interleaved levels 0..D are the well-used fetches, and a block counts
 *      as one fetch with EU 1;
 *   2. within each layout it times the top_k candidates by that score (one
 *      launch shape per layout kind);
 *   3. on the fastest packing it searches the launch mapping (rows per
 *      workgroup, workgroup size, cursors, refill threshold, tree groups)
 *      as fp_tune_launch does.
 * Times are HIP-event times on the first min(n_rows, sample_rows) rows.
 * Votes never depend on any candidate.  Results are kept per (forest
 * fingerprint, sample size, options) for the process and, when the
 * FP_TUNE_CACHE environment variable names a file, appended to it and read
 * back by later processes.
 *
 *   X_dev, n_rows, ld  device fp32 rows used for timing
 *   opts               NULL for defaults; block_threads / cursors > 0 fix
 *                      those parameters (a batched plan needs one workgroup
 *                      size and cursor count for all forests)
 *   opts->trials       NULL, or caller memory for max_trials entries: one per
 *                      packed candidate (model score, time if timed)
 * The library allocates and frees its own temporary device buffers.
 * Errors: FP_EINVAL, FP_ECORRUPT (forest), FP_ENOMEM, FP_EHIP.
 */
typedef struct fp_autotune_trial {
    fp_pack_opts pack;      /* the candidate packing */
    double model_cost;      /* Eq. 2 estimate: T x (expected fetches - well-used) / EU */
    double ms;              /* timed launch over the sample, -1 if not timed */
} fp_autotune_trial;

typedef struct fp_autotune_opts {
    int32_t block_threads;  /* 0: searched (256, 512, 1024) */
    int32_t cursors;        /* 0: searched (1, 2, 4) */
    int32_t reps;           /* timed launches per candidate (0: 3) */
    int32_t top_k;          /* packings timed per layout, best model score first (0: 2) */
    int64_t sample_rows;    /* 0: 65536 */
    fp_autotune_trial *trials; /* nullable: the candidate table */
    int32_t max_trials;     /* entries trials can hold */
    int32_t reserved;
} fp_autotune_opts;

typedef struct fp_autotune_result {
    fp_pack_opts pack;      /* best layout, bin size, interleave depth */
    fp_tune tune;           /* best launch parameters */
    double best_ms;         /* time of one launch over the sample, best candidate */
    double default_ms;      /* same, library defaults (PACKED, B = T, D = 4) */
    int32_t n_tried;        /* launches timed (packings and launch mappings) */
    int32_t cache_hit;      /* 1: answered from the table or file, nothing timed */
    int32_t n_candidates;   /* packings scored by the model */
    int32_t n_trials;       /* entries written to opts->trials */
} fp_autotune_result;

int fp_autotune(const fp_forest_view *forest, const float *X_dev, int64_t n_rows, int64_t ld,
                const fp_autotune_opts *opts, fp_autotune_result *out, void *stream);

/* ------------------------------------------------------------------------ */
/* Batched prediction: many forests, one persistent launch, one hipGraph      */
/* ------------------------------------------------------------------------ */
/*
 * Bins are independent work (Sec. III: each bin is assigned to a thread or a
 * process); many resident forests with uneven batches are served by one
 * persistent kernel whose workgroups pull (forest, tree group, row tiles)
 * work items from a device counter, largest estimated cost first (cost =
 * rows x trees x expected depth, the cost model of Eqs. 1-2).  The launch is
 * captured once in a hipGraph (counter reset, vote zeroing, kernel, argmax)
 * and replayed by fp_predict_batched.
 *
 * fp_job: one forest (uploaded, packed layout) with its rows.  Pointers are
 * fixed when the plan is created and must stay valid while the plan is used:
 *   X      device fp32 [n_rows][ld]
 *   votes  device int32 [n_rows][n_classes] (overwritten by every run)
 *   cls    device int32 [n_rows] or NULL
 * Each job uses its forest's launch parameters (fp_packed_set_tune, for
 * example from fp_autotune), except block_threads and cursors, which the plan
 * fixes for all jobs.
 */
typedef struct fp_job {
    const fp_packed *forest;
    const float *X;
    int64_t n_rows;
    int64_t ld;
    int32_t *votes;
    int32_t *cls;
} fp_job;

typedef struct fp_plan_opts {
    int32_t block_threads;  /* 0: 1024 */
    int32_t cursors;        /* 0: 2 (two walks per lane in node layouts; block
                               layouts walk one block per lane) */
    int32_t use_graph;      /* 1 (default when opts is NULL): capture a hipGraph; 0: plain launches */
    int32_t items_per_block;/* work items per persistent workgroup to aim for (0: 16) */
    int64_t lds_budget;     /* LDS bytes per workgroup (0: half of a CU's LDS) */
    int32_t autotune;       /* 1 (default when opts is NULL): each job with rows
                               uses the tune recorded for (its forest, its size
                               bucket, block_threads, cursors) and, if there is
                               none, runs fp_tune_launch on its own rows first;
                               0: each job uses its forest's own tune */
    int32_t reserved;
} fp_plan_opts;

typedef struct fp_plan fp_plan;

typedef struct fp_plan_info {
    int32_t n_jobs, n_items, blocks, block_threads;
    int32_t cursors, graph, lds_bytes, jobs_tuned; /* jobs timed by fp_tune_launch at creation */
    double total_cost;      /* sum of estimated node visits */
    int32_t jobs_cached;    /* jobs whose tune came from the tune table or file */
    int32_t reserved;
} fp_plan_info;

/* Build the work list and (optionally) the graph (opts NULL: defaults,
 * autotune on).  With autotune the library times launch candidates of jobs
 * that have no recorded tune, on their own rows (synchronising the device).
 * The library allocates the plan's device tables (released by fp_plan_free).
 * Errors: FP_EINVAL (bad job), FP_ENODEV (forest not uploaded / other
 * device), FP_E2BIG (LDS), FP_ENOMEM, FP_EHIP. */
int fp_plan_create(const fp_job *jobs, int32_t n_jobs, const fp_plan_opts *opts, fp_plan **out);

/* Run every job of the plan on `stream` (graph replay or plain launches). */
int fp_predict_batched(fp_plan *plan, void *stream);

int fp_plan_info_get(const fp_plan *plan, fp_plan_info *out);

void fp_plan_free(fp_plan *plan);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one batched
 * run of `jobs` -- what fp_plan_create followed by fp_predict_batched computes,
 * with the same kernels -- that allocates nothing.  The job table, the work
 * list and the work counter go to a fixed device array of 1 MiB inside the
 * library (one per GPU, held until the process ends), filled by a copy from
 * a static host area that HIP performs synchronously; no hipMalloc, hipFree
 * or other allocating call is made.  Limits: at most 4,096 jobs and as many
 * work items as fit the array after the job table (about 50,000 for a few
 * jobs); larger requests return FP_E2BIG.  Each job uses the tune recorded
 * for its forest, size bucket, block_threads and cursors, else its forest's
 * own tune; opts->autotune must be 0 (FP_EINVAL), use_graph is ignored.
 * Calls on one GPU share its array: a call waits for earlier work on
 * `stream` before overwriting it, but calls that overlap on different
 * streams of one GPU race.  Arguments, ownership and other errors are those
 * of fp_plan_create and fp_predict_batched.
 */
int fp_predict_batched_noalloc(const fp_job *jobs, int32_t n_jobs, const fp_plan_opts *opts, void *stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of prediction requests                       */
/* ------------------------------------------------------------------------ */
/*
 * Classification is trained once and used repeatedly (Sec. II); a server
 * keeps packed forests resident in HBM and answers a stream of requests of
 * varying size.  A scheduler thread admits pending requests in arrival order
 * while device staging memory (the HBM budget) and launch slots allow,
 * coalesces every admitted request into one batched persistent launch (same
 * kernel as fp_predict_batched), and overlaps up to max_inflight launches,
 * each on its own stream with its own H2D copy of the rows and D2H copy of
 * the votes.  Requests that arrive while launches run join the next launch
 * (continuous batching).  Results are bit-identical to fp_predict on the
 * same rows: a request's votes do not depend on what it was batched with.
 *
 * Ownership: the server borrows added forests (they must stay uploaded and
 * alive until fp_server_destroy); fp_serve_submit copies X_host before
 * returning; votes_host_out (int32 [n_rows][n_classes], host) must stay
 * valid until fp_serve_poll returns FP_OK for the ticket (or the server is
 * destroyed).  fp_serve_submit / fp_serve_poll may be called from any thread.
 */
enum {
    FP_EXECUTOR_HIP = 0,  /* launches on the current HIP device (the product path) */
    /* A CPU stand-in for the device, for testing the scheduler (admission,
     * coalescing, retries, time-outs) on hosts without a GPU: the "device"
     * rings are host memory, a launch completes fake_delay_us after it is
     * issued, and its "votes" are not a classification but a checksum of
     * each row: votes[i][c] = (h ^ (c * 0x9E3779B9)) & 0x7FFFFFFF with h the
     * 32-bit FNV-1a hash (offset 2166136261, prime 16777619) of row i's
     * n_features fp32 values as little-endian bytes.  Forests need not be
     * uploaded; fake_fail_every = k > 0 makes every k-th launch fail. */
    FP_EXECUTOR_CPU_FAKE = 1
};

typedef struct fp_server_opts {
    int64_t hbm_budget_bytes;    /* device staging for in-flight rows + votes (0: 1 GiB) */
    int64_t max_rows_per_launch; /* coalescing cap per launch (0: 262144) */
    int32_t max_inflight;        /* launches in flight (0: 4) */
    int32_t max_queue;           /* pending requests before FP_EAGAIN (0: 1 << 20) */
    int32_t block_threads;       /* workgroup size of the launches (0: 1024) */
    int32_t cursors;             /* cursors per lane (0: 2) */
    int32_t max_retries;         /* a request whose launch failed is queued again at
                                    the head this many times before it fails (0: 2;
                                    -1: never retried) */
    int32_t executor;            /* FP_EXECUTOR_HIP (0) or FP_EXECUTOR_CPU_FAKE */
    int32_t fake_delay_us;       /* CPU fake: microseconds from issue to completion */
    int32_t fake_fail_every;     /* CPU fake: every k-th launch fails (0: none) */
} fp_server_opts;

typedef struct fp_serve_stats {
    int64_t submitted, completed, rejected, launches, rows;
    int64_t pending, inflight;
    double mean_ms, p50_ms, p99_ms, max_ms; /* submit -> result ready, completed requests */
    double mean_rows_per_launch;
    double elapsed_s;                       /* since creation or the last reset */
    int64_t failed_launches;                /* launches whose issue or completion failed */
    int64_t retried;                        /* requests queued again after a failed launch */
    int64_t failed;                         /* requests that failed after their retries */
} fp_serve_stats;

typedef struct fp_server fp_server;

/* Allocates the HBM staging arena, its pinned host mirror, streams and the
 * scheduler thread (the CPU fake executor: host rings and the thread only).
 * Errors: FP_EINVAL, FP_ENOMEM, FP_EHIP. */
int fp_server_create(const fp_server_opts *opts, fp_server **out);

/* Register a packed forest (any packed layout, not NAIVE), uploaded on the
 * server's device (the CPU fake executor needs no upload); *forest_id
 * receives its id.  Its fp_tune (rows_per_block, tree_groups, tree_passes,
 * lds_top_nodes, feature_lds, refill_lanes) is used for its requests; its
 * tables must fit the server's LDS budget.  Requests are small, so small
 * tiles (16-32 rows) and, for a forest of many bins, tree groups spread a
 * request over more workgroups and cut its latency (tree passes run as
 * concurrent groups here).  Errors: FP_EINVAL (NULL, naive layout),
 * FP_ENODEV (not uploaded, other device), FP_E2BIG (LDS). */
int fp_server_add_forest(fp_server *s, const fp_packed *forest, int32_t *forest_id);

/* Queue a request: rows X_host [n_rows][ld] (host fp32, copied before return).
 * Never blocks.  Errors: FP_EINVAL, FP_E2BIG (request larger than the whole
 * HBM budget or than max_rows_per_launch), FP_EAGAIN (queue full). */
int fp_serve_submit(fp_server *s, int32_t forest_id, const float *X_host, int64_t n_rows, int64_t ld,
                    int32_t *votes_host_out, uint64_t *ticket);

/* Wait up to timeout_us (0: just test, < 0: forever) for a ticket.  FP_OK:
 * votes written, ticket retired.  FP_ENOTREADY: not yet.  FP_EINVAL: unknown
 * ticket.  FP_EHIP: the request's launches failed max_retries + 1 times (the
 * ticket is retired). */
int fp_serve_poll(fp_server *s, uint64_t ticket, int64_t timeout_us);

int fp_server_stats(fp_server *s, fp_serve_stats *out);
int fp_server_reset_stats(fp_server *s);

/* Stops the scheduler after in-flight launches finish; pending requests are
 * dropped.  Frees every server resource. */
void fp_server_destroy(fp_server *s);

/*
 * Open-loop load driver used to measure a server without client-side
 * coordinated omission: `submit_threads` library threads submit request i at
 * replay start + arrival_s (arrival times must be non-decreasing), and the
 * call returns once every request is answered.  latency_ms[i] = votes ready
 * - scheduled arrival (so time a request waited in the client counts);
 * lag_ms[i] = actual submit - scheduled arrival.  A request that failed has
 * latency -1 and the call returns its error.  Arrays are host memory of n
 * entries; rows and vote buffers follow fp_serve_submit's rules.
 */
typedef struct fp_replay_request {
    int32_t forest_id;
    int32_t reserved;
    const float *X_host;
    int64_t n_rows;
    int64_t ld;
    int32_t *votes_host_out;
    double arrival_s;
} fp_replay_request;

int fp_serve_replay(fp_server *s, const fp_replay_request *reqs, int64_t n, int32_t submit_threads,
                    double *latency_ms, double *lag_ms);

/* ------------------------------------------------------------------------ */
/* Measurement probes (the ceilings the walk is measured against; not part of */
/* classification)                                                          */
/* ------------------------------------------------------------------------ */
/*
 * HBM stream rate: copies `bytes` (a multiple of 16) from src_dev to dst_dev
 * (device buffers, 16-byte aligned, caller-owned) with 16-byte coalesced
 * loads and stores, once to warm up and once timed with HIP events on
 * `stream`; *gbps = bytes read + written per second / 1e9.
 * Errors: FP_EINVAL, FP_EHIP.
 */
int fp_probe_stream(const void *src_dev, void *dst_dev, uint64_t bytes, double *gbps, void *stream);

/*
 * Dependent random-gather rate, the ceiling of a walk whose every fetch
 * needs the previous one (Sec. III: a cache miss per node; on the GPU a
 * dependent load per node or block).  buf_dev (caller-owned, 16-byte
 * aligned, `bytes` long, overwritten) is laid out as one pseudo-random cycle
 * over n elements of fetch_bytes (16, 48 or 64) bytes, n the largest power of
 * two that fits (at least 64, at most 2^31); every lane of a full GPU
 * (2 x CUs workgroups of 1024) follows `chains` (1, 2, 4, 8) independent
 * chains for `steps` steps, loading each element whole.  *fetches_per_s =
 * element fetches per second (timed launch after a warm-up).
 * Errors: FP_EINVAL, FP_EHIP.
 */
int fp_probe_gather(void *buf_dev, uint64_t bytes, int32_t fetch_bytes, int32_t chains, int32_t steps,
                    double *fetches_per_s, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FORESTPACK_H */
