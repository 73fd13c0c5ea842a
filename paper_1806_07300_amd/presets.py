"""Launch presets for the named workloads (pack options + kernel launch
parameters).  The image-shaped workload (784 features, 10 classes, 128 trees
grown to purity) is the one the benchmark times."""

IMAGE = {
    "pack": {"layout": 4, "bin_size": 128, "interleave_depth": 3, "line_align": 0},
    # 96 rows of 353 used features, staged as fp16 (every threshold of this
    # forest is exact in fp16), fill the LDS share of one of two workgroups
    # per CU but for 139 blocks: the 128 trees' root blocks are served from
    # LDS (104 rows fit too, as fast, with no blocks in LDS); feature_lds 1
    # turns a tile that no longer fits into an error instead of a silent fall
    # back to features read from memory
    "tune": {"rows_per_block": 96, "cursors": 1, "tree_groups": 1, "block_threads": 1024, "refill_lanes": 48,
             "feature_lds": 1},
    "naive_tune": {"block_threads": 256},
}
