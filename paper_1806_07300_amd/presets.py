"""Launch presets for the named workloads (pack options + kernel launch
parameters).  The image-shaped workload (784 features, 10 classes, 128 trees
grown to purity) is the one the benchmark times."""

IMAGE = {
    "pack": {"layout": 4, "bin_size": 128, "interleave_depth": 3, "line_align": 0},
    "tune": {"rows_per_block": 48, "cursors": 1, "tree_groups": 1, "block_threads": 1024, "refill_lanes": 32},
    "naive_tune": {"block_threads": 256},
}
