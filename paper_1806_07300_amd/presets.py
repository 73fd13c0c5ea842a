"""Launch presets for the named workloads (pack options + kernel launch
parameters).  The large tabular workload (28 features, 1,024 trees, bins of
16 trees) is the one the benchmark headlines; the image-shaped and small
ones are its extra keys."""

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

# Gaussian thresholds are not exact in fp16, so the clustered blocks take
# their 64-byte form with fp32 thresholds.  The 2.8 GB forest does not fit
# any cache: the 64 bins are walked in 16 passes of four bins (64 trees,
# about 177 MB), one launch each over all rows, so that a pass's blocks stay
# in the last-level cache while every row walks them.  One 1024-thread
# workgroup per CU takes the CU's whole LDS (lds_bytes 160 KB): a 768-row
# tile of 28 fp32 features and, in the rest, the first blocks of the pass's
# bins, which two workgroups per CU would each have to hold a copy of; with
# half the wavefronts, lanes are refilled once 24 of a wavefront's are idle.
# Measured on 10M rows: one pass 408 ms; 32 passes of 512-row tiles, two
# workgroups per CU 345 ms; this launch 269 ms
TABULAR = {
    "pack": {"layout": 4, "bin_size": 16, "interleave_depth": 3, "line_align": 0},
    "tune": {"rows_per_block": 768, "cursors": 1, "tree_groups": 1, "block_threads": 1024, "refill_lanes": 24,
             "feature_lds": 1, "tree_passes": 16, "lds_bytes": 163840},
    "naive_tune": {"block_threads": 256},
}

SMALL = {
    "pack": {"layout": 4, "bin_size": 16, "interleave_depth": 3, "line_align": 0},
    "tune": {"rows_per_block": 48, "cursors": 1, "tree_groups": 1, "block_threads": 1024, "refill_lanes": 32},
    "naive_tune": {"block_threads": 256},
}
