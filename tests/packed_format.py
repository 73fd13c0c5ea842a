"""Test helper: decodes the packed-forest byte format documented in
include/forestpack.h and paper_1806_07300_amd/csrc/fp_internal.h, and walks it
on the CPU (numpy) so that the host packer's output can be checked against
the checker without a GPU.  Test code only; the library never uses it."""
import struct

import numpy as np

HEADER = struct.Struct("<QIi" + "i" * 8 + "q" * 7 + "ii" + "Q" + "ii" + "q" + "d")
NODE = np.dtype([("thr", "<f4"), ("feat", "<i4"), ("left", "<i4"), ("right", "<i4")])
BIN = np.dtype([("node_base", "<i8"), ("first_tree", "<i4"), ("n_trees", "<i4"), ("top_len", "<i4"),
                ("deep_len", "<i4"), ("root_base", "<i4"), ("pad", "<i4")])


def decode(buf: np.ndarray) -> dict:
    b = buf.tobytes()
    f = HEADER.unpack_from(b, 0)
    keys = ["magic", "version", "layout", "n_trees", "n_features", "n_classes", "bin_size",
            "interleave_depth", "n_bins", "max_top_len", "max_bin_trees", "total_bytes", "table_offset",
            "roots_offset", "nodes_offset", "n_nodes", "n_internal", "n_leaves", "max_depth", "line_align",
            "checksum", "n_used_features", "pad0", "fmap_offset", "expected_depth"]
    h = dict(zip(keys, f))
    nodes = np.frombuffer(b, NODE, count=h["n_nodes"], offset=h["nodes_offset"])
    out = {"h": h, "nodes": nodes}
    if h["layout"] == 0:
        out["tree_off"] = np.frombuffer(b, "<i8", count=h["n_trees"] + 1, offset=h["table_offset"])
    else:
        out["bins"] = np.frombuffer(b, BIN, count=h["n_bins"], offset=h["table_offset"])
        out["roots"] = np.frombuffer(b, "<i4", count=h["n_trees"], offset=h["roots_offset"])
        out["fmap"] = np.frombuffer(b, "<i4", count=h["n_used_features"], offset=h["fmap_offset"])
    return out


def walk(dec: dict, X: np.ndarray) -> np.ndarray:
    """Votes [n, C] obtained by walking the decoded buffer (vectorised over rows)."""
    h = dec["h"]
    n, C = X.shape[0], h["n_classes"]
    votes = np.zeros((n, C), np.int32)
    nodes = dec["nodes"]
    rows = np.arange(n)
    if h["layout"] == 0:
        off = dec["tree_off"]
        for t in range(h["n_trees"]):
            tn = nodes[off[t]:off[t + 1]]
            cur = np.zeros(n, np.int64)
            while True:
                nd = tn[cur]
                leaf = nd["feat"] < 0
                if leaf.all():
                    np.add.at(votes, (rows, nd["left"]), 1)
                    break
                f = np.where(leaf, 0, nd["feat"])
                go_left = X[rows, f] <= nd["thr"]
                cur = np.where(leaf, cur, np.where(go_left, nd["left"], nd["right"]))
        return votes
    for be in dec["bins"]:
        bn = nodes[be["node_base"]:be["node_base"] + be["top_len"] + be["deep_len"]]
        for j in range(be["n_trees"]):
            ref = np.full(n, dec["roots"][be["root_base"] + j], np.int64)
            while (ref >= 0).any():
                live = ref >= 0
                nd = bn[np.where(live, ref, 0)]
                go_left = X[rows, dec["fmap"][nd["feat"]]] <= nd["thr"]
                ref = np.where(live, np.where(go_left, nd["left"], nd["right"]), ref)
            np.add.at(votes, (rows, -ref - 1), 1)
    return votes
