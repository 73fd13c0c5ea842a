"""Test helper: decodes the packed-forest byte format documented in
include/forestpack.h and paper_1806_07300_amd/csrc/fp_internal.h, and walks it
on the CPU (numpy) so that the host packer's output can be checked against
the checker without a GPU.  Test code only; the library never uses it."""
import struct

import numpy as np

HEADER = struct.Struct("<QIi" + "i" * 8 + "q" * 7 + "ii" + "Q" + "ii" + "q" + "d" + "ii" + "ii" + "dd")
NODE8 = np.dtype([("thr", "<f4"), ("w", "<u4")])
NODE = np.dtype([("thr", "<f4"), ("feat", "<i4"), ("left", "<i4"), ("right", "<i4")])
BIN = np.dtype([("node_base", "<i8"), ("first_tree", "<i4"), ("n_trees", "<i4"), ("top_len", "<i4"),
                ("deep_len", "<i4"), ("root_base", "<i4"), ("pad", "<i4")])


def decode(buf: np.ndarray) -> dict:
    b = buf.tobytes()
    f = HEADER.unpack_from(b, 0)
    keys = ["magic", "version", "layout", "n_trees", "n_features", "n_classes", "bin_size",
            "interleave_depth", "n_bins", "max_top_len", "max_bin_trees", "total_bytes", "table_offset",
            "roots_offset", "nodes_offset", "n_nodes", "n_internal", "n_leaves", "max_depth", "line_align",
            "checksum", "n_used_features", "pad0", "fmap_offset", "expected_depth", "compact_fbits",
            "compact_cbits", "block_bytes", "pad1", "mean_bias", "expected_fetches"]
    h = dict(zip(keys, f))
    if h["layout"] in (2, 3, 4):
        nodes = np.frombuffer(b, NODE8, count=h["n_nodes"], offset=h["nodes_offset"])
    else:
        nodes = np.frombuffer(b, NODE, count=h["n_nodes"], offset=h["nodes_offset"])
    out = {"h": h, "nodes": nodes, "raw": b}
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
    if h["layout"] == 2:
        return walk_compact(dec, X)
    if h["layout"] == 3:
        return walk_blocked(dec, X)
    if h["layout"] == 4:
        return walk_clustered(dec, X)
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


def compact_bin(dec: dict, be):
    """(top Node16 array, deep Node8 array) of one bin of a COMPACT buffer."""
    h, b = dec["h"], dec["raw"]
    off = h["nodes_offset"] + 8 * int(be["node_base"])
    top = np.frombuffer(b, NODE, count=int(be["top_len"]), offset=off)
    deep = np.frombuffer(b, NODE8, count=int(be["deep_len"]), offset=off + 16 * int(be["top_len"]))
    return top, deep


def decode_node8(h, w):
    """Fields of compact deep-node words (vectorised)."""
    fb, cb = h["compact_fbits"], h["compact_cbits"]
    w = w.astype(np.int64)
    pay = w >> (fb + 3)
    return {"feat": w & ((1 << fb) - 1), "adj": (w >> fb) & 1, "adj_left": (w >> (fb + 1)) & 1,
            "cold_class": (w >> (fb + 2)) & 1, "payload": pay, "lclass": pay & ((1 << cb) - 1), "rclass": pay >> cb}


def walk_compact(dec: dict, X: np.ndarray) -> np.ndarray:
    h = dec["h"]
    n, C = X.shape[0], h["n_classes"]
    votes = np.zeros((n, C), np.int32)
    rows = np.arange(n)
    for be in dec["bins"]:
        top, deep = compact_bin(dec, be)
        tl = int(be["top_len"])
        fields = decode_node8(h, deep["w"]) if len(deep) else None
        for j in range(int(be["n_trees"])):
            ref = np.full(n, dec["roots"][be["root_base"] + j], np.int64)
            while (ref >= 0).any():
                live = ref >= 0
                is_top = live & (ref < tl)
                is_deep = live & (ref >= tl)
                new = ref.copy()
                if is_top.any():
                    nd = top[np.where(is_top, ref, 0)]
                    go = X[rows, dec["fmap"][nd["feat"]]] <= nd["thr"]
                    new = np.where(is_top, np.where(go, nd["left"], nd["right"]), new)
                if is_deep.any():
                    i = np.where(is_deep, ref - tl, 0)
                    f = {k: v[i] for k, v in fields.items()}
                    go = X[rows, dec["fmap"][f["feat"]]] <= deep["thr"][i]
                    adj_taken = go == (f["adj_left"] == 1)
                    nxt_adj = np.where(adj_taken, ref + 1,
                                       np.where(f["cold_class"] == 1, -f["payload"] - 1, ref + f["payload"]))
                    nxt_leaf = -np.where(go, f["lclass"], f["rclass"]) - 1
                    new = np.where(is_deep, np.where(f["adj"] == 1, nxt_adj, nxt_leaf), new)
                ref = new
            np.add.at(votes, (rows, -ref - 1), 1)
    return votes


BLOCK = np.dtype({"names": ["child_base", "ranks", "slot"],
                  "formats": ["<u4", "<u4", np.dtype((NODE8, 7))]})
BLOCK48 = np.dtype([("words", "<u4", 5), ("thr", "<f4", 7)])
BLOCKC = np.dtype([("thr", "<f4", 7), ("care", "u1", 8), ("val", "u1", 8), ("rest", "<u4", 5)])
BLOCKC48 = np.dtype([("thr16", "<f2", 7), ("rest_hi", "<u2"), ("care", "u1", 8), ("val", "u1", 8),
                     ("rest", "<u4", 4)])
WORD48_BITS = 19
C48_FEAT_POS = [48, 64, 73, 82, 96, 105, 114]  # 9-bit feature fields of a 48-byte CLUSTERED block


def blocked_bin(dec: dict, be):
    """(top Node16 array (empty), raw block array) of one bin of a BLOCKED buffer."""
    h, b = dec["h"], dec["raw"]
    off = h["nodes_offset"] + 8 * int(be["node_base"])
    tl = int(be["top_len"])
    top = np.frombuffer(b, NODE, count=tl, offset=off)
    if h["layout"] == 4:
        dt = BLOCKC48 if h["block_bytes"] == 48 else BLOCKC
    else:
        dt = BLOCK48 if h["block_bytes"] == 48 else BLOCK
    blocks = np.frombuffer(b, dt, count=int(be["deep_len"]), offset=off + 8 * ((2 * tl + 7) // 8 * 8))
    return top, blocks


def block_fields(h, blocks):
    """Either block form as plain arrays: child_base [n], thr [n, 7],
    word [n, 7], feat [n, 7], kind [n, 7, 2] (1 = class), pay [n, 7, 2]
    (class, or exit rank of a bottom slot's internal child)."""
    fb, cb = h["compact_fbits"], h["compact_cbits"]
    n = len(blocks)
    if h["block_bytes"] == 48:
        P = max(cb, 3)
        big = np.zeros(n, object)
        wd = blocks["words"].astype(object)
        for i in range(5):
            big = big + (wd[:, i] << (32 * i))
        word = np.zeros((n, 7), np.int64)
        for sl in range(7):
            word[:, sl] = [int((v >> (WORD48_BITS * sl)) & ((1 << WORD48_BITS) - 1)) for v in big]
        child_base = (blocks["words"][:, 4].astype(np.int64) >> 8)
        thr = blocks["thr"]
        cw = 1 + P
    else:
        word = blocks["slot"]["w"].astype(np.int64)
        child_base = blocks["child_base"].astype(np.int64)
        thr = blocks["slot"]["thr"]
        cw = 1 + cb
    feat = word & ((1 << fb) - 1)
    kind = np.zeros((n, 7, 2), np.int64)
    pay = np.zeros((n, 7, 2), np.int64)
    for side in range(2):
        c = (word >> (fb + side * cw)) & ((1 << cw) - 1)
        kind[:, :, side] = c & 1
        pay[:, :, side] = c >> 1
    if h["block_bytes"] != 48:  # exit ranks live in the ranks table
        ranks = blocks["ranks"].astype(np.int64)
        for sl in range(3, 7):
            for side in range(2):
                e = 2 * (sl - 3) + side
                internal = kind[:, sl, side] == 0
                pay[:, sl, side] = np.where(internal, (ranks >> (4 * e)) & 7, pay[:, sl, side])
    return {"child_base": child_base, "thr": thr, "word": word, "feat": feat, "kind": kind, "pay": pay}


def walk_blocked(dec: dict, X: np.ndarray, stats: dict | None = None) -> np.ndarray:
    """Votes [n, C] from walking a BLOCKED buffer (vectorised over rows);
    stats["fetches"] counts the blocks the walks load."""
    h = dec["h"]
    n, C = X.shape[0], h["n_classes"]
    votes = np.zeros((n, C), np.int32)
    rows = np.arange(n)
    fmap = dec["fmap"]
    for be in dec["bins"]:
        _, blocks = blocked_bin(dec, be)
        bf = block_fields(h, blocks) if len(blocks) else None
        for j in range(int(be["n_trees"])):
            ref = np.full(n, dec["roots"][be["root_base"] + j], np.int64)
            k = np.where(ref >= 0, ref, 0)
            slot = np.zeros(n, np.int64)
            live = ref >= 0
            if stats is not None:
                stats["fetches"] = stats.get("fetches", 0) + int(live.sum())
            while live.any():
                f = bf["feat"][k, slot]
                side = np.where(X[rows, fmap[f]] <= bf["thr"][k, slot], 0, 1)
                kind = bf["kind"][k, slot, side]
                pay = bf["pay"][k, slot, side]
                leaf = live & (kind == 1)
                ref = np.where(leaf, -pay - 1, ref)
                inner = live & ~leaf & (slot < 3)
                ex = live & ~leaf & (slot >= 3)
                k = np.where(ex, bf["child_base"][k] + pay, k)
                slot = np.where(inner, 2 * slot + 1 + side, np.where(ex, 0, slot))
                live = live & ~leaf
                if stats is not None:
                    stats["fetches"] += int(ex.sum())
            np.add.at(votes, (rows, -ref - 1), 1)
    return votes


def reseal(buf: np.ndarray) -> np.ndarray:
    """Copy of a packed buffer with its header checksum recomputed (FNV-1a
    over the little-endian 64-bit words after the 256-byte header), so that
    tests can plant structural faults behind a valid checksum."""
    out = buf.copy()
    words = out[256:].view("<u8")
    h = 0xcbf29ce484222325
    for v in words.tolist():
        h = ((h ^ v) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    pos = struct.calcsize("<QIi" + "i" * 8 + "q" * 7 + "ii")
    out[pos:pos + 8] = np.frombuffer(struct.pack("<Q", h), np.uint8)
    return out


def cluster_fields(blocks):
    """CLUSTERED blocks, either form, as plain arrays: thr [n, 7] (fp32),
    feat [n, 7], care, val, target [n, 8], child_base, n_children,
    n_exits [n] (unused exits have care = val = 0x80), and the bits above
    the last field (must be zero)."""
    n = len(blocks)
    c48 = blocks.dtype == BLOCKC48
    if c48:  # features placed so that none crosses a 32-bit word
        fw, fpos, (p_base, w_base), p_nchild = 9, C48_FEAT_POS, (123, 21), 57
        spare = [(61, 3), (91, 5)]
    else:
        fw, fpos, (p_base, w_base), p_nchild = 12, [48 + 12 * s for s in range(7)], (132, 24), 156
        spare = []
    big = [sum(int(w) << (32 * i) for i, w in enumerate(row)) for row in blocks["rest"]]
    if c48:
        big = [v | int(hi) << 128 for v, hi in zip(big, blocks["rest_hi"])]
    get = lambda pos, width: np.array([(v >> pos) & ((1 << width) - 1) for v in big], np.int64).reshape(n)
    care = blocks["care"].astype(np.int64)
    stray = np.zeros(n, np.int64)
    for pos, width in spare:
        stray |= get(pos, width)
    return {"thr": blocks["thr16"].astype(np.float32) if c48 else blocks["thr"],
            "feat": np.stack([get(p, fw) for p in fpos], 1) if n else np.zeros((0, 7), np.int64),
            "care": care, "val": blocks["val"].astype(np.int64),
            "target": np.stack([get(6 * e, 6) for e in range(8)], 1) if n else np.zeros((0, 8), np.int64),
            "child_base": get(p_base, w_base), "n_children": get(p_nchild, 4), "n_exits": (care != 0x80).sum(1),
            "stray": stray}


def walk_clustered(dec: dict, X: np.ndarray, stats: dict | None = None) -> np.ndarray:
    """Votes [n, C] from walking a CLUSTERED buffer (vectorised over rows):
    all seven split outcomes of a block, then the one exit they select;
    stats["fetches"] counts the blocks the walks load."""
    h = dec["h"]
    n, C = X.shape[0], h["n_classes"]
    votes = np.zeros((n, C), np.int32)
    rows = np.arange(n)
    fmap = dec["fmap"]
    for be in dec["bins"]:
        _, blocks = blocked_bin(dec, be)
        cf = cluster_fields(blocks) if len(blocks) else None
        for j in range(int(be["n_trees"])):
            ref = np.full(n, dec["roots"][be["root_base"] + j], np.int64)
            while (ref >= 0).any():
                live = ref >= 0
                if stats is not None:
                    stats["fetches"] = stats.get("fetches", 0) + int(live.sum())
                k = np.where(live, ref, 0)
                g = np.zeros(n, np.int64)
                for s in range(7):
                    right = ~(X[rows, fmap[cf["feat"][k, s]]] <= cf["thr"][k, s])
                    g |= right.astype(np.int64) << s
                t = np.zeros(n, np.int64)
                hits = np.zeros(n, np.int64)
                for e in range(8):
                    used = e < cf["n_exits"][k]
                    m = used & (((g ^ cf["val"][k, e]) & cf["care"][k, e]) == 0)
                    t = np.where(m, cf["target"][k, e], t)
                    hits += m
                assert (hits[live] == 1).all(), "exactly one exit per block"
                nxt = np.where(t & 32, cf["child_base"][k] + (t & 7), -(t & 31) - 1)
                ref = np.where(live, nxt, ref)
            np.add.at(votes, (rows, -ref - 1), 1)
    return votes
