"""Hand-built forests for limit and edge-case tests (no training)."""
import numpy as np

import synth


def depth3_forest(n_trees, features, n_classes, thr=0.5):
    """Hand-built forest of complete depth-3 trees (7 internal nodes, 8 leaves,
    breadth-first ids: node k's children are 2k+1, 2k+2); tree t splits on
    features[t] (7 each), leaf l of tree t gets class (7t + l) mod C."""
    per = 15
    feat = np.full(n_trees * per, -1, np.int32)
    left = np.full(n_trees * per, -1, np.int32)
    right = np.full(n_trees * per, -1, np.int32)
    cls = np.zeros(n_trees * per, np.int32)
    card = np.zeros(n_trees * per, np.int64)
    depth = np.zeros(n_trees * per, np.int32)
    for t in range(n_trees):
        o = t * per
        for k in range(per):
            depth[o + k] = int(np.log2(k + 1))
            if k < 7:
                feat[o + k] = features[t][k]
                left[o + k], right[o + k] = 2 * k + 1, 2 * k + 2
            else:
                cls[o + k] = (7 * t + k - 7) % n_classes
                card[o + k] = 1 + (k * 3 + t) % 5
        for k in range(6, -1, -1):
            card[o + k] = card[o + 2 * k + 1] + card[o + 2 * k + 2]
    F = max(max(f) for f in features) + 1
    return synth.Forest(n_trees, F, n_classes, np.arange(n_trees + 1, dtype=np.int64) * per, feat,
                        np.full(n_trees * per, thr, np.float32), left, right, cls, card, depth)
