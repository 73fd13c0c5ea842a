/*
 * CPU checker for forest classification -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code with the GPU library.
 *
 * It computes the plain definition of what a packed forest must reproduce:
 * forest packing changes memory layout and evaluation order but not the
 * prediction itself (Sec. III-A), so the result is the classic per-tree
 * root-to-leaf walk of every observation over an unpacked forest stored in
 * node-creation order (the BF layout of Sec. III-A), with each leaf casting
 * one vote for its single class label (Sec. III: every leaf holds one class),
 * the votes summed over the T trees, and the predicted class their argmax.
 *
 * Readings where the paper is silent:
 *   - the split test is  x[feature] <= threshold  -> left child, in fp32 (the
 *     threshold is an fp32 value and x is fp32; NaN compares false -> right);
 *   - argmax ties go to the lowest class index.
 *
 * Built with plain -O2 (no fast-math, so no flush-to-zero of denormals).
 */
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/*
 * votes  : int32 [n_rows][n_classes], overwritten
 * pred   : int32 [n_rows] argmax of votes (lowest index on ties), may be NULL
 * visits : out, total internal nodes visited (may be NULL)
 * Returns 0, or -1 if a walk leaves the tree or reaches an out-of-range class.
 */
int oracle_predict(int32_t n_trees, int32_t n_features, int32_t n_classes,
                   const int64_t *tree_node_offset, const int32_t *feature,
                   const float *threshold, const int32_t *left, const int32_t *right,
                   const int32_t *leaf_class, const float *X, int64_t n_rows, int64_t ld,
                   int32_t *votes, int32_t *pred, int64_t *visits, int32_t n_threads) {
    int64_t total_visits = 0;
    int bad = 0;
#ifdef _OPENMP
    int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(static, 64) num_threads(nt) reduction(+ : total_visits) reduction(| : bad)
#endif
    for (int64_t i = 0; i < n_rows; i++) {
        const float *x = X + i * ld;
        int32_t *v = votes + i * n_classes;
        for (int32_t c = 0; c < n_classes; c++) v[c] = 0;
        for (int32_t t = 0; t < n_trees; t++) {
            const int64_t base = tree_node_offset[t];
            const int64_t size = tree_node_offset[t + 1] - base;
            int64_t node = 0;
            int64_t steps = 0;
            while (feature[base + node] >= 0) {
                int32_t f = feature[base + node];
                if (f >= n_features || steps > size) { bad = 1; break; }
                node = (x[f] <= threshold[base + node]) ? left[base + node] : right[base + node];
                steps++;
                if (node < 0 || node >= size) { bad = 1; break; }
            }
            total_visits += steps;
            if (bad) continue;
            int32_t c = leaf_class[base + node];
            if (c < 0 || c >= n_classes) { bad = 1; continue; }
            v[c] += 1;
        }
        if (pred) {
            int32_t best = 0;
            for (int32_t c = 1; c < n_classes; c++) if (v[c] > v[best]) best = c;
            pred[i] = best;
        }
    }
    if (visits) *visits = total_visits;
    return bad ? -1 : 0;
}
