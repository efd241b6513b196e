/*
 * rpForests CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised C implementation of kNN search by random
 * projection forests (Yan, Wang, Wang, Wang, Li, "K-nearest Neighbor Search by Random
 * Projection Forests", arXiv 1812.11689).  Only the tests, the smoke check and the CPU
 * baseline of the benchmark load it; the HIP library never does, and the two share no
 * code, header, table or helper.
 *
 * Floating point is IEEE binary64 throughout, compiled with -ffp-contract=off.  Where
 * the paper leaves the arithmetic open, the oracle fixes one canonical definition (the
 * same definition the GPU path implements on its own):
 *
 *   canonical sum   canon_sum(v[0..m)): pad v with +0.0 to the next power of two and add
 *                   adjacent pairs level by level (a balanced binary tree in index order).
 *   projection      p = r.x (Sec. 2, projection coefficient): 32 partial sums,
 *                   s_c = sum over j = c (mod 32), j ascending, of (double)x_j*(double)r_j
 *                   (each product of two binary32 values is exact in binary64), then
 *                   p = canon_sum(s_0..s_31) + 0.0  (the "+ 0.0" maps -0 to +0).
 *   distance        D = |a - b|^2 (Alg. 3, distances to the candidates): 32 partial sums
 *                   s_c <- fma(delta_j, delta_j, s_c), delta_j = (double)a_j - (double)b_j
 *                   rounded, then D = canon_sum(s_0..s_31).
 *
 * Tree growth follows Alg. 1 with the median split point of Sec. 2: a node W with
 * |W| >= n_s = n0 + 1 is split; its members, kept in ascending original index, are
 * ordered by the key (p, index); the floor(m/2) smallest go left, the rest right, and the
 * split value c is p of the member of rank floor(m/2).  Direction choice follows Alg. 2
 * with the spread measured by S2 = canon_sum((p_i - mean)^2) (same argmax as the standard
 * deviation, since m is fixed within a node); the first try attaining the largest S2 wins
 * and try 0 is used when every S2 is 0.  Random directions are an input:
 * R[t][h-1][try][0..d) for heap id h (root 1, children 2h and 2h+1).
 *
 * The uniform split point that Alg. 1 prints (c drawn uniformly between the smallest and
 * the largest projection) is grown as well, with its random numbers from a counter-based
 * generator; its section below states the rule.
 *
 * kNN follows Alg. 3: each query falls through every tree to one leaf, the union of the
 * leaves' members is formed, exact distances are computed and the K closest are kept,
 * ordered by (D, index).  Fewer than K candidates leave (-1, +inf) in the tail.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define RPFO_CLASSES 32

/* ---- canonical arithmetic ------------------------------------------------------------ */

double rpfo_canon_sum(const double *v, int64_t m)
{
    if (m <= 0) return 0.0;
    int64_t p = 1;
    while (p < m) p <<= 1;
    double *a = (double *)malloc((size_t)p * sizeof(double));
    for (int64_t i = 0; i < p; i++) a[i] = (i < m) ? v[i] : 0.0;
    for (int64_t w = p; w > 1; w >>= 1)
        for (int64_t i = 0; i < w / 2; i++) a[i] = a[2 * i] + a[2 * i + 1];
    double r = a[0];
    free(a);
    return r;
}

double rpfo_canon_dot64(const float *x, const float *r, int d)
{
    double s[RPFO_CLASSES];
    for (int c = 0; c < RPFO_CLASSES; c++) s[c] = 0.0;
    for (int j = 0; j < d; j++) s[j % RPFO_CLASSES] = s[j % RPFO_CLASSES] + (double)x[j] * (double)r[j];
    return rpfo_canon_sum(s, RPFO_CLASSES) + 0.0;
}

double rpfo_canon_dist64(const float *a, const float *b, int d)
{
    double s[RPFO_CLASSES];
    for (int c = 0; c < RPFO_CLASSES; c++) s[c] = 0.0;
    for (int j = 0; j < d; j++) {
        double delta = (double)a[j] - (double)b[j];
        s[j % RPFO_CLASSES] = fma(delta, delta, s[j % RPFO_CLASSES]);
    }
    return rpfo_canon_sum(s, RPFO_CLASSES);
}

/* ---- tree shape (median rule) ---------------------------------------------------------- */

/* Number of split levels L: a node of size m is split iff m > n0, children get floor(m/2)
 * and ceil(m/2) points, so the deepest nodes have ceil(n/2^L) <= n0. */
int rpfo_depth(int64_t n, int64_t n0)
{
    int L = 0;
    while ((n + ((int64_t)1 << L) - 1) / ((int64_t)1 << L) > n0) L++;
    return L;
}

/* Offset (in the left-to-right leaf order) and size of heap node h, or -1 if h is not a
 * node of the tree (an ancestor of h is a leaf). */
int64_t rpfo_node_range(int64_t n, int64_t n0, int64_t h, int64_t *off)
{
    int depth = 0;
    while ((h >> depth) > 1) depth++;
    int64_t o = 0, m = n;
    for (int k = depth - 1; k >= 0; k--) {
        if (m <= n0) return -1;
        int right = (int)((h >> k) & 1);
        if (right) { o += m / 2; m = m - m / 2; }
        else m = m / 2;
    }
    if (off) *off = o;
    return m;
}

/* ---- Alg. 2 (whichProjection) ------------------------------------------------------------ */

static int which_projection(const float *X, int d, const int32_t *W, int64_t m,
                            const float *Rnode, int n_try, double *P)
{
    if (n_try == 1) return 0;
    double disp = 0.0;
    int dir = -1;
    double *w = (double *)malloc((size_t)m * sizeof(double));
    for (int i = 0; i < n_try; i++) {
        const float *r = Rnode + (int64_t)i * d;
        for (int64_t k = 0; k < m; k++) P[k] = rpfo_canon_dot64(X + (int64_t)W[k] * d, r, d);
        double mu = rpfo_canon_sum(P, m) / (double)m;
        for (int64_t k = 0; k < m; k++) {
            double dev = P[k] - mu;
            w[k] = dev * dev;
        }
        double t_disp = rpfo_canon_sum(w, m);
        if (t_disp > disp) {
            disp = t_disp;
            dir = i;
        }
    }
    free(w);
    return dir < 0 ? 0 : dir;
}

/* ---- Alg. 1 (rpTree), median split ------------------------------------------------------- */

typedef struct { double p; int32_t idx; } keyed_t;

static int cmp_keyed(const void *a, const void *b)
{
    const keyed_t *x = (const keyed_t *)a, *y = (const keyed_t *)b;
    if (x->p < y->p) return -1;
    if (x->p > y->p) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

typedef struct { int64_t heap; int64_t m; int32_t *idx; } node_t;
typedef struct { int64_t pos_key; int64_t heap; int64_t m; int32_t *idx; } leaf_t;

static int cmp_leaf(const void *a, const void *b)
{
    const leaf_t *x = (const leaf_t *)a, *y = (const leaf_t *)b;
    return (x->pos_key > y->pos_key) - (x->pos_key < y->pos_key);
}

/* Grow tree t.  Outputs: split value / split index / chosen try per heap slot (NaN, -1, -1
 * where the slot is not an internal node), the left-to-right concatenation of the leaves
 * (perm, members of each leaf ascending) and the heap id of each point's leaf. */
static void grow_tree(const float *X, int64_t n, int d, const float *Rt, int n_try, int64_t n0,
                      int L, double *split, int32_t *split_idx, int32_t *chosen, int32_t *perm,
                      int32_t *leaf_of)
{
    int64_t H = ((int64_t)1 << L) - 1;
    for (int64_t h = 0; h < H; h++) { split[h] = NAN; split_idx[h] = -1; chosen[h] = -1; }

    /* the working set of Alg. 1, kept as a stack: the order in which nodes are picked does
     * not change the tree, since each node's direction is fixed by its heap id */
    node_t *work = (node_t *)malloc(sizeof(node_t) * (size_t)(2 * L + 4));
    int top = 0;
    int32_t *root = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) root[i] = (int32_t)i;
    work[top++] = (node_t){1, n, root};

    leaf_t *leaves = (leaf_t *)malloc(sizeof(leaf_t) * (size_t)((int64_t)1 << L));
    int64_t n_leaves = 0;
    keyed_t *kp = (keyed_t *)malloc((size_t)n * sizeof(keyed_t));
    double *P = (double *)malloc((size_t)n * sizeof(double));

    while (top > 0) {
        node_t W = work[--top];
        int depth = 0;
        while ((W.heap >> depth) > 1) depth++;
        if (W.m < n0 + 1) { /* |W| < n_s: no further split, W is a neighbourhood (leaf) */
            leaves[n_leaves++] = (leaf_t){W.heap << (L - depth), W.heap, W.m, W.idx};
            continue;
        }
        const float *Rnode = Rt + (W.heap - 1) * (int64_t)n_try * d;
        int ch = which_projection(X, d, W.idx, W.m, Rnode, n_try, P);
        const float *r = Rnode + (int64_t)ch * d;
        for (int64_t k = 0; k < W.m; k++) {
            kp[k].p = rpfo_canon_dot64(X + (int64_t)W.idx[k] * d, r, d);
            kp[k].idx = W.idx[k];
        }
        /* the projections in ascending original index, kept for the partition below */
        for (int64_t k = 0; k < W.m; k++) P[k] = kp[k].p;
        qsort(kp, (size_t)W.m, sizeof(keyed_t), cmp_keyed);
        int64_t half = W.m / 2;
        keyed_t c = kp[half]; /* median split point: member of rank floor(m/2) */
        split[W.heap - 1] = c.p;
        split_idx[W.heap - 1] = c.idx;
        chosen[W.heap - 1] = ch;

        int32_t *left = (int32_t *)malloc((size_t)half * sizeof(int32_t));
        int32_t *right = (int32_t *)malloc((size_t)(W.m - half) * sizeof(int32_t));
        int64_t nl = 0, nr = 0;
        for (int64_t k = 0; k < W.m; k++) { /* W_L = {key < c}, W_R = the rest */
            keyed_t e = {P[k], W.idx[k]};
            if (cmp_keyed(&e, &c) < 0) left[nl++] = e.idx;
            else right[nr++] = e.idx;
        }
        free(W.idx);
        work[top++] = (node_t){2 * W.heap, nl, left};
        work[top++] = (node_t){2 * W.heap + 1, nr, right};
    }

    qsort(leaves, (size_t)n_leaves, sizeof(leaf_t), cmp_leaf);
    int64_t pos = 0;
    for (int64_t a = 0; a < n_leaves; a++) {
        for (int64_t k = 0; k < leaves[a].m; k++) {
            perm[pos++] = leaves[a].idx[k];
            leaf_of[leaves[a].idx[k]] = (int32_t)leaves[a].heap;
        }
        free(leaves[a].idx);
    }
    free(P);
    free(kp);
    free(work);
    free(leaves);
}

/* Alg. 3, forest growth: grow T independent trees.  R is [T][2^L-1][n_try][d].
 * Outputs split/split_idx/chosen [T][2^L-1], perm and leaf_of [T][n].  Returns L. */
int rpfo_build(const float *X, int64_t n, int d, const float *R, int T, int n_try, int64_t n0,
               double *split, int32_t *split_idx, int32_t *chosen, int32_t *perm,
               int32_t *leaf_of)
{
    int L = rpfo_depth(n, n0);
    int64_t H = ((int64_t)1 << L) - 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < T; t++)
        grow_tree(X, n, d, R + (int64_t)t * H * n_try * d, n_try, n0, L, split + t * H,
                  split_idx + t * H, chosen + t * H, perm + (int64_t)t * n, leaf_of + (int64_t)t * n);
    return L;
}

/* Alg. 3, descent: let each query fall through every tree.  At an internal node h the
 * query goes to the right child iff its projection onto the node's chosen direction is
 * >= the split value (W_R = {P >= c}).  Output: heap id of the leaf, [T][m]. */
void rpfo_route(const float *R, int T, int n_try, int d, int64_t n, int64_t n0,
                const int32_t *chosen, const double *split, const float *Q, int64_t m,
                int32_t *out_leaf)
{
    int L = rpfo_depth(n, n0);
    int64_t H = ((int64_t)1 << L) - 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < m; q++) {
        for (int t = 0; t < T; t++) {
            int64_t h = 1, size = n;
            while (size > n0) {
                const float *r = R + (((int64_t)t * H + (h - 1)) * n_try + chosen[t * H + h - 1]) * d;
                double p = rpfo_canon_dot64(Q + q * d, r, d);
                int right = p >= split[t * H + h - 1];
                size = right ? size - size / 2 : size / 2;
                h = 2 * h + right;
            }
            out_leaf[(int64_t)t * m + q] = (int32_t)h;
        }
    }
}

typedef struct { double D; int32_t idx; } cand_t;

static int cmp_cand(const void *a, const void *b)
{
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (x->D < y->D) return -1;
    if (x->D > y->D) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Alg. 3, union of the reached leaves and exact ranking, for a batch of queries whose leaves are known: N_q = union over trees
 * of the members of q's leaf (minus q itself if self[q] >= 0), exact distances to every
 * member of N_q, the K closest by (D, index).  out_dist holds sqrt(D).  qleaf is [T][m]. */
void rpfo_knn(const float *X, int64_t n, int d, int T, int64_t n0, const int32_t *perm,
              const float *Q, int64_t m, const int32_t *qleaf, const int64_t *self, int K,
              int32_t *out_idx, double *out_dist)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < m; q++) {
        int64_t cap = (int64_t)T * (n0 < n ? n0 : n);
        int32_t *u = (int32_t *)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(int32_t));
        int64_t nu = 0;
        for (int t = 0; t < T; t++) {
            int64_t off = 0;
            int64_t sz = rpfo_node_range(n, n0, qleaf[(int64_t)t * m + q], &off);
            for (int64_t k = 0; k < sz; k++) u[nu++] = perm[(int64_t)t * n + off + k];
        }
        qsort(u, (size_t)nu, sizeof(int32_t), cmp_i32);
        cand_t *c = (cand_t *)malloc((size_t)(nu > 0 ? nu : 1) * sizeof(cand_t));
        int64_t nc = 0;
        for (int64_t k = 0; k < nu; k++) {
            if (k > 0 && u[k] == u[k - 1]) continue; /* the union: each member once */
            if (self && self[q] == u[k]) continue;
            c[nc].idx = u[k];
            c[nc].D = rpfo_canon_dist64(Q + q * d, X + (int64_t)u[k] * d, d);
            nc++;
        }
        qsort(c, (size_t)nc, sizeof(cand_t), cmp_cand);
        for (int k = 0; k < K; k++) {
            out_idx[q * K + k] = k < nc ? c[k].idx : -1;
            out_dist[q * K + k] = k < nc ? sqrt(c[k].D) : INFINITY;
        }
        free(c);
        free(u);
    }
}

/* Exact kNN by brute force over all of U (the ground truth of Sec. 5.1): the K closest
 * points by (D, index), excluding self[q] when self is given and self[q] >= 0. */
void rpfo_bruteforce(const float *X, int64_t n, int d, const float *Q, int64_t m,
                     const int64_t *self, int K, int32_t *out_idx, double *out_dist)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < m; q++) {
        cand_t *best = (cand_t *)malloc(sizeof(cand_t) * (size_t)(K + 1));
        int nb = 0;
        for (int64_t j = 0; j < n; j++) {
            if (self && self[q] == j) continue;
            cand_t e = {rpfo_canon_dist64(Q + q * d, X + j * d, d), (int32_t)j};
            if (nb == K && cmp_cand(&e, &best[K - 1]) >= 0) continue;
            int k = nb < K ? nb++ : K - 1; /* insertion into the sorted top-K list */
            while (k > 0 && cmp_cand(&e, &best[k - 1]) < 0) {
                best[k] = best[k - 1];
                k--;
            }
            best[k] = e;
        }
        for (int k = 0; k < K; k++) {
            out_idx[q * K + k] = k < nb ? best[k].idx : -1;
            out_dist[q * K + k] = k < nb ? sqrt(best[k].D) : INFINITY;
        }
        free(best);
    }
}

/* ---- uniform split rule: Alg. 1 as printed, c drawn uniformly in [a, b] ----------------
 *
 * The trees' shapes depend on the data, so the random numbers of a node cannot be laid out
 * in advance as the median rule's direction array is.  They come from a counter-based
 * generator instead, keyed by (seed, tree, heap id of the node): SplitMix64 (Steele, Lea
 * and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).  Its stream
 * with seed s has the outputs  out(s, i) = mix64(s + (i + 1) * GAMMA), i = 0, 1, ...  with
 * GAMMA = 0x9E3779B97F4A7C15 and mix64 the published finaliser below (all arithmetic mod
 * 2^64).  The stream of node h of tree t has the seed out(out(seed, t), h), and its draws
 * are used as follows:
 *
 *   draw 0          the split fraction u = (draw >> 11) * 2^-53, a uniform in [0, 1) on
 *                   the 2^-53 grid;
 *   draws 1, 2, ..  the nTry random directions (Alg. 1 and Alg. 2): coordinate j of try i
 *                   takes the six draws 1 + 6 (i d + j) + q, q = 0..5, splits each into its
 *                   two 32-bit halves, and is (sum of the twelve halves) * 2^-32 - 6, exact in
 *                   binary64, rounded once to binary32 (an Irwin-Hall approximation of a
 *                   standard normal coordinate: mean 0, variance 1).
 *
 * A node W is split when |W| > n0 and its depth is below RPFO_UNIFORM_DEPTH: the direction
 * is chosen among the tries as for the median rule (Alg. 2), a = min and b = max of the
 * projections, c = RN(a + RN(u * RN(b - a))), W_L = {p < c}, W_R = {p >= c}, both kept in
 * ascending original index.  When one side is empty (a = b, or c rounded onto a) the node
 * is a leaf, so a leaf larger than n0 holds points that the node's direction does not
 * separate.  Leaves are ordered left to right; a point's leaf id is the ordinal of its leaf
 * in that order. */

#define RPFO_GAMMA 0x9E3779B97F4A7C15ull
#define RPFO_UNIFORM_DEPTH 62

uint64_t rpfo_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t rpfo_stream(uint64_t s, uint64_t i) { return rpfo_mix64(s + (i + 1) * RPFO_GAMMA); }

uint64_t rpfo_node_key(uint64_t seed, int t, int64_t h)
{
    return rpfo_stream(rpfo_stream(seed, (uint64_t)t), (uint64_t)h);
}

double rpfo_node_u(uint64_t key) { return (double)(rpfo_stream(key, 0) >> 11) * 0x1p-53; }

/* Direction `try` of the node with stream seed `key`: r[0..d). */
void rpfo_node_direction(uint64_t key, int try_i, int d, float *r)
{
    for (int j = 0; j < d; j++) {
        uint64_t sum = 0;
        for (int q = 0; q < 6; q++) {
            uint64_t w = rpfo_stream(key, 1 + 6 * ((uint64_t)try_i * (uint64_t)d + (uint64_t)j) + (uint64_t)q);
            sum += (w >> 32) + (w & 0xffffffffull);
        }
        r[j] = (float)((double)sum * 0x1p-32 - 6.0);
    }
}

typedef struct { int64_t heap; int depth; int64_t m; int32_t *idx; } unode_t;

/* Grow tree t by the uniform rule.  Outputs perm and leaf_of (leaf ordinals) of the tree;
 * returns the number of leaves.  *max_depth gets the depth of the deepest leaf.  When
 * node_heap is not NULL, every node where a split was attempted is listed (at most n of
 * them): heap id, (a, b, c), (size, left size, chosen try, depth). */
static int64_t grow_tree_uniform(const float *X, int64_t n, int d, uint64_t seed, int t, int n_try,
                                 int64_t n0, int32_t *perm, int32_t *leaf_of, int32_t *max_depth,
                                 int64_t *n_nodes, int64_t *node_heap, double *node_abc,
                                 int32_t *node_info)
{
    /* depth-first, left child first: leaves come off the stack in left-to-right order */
    unode_t *stack = (unode_t *)malloc(sizeof(unode_t) * (RPFO_UNIFORM_DEPTH + 2));
    int top = 0;
    int32_t *root = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) root[i] = (int32_t)i;
    stack[top++] = (unode_t){1, 0, n, root};
    float *Rnode = (float *)malloc((size_t)n_try * d * sizeof(float));
    double *P = (double *)malloc((size_t)n * sizeof(double));
    int64_t pos = 0, nleaf = 0, nn = 0;
    *max_depth = 0;
    while (top > 0) {
        unode_t W = stack[--top];
        int is_leaf = W.m <= n0 || W.depth >= RPFO_UNIFORM_DEPTH;
        int32_t *left = NULL, *right = NULL;
        int64_t nl = 0, nr = 0;
        if (!is_leaf) {
            uint64_t key = rpfo_node_key(seed, t, W.heap);
            for (int i = 0; i < n_try; i++) rpfo_node_direction(key, i, d, Rnode + (int64_t)i * d);
            int ch = which_projection(X, d, W.idx, W.m, Rnode, n_try, P);
            const float *r = Rnode + (int64_t)ch * d;
            for (int64_t k = 0; k < W.m; k++) P[k] = rpfo_canon_dot64(X + (int64_t)W.idx[k] * d, r, d);
            double a = P[0], b = P[0];
            for (int64_t k = 1; k < W.m; k++) {
                if (P[k] < a) a = P[k];
                if (P[k] > b) b = P[k];
            }
            double u = rpfo_node_u(key);
            double c = a + u * (b - a); /* three roundings: no contraction in this file */
            left = (int32_t *)malloc((size_t)W.m * sizeof(int32_t));
            right = (int32_t *)malloc((size_t)W.m * sizeof(int32_t));
            for (int64_t k = 0; k < W.m; k++) {
                if (P[k] < c) left[nl++] = W.idx[k];
                else right[nr++] = W.idx[k];
            }
            if (node_heap) {
                node_heap[nn] = W.heap;
                node_abc[3 * nn] = a;
                node_abc[3 * nn + 1] = b;
                node_abc[3 * nn + 2] = c;
                node_info[4 * nn] = (int32_t)W.m;
                node_info[4 * nn + 1] = (int32_t)nl;
                node_info[4 * nn + 2] = ch;
                node_info[4 * nn + 3] = W.depth;
            }
            nn++;
            if (nl == 0 || nr == 0) is_leaf = 1; /* an empty child: W stays whole */
        }
        if (is_leaf) {
            for (int64_t k = 0; k < W.m; k++) {
                perm[pos++] = W.idx[k];
                leaf_of[W.idx[k]] = (int32_t)nleaf;
            }
            nleaf++;
            if (W.depth > *max_depth) *max_depth = W.depth;
            free(left);
            free(right);
            free(W.idx);
            continue;
        }
        free(W.idx);
        stack[top++] = (unode_t){2 * W.heap + 1, W.depth + 1, nr, right};
        stack[top++] = (unode_t){2 * W.heap, W.depth + 1, nl, left};
    }
    if (n_nodes) *n_nodes = nn;
    free(P);
    free(Rnode);
    free(stack);
    return nleaf;
}

/* Alg. 3 forest growth with the uniform rule: T independent trees.  perm and leaf_of are
 * [T][n]; nleaf and max_depth [T]; the optional node lists are [T][n] slabs (node_abc
 * [T][n][3], node_info [T][n][4]) with n_nodes [T] entries used. */
void rpfo_build_uniform(const float *X, int64_t n, int d, int T, int n_try, int64_t n0, uint64_t seed,
                        int32_t *perm, int32_t *leaf_of, int32_t *nleaf, int32_t *max_depth,
                        int64_t *n_nodes, int64_t *node_heap, double *node_abc, int32_t *node_info)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < T; t++) {
        int64_t nn = 0;
        nleaf[t] = (int32_t)grow_tree_uniform(
            X, n, d, seed, t, n_try, n0, perm + (int64_t)t * n, leaf_of + (int64_t)t * n, max_depth + t, &nn,
            node_heap ? node_heap + (int64_t)t * n : NULL, node_abc ? node_abc + (int64_t)t * n * 3 : NULL,
            node_info ? node_info + (int64_t)t * n * 4 : NULL);
        if (n_nodes) n_nodes[t] = nn;
    }
}

/* Alg. 3 union and exact ranking over leaves given as ordinals: leaf_of [T][n] holds the
 * leaf ordinal of every point (its leaf's members sit together in perm [T][n]); query q
 * reaches leaf qleaf[t][q] of tree t.  Same outputs and conventions as rpfo_knn. */
void rpfo_knn_ordinal(const float *X, int64_t n, int d, int T, const int32_t *perm, const int32_t *leaf_of,
                      const float *Q, int64_t m, const int32_t *qleaf, const int64_t *self, int K,
                      int32_t *out_idx, double *out_dist)
{
    /* leaf ranges of every tree: a leaf's members are consecutive in perm */
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)T * (size_t)(n + 1));
    for (int t = 0; t < T; t++) {
        int64_t *st = start + (int64_t)t * (n + 1);
        int32_t prev = -1;
        int64_t nl = 0;
        for (int64_t pos = 0; pos < n; pos++) {
            int32_t lf = leaf_of[(int64_t)t * n + perm[(int64_t)t * n + pos]];
            if (lf != prev) {
                st[nl++] = pos;
                prev = lf;
            }
        }
        st[nl] = n;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < m; q++) {
        int64_t cap = 0;
        for (int t = 0; t < T; t++) {
            const int64_t *st = start + (int64_t)t * (n + 1);
            int32_t lf = qleaf[(int64_t)t * m + q];
            cap += st[lf + 1] - st[lf];
        }
        int32_t *u = (int32_t *)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(int32_t));
        int64_t nu = 0;
        for (int t = 0; t < T; t++) {
            const int64_t *st = start + (int64_t)t * (n + 1);
            int32_t lf = qleaf[(int64_t)t * m + q];
            for (int64_t pos = st[lf]; pos < st[lf + 1]; pos++) u[nu++] = perm[(int64_t)t * n + pos];
        }
        qsort(u, (size_t)nu, sizeof(int32_t), cmp_i32);
        cand_t *c = (cand_t *)malloc((size_t)(nu > 0 ? nu : 1) * sizeof(cand_t));
        int64_t nc = 0;
        for (int64_t k = 0; k < nu; k++) {
            if (k > 0 && u[k] == u[k - 1]) continue;
            if (self && self[q] == u[k]) continue;
            c[nc].idx = u[k];
            c[nc].D = rpfo_canon_dist64(Q + q * d, X + (int64_t)u[k] * d, d);
            nc++;
        }
        qsort(c, (size_t)nc, sizeof(cand_t), cmp_cand);
        for (int k = 0; k < K; k++) {
            out_idx[q * K + k] = k < nc ? c[k].idx : -1;
            out_dist[q * K + k] = k < nc ? sqrt(c[k].D) : INFINITY;
        }
        free(c);
        free(u);
    }
    free(start);
}

/* Number of OpenMP threads the oracle runs with (1 when built without OpenMP). */
int rpfo_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
