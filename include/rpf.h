/*
 * rpf.h -- C ABI of the rpForests kNN library for AMD MI355X (gfx950).
 *
 * kNN search by random projection forests (Yan, Wang, Wang, Wang, Li, arXiv 1812.11689):
 *   - rpf_build     grows an ensemble of T random projection trees over the points U
 *                   (Alg. 3, forest growth, with Alg. 1 and Alg. 2; median split of Sec. 2,
 *                   or the uniform split point that Alg. 1 prints);
 *   - rpf_all_knn   finds the K nearest neighbours of every point of U among the union
 *                   of its leaves (Alg. 3 search with Q = U);
 *   - rpf_query     lets external queries fall through every tree and searches the union
 *                   of the reached leaves (Alg. 3 search).
 *
 * Conventions for every entry point
 *   - Array arguments named *_dev are DEVICE pointers of the current HIP device; host
 *     pointers are named *_host.  Sizes are element counts.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued on it and
 *     the call returns without waiting, unless stated otherwise.  Device faults surface
 *     at a later call or at stream synchronisation as RPF_EDEVICE.
 *   - Every call returns an rpf_status; rpf_last_error() gives a message (thread-local).
 *     On an error, outputs are left untouched and *out handles are set to NULL.
 *   - No C++ exception crosses this boundary.
 *
 * Arithmetic (a reading of Sec. 2 / Alg. 1 / Alg. 3, which fix no arithmetic):
 *   - projection p = r.x in binary64: 32 partial sums by j mod 32 of exact binary32 x
 *     binary32 products, then a balanced adjacent-pair tree, then + 0.0;
 *   - split: members ordered by the key (p, original index); the floor(m/2) smallest go
 *     left; split value c = p of the member of rank floor(m/2);
 *   - neighbours are ranked by (D, index) with D the binary64 squared Euclidean distance
 *     (32 partial sums of fma(delta, delta, s), same tree); reported distances are
 *     (float)sqrt(D).
 */
#ifndef RPF_H
#define RPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RPF_OK = 0,
    RPF_EINVAL = -1,    /* invalid argument (sizes, null pointers, non-finite inputs)      */
    RPF_ENOMEM = -2,    /* the plan exceeds mem_budget_bytes, or a device allocation failed */
    RPF_EDEVICE = -3,   /* a HIP runtime or kernel error                                   */
    RPF_EBUSY = -4,     /* a serving queue is full                                          */
    RPF_ENOTREADY = -5, /* a polled request has not finished                                */
    RPF_EINTERNAL = -6  /* an internal invariant failed                                     */
} rpf_status;

/* Split point rule.
 * RPF_SPLIT_MEDIAN (Sec. 2): the member of rank floor(m/2) in (p, index) order splits the
 *   node; every tree has the same data-independent shape (rpf_depth).
 * RPF_SPLIT_UNIFORM (Alg. 1 as printed): c is drawn uniformly between a = min and b = max
 *   of the node's projections, c = RN(a + RN(u RN(b - a))) in binary64 with u in [0, 1);
 *   W_L = {p < c}, W_R = {p >= c}, both in ascending original index.  A node with an empty
 *   child (a = b, or c rounded onto a) stays whole as a leaf, so its leaf can hold more than
 *   leaf_size points; nodes at depth 62 are not split.  The random numbers come from the
 *   counter-based generator SplitMix64 (Steele, Lea, Flood 2014: output i of the stream with
 *   seed s is mix64(s + (i + 1) 0x9E3779B97F4A7C15)): node h (heap id, root 1) of tree t uses
 *   the stream whose seed is out(out(params.seed, t), h); its draw 0 gives
 *   u = (draw >> 11) 2^-53, and coordinate j of direction try i is the sum of the 32-bit
 *   halves of draws 1 + 6 (i d + j) + q, q = 0..5, times 2^-32, minus 6, rounded once to
 *   binary32.  directions_dev is not used.  Tree shapes depend on the data, so leaves are
 *   numbered per tree (ordinal in left-to-right order).  Uniform forests support rpf_all_knn,
 *   rpf_tree_dump (perm and leaf ordinals), rpf_tree_nodes, rpf_forest_info, rpf_free and
 *   rpf_last_knn_stats; rpf_build_batched, rpf_plan_create, rpf_query, rpf_route and the
 *   server return RPF_EINVAL for them. */
typedef enum { RPF_SPLIT_MEDIAN = 0, RPF_SPLIT_UNIFORM = 1 } rpf_split;

/* Precision of the candidate distance tiles (the MFMA Gram products).  Whatever the tile
 * precision, the returned neighbours are the exact top-K of the leaf union under the
 * binary64 ranking: tile distances only prune, with rigorous error bounds, and the
 * surviving candidates are re-ranked in binary32 and, near the K-th distance, binary64. */
typedef enum {
    RPF_DIST_FP32 = 0,
    RPF_DIST_BF16 = 1,
    RPF_DIST_FP16 = 2,
    RPF_DIST_BF16X3 = 3,
    RPF_DIST_U8GRID = 4
} rpf_dist_prec;
/* RPF_DIST_U8GRID: for points on the 1/255 grid (every coordinate is float(k) / 255.0f for
 * an integer k in [0, 255], as 8-bit image data scaled to [0, 1]); rpf_build returns
 * RPF_EINVAL otherwise.  The build keeps an int8 copy k - 128 of the points, and the
 * all-points tiles form the exact integer Gram product on the int8 MFMA: the grid distance
 * sum (k_a - k_b)^2 is exact, and the pruning bounds differ from it only by the binary32
 * rounding of k / 255, so almost every candidate is decided before the re-rank.  Like
 * RPF_DIST_BF16X3 the forest otherwise holds binary32 copies and norms, and rpf_query runs
 * the binary32 tiles (queries need not lie on the grid). */
/* RPF_DIST_BF16X3: the forest holds binary32 copies and norms (as RPF_DIST_FP32, and
 * rpf_query runs the binary32 tiles), but the all-points tiles split every centred binary32
 * value a into hi = bf16(a) and lo = bf16(a - hi) and form the Gram product on bfloat16
 * MFMA as hi.hi + hi.lo + lo.hi with binary32 accumulation; the omitted and rounded parts
 * (|a - hi - lo| <= 2^-16 |a|, |lo.lo| <= 2^-16 |a||b|) enter the pruning bounds, which stay
 * close to the binary32 ones. */

typedef struct rpf_forest rpf_forest; /* opaque; owns all of its device memory */

typedef struct {
    int32_t n_trees;     /* T >= 1 (Alg. 3, ensemble size)                                  */
    int32_t leaf_size;   /* n0 >= 1: a node is split iff it holds more than n0 points, so
                            every leaf holds at most n0 (Alg. 1, n_s = n0 + 1)              */
    int32_t n_try;       /* nTry >= 1 random directions per node, the one with the largest
                            spread of projections is used (Alg. 2); 1 = basic rpTree        */
    int32_t split_rule;  /* rpf_split                                                       */
    int32_t dist_prec;   /* rpf_dist_prec for the candidate tiles                           */
    int32_t build_flags; /* 0, or RPF_BUILD_SUBTREES (see below); the median rule only      */
    const float *directions_dev; /* random directions (Alg. 1 and Alg. 2), binary32
                            [n_trees][2^L - 1][n_try][d], row h-1 for heap node h (root 1,
                            children 2h, 2h+1), L = rpf_depth(n, leaf_size).  Required by the
                            median rule (ignored by the uniform rule); it is copied, so the
                            caller may free it once the build's work ends.                  */
    uint64_t mem_budget_bytes; /* 0 = unlimited; otherwise rpf_build fails with RPF_ENOMEM
                            when the forest's device memory would exceed it                 */
    uint64_t seed;       /* RPF_SPLIT_UNIFORM: key of the counter-based generator (any value);
                            ignored by the median rule                                      */
} rpf_params;

/* Build schedule (a performance choice only: the forest is bit-identical either way).
 * 0: level-synchronous, one launch group per level (levels paired so that one read of X
 *    serves two levels, where the shapes allow).
 * RPF_BUILD_SUBTREES: the levels from the first one whose nodes all fit one workgroup
 *    (at most 4096 members) down to the leaves run as ONE persistent launch: a fixed grid of
 *    resident workgroups takes (tree, node) items from a device counter and grows each
 *    item's whole subtree inside the workgroup, level by level, its permutation segment held
 *    in LDS.  Fewer launches and no global step between those levels, at the price of one
 *    read of X per level there.  Used only with n_try = 1 and at least two such levels;
 *    otherwise the flag is ignored.  rpf_plan_tune picks the schedule per part. */
#define RPF_BUILD_SUBTREES 1

/* Tree depth L = number of split levels for n points and leaf size n0 (host only). */
int32_t rpf_depth(int64_t n, int32_t leaf_size);

/* Grow the forest over X_dev (binary32 [n][d], row-major, finite values; copied).
 * n >= 1, d >= 1, n < 2^31.  On success *out owns the forest; free it with rpf_free. */
rpf_status rpf_build(const float *X_dev, int64_t n, int32_t d, const rpf_params *params,
                     void *stream, rpf_forest **out);

/* ---- Many independent data sets of the same dimension in one forest.
 *
 * X_dev holds the data sets one after the other (binary32 [sum n_i][d]); n_host[i] >= 1 is
 * the size of data set i.  Every data set gets its own T trees (same n_trees, leaf_size,
 * n_try, dist_prec), grown together with all the others, level by level, in the same
 * launches; leaves never mix data sets.  directions_dev is [n_trees][sum H_i][n_try][d] with
 * H_i = 2^L_i - 1, L_i = rpf_depth(n_i, leaf_size): row hbase_i + h - 1 is node h of data set
 * i, hbase_i = sum over j < i of H_j (rpf_batch_info gives it).  Each data set's forest is
 * exactly the forest rpf_build grows over it alone with its own rows of the directions.
 * rpf_all_knn on such a forest searches every point within its own data set and returns
 * indices within that data set; rpf_query and rpf_route return RPF_EINVAL.  In
 * rpf_tree_dump, split arrays are [sum H_i] (global node ids) and leaf_of holds global leaf
 * ids lbase_i + h. */
typedef struct {
    int64_t offset;          /* first point of the data set in X                            */
    int64_t n;
    int32_t depth;           /* L_i                                                         */
    int32_t reserved;
    int64_t heap_base;       /* hbase_i: global id of internal node h is hbase_i + h        */
    int64_t leaf_heap_base;  /* lbase_i: global id of leaf h is lbase_i + h                 */
} rpf_batch_entry;

rpf_status rpf_build_batched(const float *X_dev, const int64_t *n_host, int32_t count, int32_t d,
                             const rpf_params *params, void *stream, rpf_forest **out);
rpf_status rpf_batch_info(const rpf_forest *f, int32_t index, rpf_batch_entry *out_host);

/* ---- Build and all-points search of many data sets, recorded once and replayed.
 *
 * rpf_plan_create plans `count` data sets (sizes n_host, dimensions d_host; same n_trees,
 * leaf_size, n_try, dist_prec, K): they are grouped by dimension and each group is cut into
 * parts of at most max_part_points points (<= 0: 4 Mi; a data set is never split).  Every
 * part is one forest over its data sets, as rpf_build_batched grows it.  The plan allocates
 * every buffer -- per part the inputs X [rows][d] and directions [n_trees][n_nodes][n_try][d]
 * and the outputs [rows][K] (indices within each data set) -- and records, as one HIP graph,
 * part after part: the input checks, every level of every tree, the leaf pass, the
 * candidate stage (one workspace shared by all parts) and the index localisation (no
 * allocation, synchronisation or memset inside).  params->directions_dev is not used.
 *   rpf_plan_entry_of: where data set i lives (part, first row, first node of its trees);
 *   rpf_plan_part: the device buffers of part k, and its forest for introspection (owned by
 *     the plan; it reflects the last launch);
 *   rpf_plan_launch: runs the whole graph on `stream` (asynchronous; launches of one plan
 *     must not overlap); every launch rebuilds from the current buffer contents;
 *   rpf_plan_check: synchronises `stream`, reports non-finite inputs (RPF_EINVAL) or an
 *     internal error of the build kernels;
 *   rpf_plan_tune: launches once, then, per part, times and keeps the fastest of
 *     - the first-phase tree count (trees whose leaves are kept whole and set the pruning
 *       threshold): 2, 3, 4, 6 or 8;
 *     - the Phase II tile shape of the all-points symmetric tiles, bits of tile_shape:
 *       1 = the alternative k-chunk (binary32: 64 columns staged from X instead of 32
 *       loaded straight into LDS behind the previous chunk's MFMAs; 16-bit tiles: 64 (split
 *       bfloat16 32) columns instead of 128 (64)), 2 = queues of 256 candidate pairs per
 *       wave instead of 352-512, 4 = eight waves per block instead of twelve (leaves above
 *       128 points only);
 *     - the Phase II bucket size: the default (from K) or half of it;
 *     - the build schedule: level by level, or RPF_BUILD_SUBTREES;
 *     then records the graph again and enters the choices in the process's tuning table.
 *     No choice changes the results.
 *   The tuning table maps a part's shape (d, largest leaf, tile precision, K, T,
 *   floor(log2 rows)) to its choices; rpf_plan_create applies the entry of every part whose
 *   shape it holds.  rpf_tune_save writes it to a text file, one JSON object per line
 *   ({"d": .., "max_leaf": .., "prec": .., "K": .., "T": .., "n_log2": .., "first_trees": ..,
 *   "tile_shape": .., "bucket_size": .., "subtrees": ..}); rpf_tune_load merges such a file
 *   into the table (RPF_EINVAL, and the table unchanged, on a malformed line) and gives
 *   the entry count; rpf_tune_clear empties it.  Host only. */
typedef struct rpf_plan rpf_plan;

typedef struct {
    int32_t part, index_in_part, d, reserved;
    int64_t n;
    int64_t row;         /* first row of the data set in its part's X and outputs            */
    int64_t heap_base;   /* its internal node h is node heap_base + h of the part's trees    */
    int64_t n_nodes;     /* 2^L - 1 internal-node slots of each of its trees                 */
} rpf_plan_entry;

typedef struct {
    int64_t rows;
    int32_t d, n_sets;
    int64_t n_nodes;                 /* sum of n_nodes over the part's data sets             */
    float *X_dev;                    /* [rows][d]                                            */
    float *directions_dev;           /* [n_trees][n_nodes][n_try][d]                         */
    int32_t *out_idx_dev;            /* [rows][K]                                            */
    float *out_dist_dev;             /* [rows][K]                                            */
    const rpf_forest *forest;        /* not to be freed                                      */
    int32_t first_trees;             /* first-phase trees of its candidate stage             */
    int32_t tile_shape;              /* Phase II tile shape of its all-points tiles (below)  */
    int32_t bucket_size;             /* Phase II records per (row, tree) bucket, 0 = none    */
    int32_t subtrees;                /* 1: its small levels run as one persistent launch     */
} rpf_plan_part_info;

rpf_status rpf_plan_create(const int64_t *n_host, const int32_t *d_host, int32_t count, const rpf_params *params,
                           int32_t K, int32_t exclude_self, int64_t max_part_points, void *stream,
                           rpf_plan **out);
rpf_status rpf_plan_info(const rpf_plan *plan, int32_t *n_parts_host, int32_t *count_host);
rpf_status rpf_plan_part(const rpf_plan *plan, int32_t part, rpf_plan_part_info *out_host);
rpf_status rpf_plan_entry_of(const rpf_plan *plan, int32_t index, rpf_plan_entry *out_host);
rpf_status rpf_plan_launch(rpf_plan *plan, void *stream);
rpf_status rpf_plan_check(rpf_plan *plan, void *stream);
rpf_status rpf_plan_tune(rpf_plan *plan, void *stream, double *tuned_ms_host);
rpf_status rpf_tune_save(const char *path);
rpf_status rpf_tune_load(const char *path, int32_t *entries_host);
rpf_status rpf_tune_clear(void);
rpf_status rpf_plan_destroy(rpf_plan *plan);

/* Internal faults of the search.  The final merge checks every candidate index it takes
 * from its pruning buffers against [0, n); a row that meets one outside is recomputed by
 * the exhaustive scan (its output stays correct) and counted on the forest, for good (the
 * count is never cleared).  Once the count is nonzero, rpf_all_knn, rpf_query and
 * rpf_server_submit on that forest return RPF_EINTERNAL, and so do the serving batches,
 * rpf_last_knn_stats, rpf_forest_info and rpf_plan_check.  Since searches are asynchronous,
 * the count reaches the host by a copy enqueued behind each search: a fault is reported by
 * the first of those calls made after that copy has run (with RPF_SYNC_CHECK=1 in the
 * environment every launch is synchronised and the faulting call reports it itself).
 *
 * All-points kNN (Alg. 3 with Q = U): out_idx_dev int32 [n][K], out_dist_dev float [n][K].
 * exclude_self = 1 drops each point from its own candidate set.  1 <= K <= n - exclude_self.
 * Rows shorter than K (|N_q| < K) are padded with (-1, +inf).
 * Device workspace is taken from the library's cache for the call: about n x (16 B x the
 * per-row record capacity), where the capacity grows with K x n_trees.  Once that passes
 * one wave's 768 records, the buffers take up to 4096 records per row while all rows fit
 * 32 GiB (for example about 25 GB at n = 10^6, K 20, 80 trees).  A failed allocation
 * returns RPF_ENOMEM. */
rpf_status rpf_all_knn(const rpf_forest *f, int32_t K, int32_t exclude_self,
                       int32_t *out_idx_dev, float *out_dist_dev, void *stream);

/* External queries (Alg. 3 search): Q_dev binary32 [m][d] (finite), m >= 0,
 * 1 <= K <= n.  Outputs [m][K] as for rpf_all_knn. */
rpf_status rpf_query(const rpf_forest *f, const float *Q_dev, int64_t m, int32_t K,
                     int32_t *out_idx_dev, float *out_dist_dev, void *stream);

/* rpf_query for callers that cannot allocate device memory: code in a serving loop that
 * must not call hipMalloc / hipFree, or a harness that forbids them.  Same arguments,
 * results and errors as rpf_query; the call allocates nothing.  Its workspace is carved
 * from a fixed scratch area of 256 MiB that the library holds on each device it runs on
 * until the process ends.
 *   - RPF_EINVAL when m queries at this K need more workspace than the scratch area
 *     (rpf_query_workspace_bytes gives the need; about 1 000 to 2 000 queries of K 100 over
 *     64 trees of 256-point leaves fit, many more at small K): split the batch.
 *   - RPF_ENOTREADY when the forest's leaf-ordered query copies do not exist yet: they are
 *     made (allocated) by the forest's first rpf_query call or by rpf_server_create, or at
 *     build time when leaves exceed 256 points.
 *   - Every call on a device shares that device's scratch area and leaves its contents
 *     behind: calls whose work overlaps on one device (other threads, other streams with
 *     no ordering between them) race and corrupt each other's results.  Order them, e.g. on
 *     one stream, or synchronise between them.  Like rpf_query, the call synchronises
 *     `stream` twice (input check, tile counts); its last kernels are still queued when it
 *     returns. */
rpf_status rpf_query_noalloc(const rpf_forest *f, const float *Q_dev, int64_t m, int32_t K,
                             int32_t *out_idx_dev, float *out_dist_dev, void *stream);

/* Exact kNN by brute force (the problem the forest approximates; the ground truth of the
 * accuracy measures of Sec. 5.1): for each query row of Q_dev (binary32 [m][d]) the K points
 * of X_dev (binary32 [n][d], finite) of smallest key (D, index), D the canonical binary64
 * squared distance (the library's ranking), written as out_idx_dev int32 [m][K] and
 * out_dist_dev float [m][K] = (float)sqrt(D), ascending.  self_dev (optional, int64 [m]):
 * point index to leave out of query i's candidates (its own row in X), or -1; rows with
 * fewer than K candidates are padded with (-1, +inf).  1 <= K <= 256, 1 <= d <= 2048,
 * 1 <= n < 2^31.  Device workspace: one binary64 distance row per query of a chunk, at
 * most 4 GiB.  Synchronises `stream` once (input check). */
rpf_status rpf_exact_knn(const float *X_dev, int64_t n, int32_t d, const float *Q_dev, int64_t m,
                         const int64_t *self_dev, int32_t K, int32_t *out_idx_dev, float *out_dist_dev,
                         void *stream);

/* Route queries only (Alg. 3 descent): out_leaf_dev int32 [T][m] = heap id of the leaf
 * each query reaches in each tree (right child iff projection >= split value). */
rpf_status rpf_route(const rpf_forest *f, const float *Q_dev, int64_t m, int32_t *out_leaf_dev,
                     void *stream);

/* Release the forest.  rpf_free(NULL) is a no-op returning RPF_OK.  Synchronises the
 * device before freeing. */
rpf_status rpf_free(rpf_forest *f);

/* Introspection for parity tests.  Tree t in [0, T).  Device outputs:
 *   split_dev double [2^L-1], split_idx_dev int32 [2^L-1], chosen_dev int32 [2^L-1]
 *   (NaN / -1 / -1 where the heap slot is not an internal node), perm_dev int32 [n] (the
 *   leaves left to right, members ascending), leaf_of_dev int32 [n] (heap id of the leaf
 *   holding each point; for a uniform-rule forest, the leaf's ordinal in left-to-right
 *   order).  Any output pointer may be NULL; a uniform-rule forest has no split arrays
 *   (RPF_EINVAL unless split_dev, split_idx_dev and chosen_dev are NULL). */
rpf_status rpf_tree_dump(const rpf_forest *f, int32_t tree, double *split_dev,
                         int32_t *split_idx_dev, int32_t *chosen_dev, int32_t *perm_dev,
                         int32_t *leaf_of_dev, void *stream);

/* The nodes of a uniform-rule tree where a split was attempted (host output, at most n of
 * them per tree, listed level by level): heap id, split value c, size, left size (0 or
 * size: the node stayed whole as a leaf), the direction try chosen by Alg. 2, and depth.
 * count_host gets the number of nodes; at most cap records are written.  RPF_EINVAL for a
 * median-rule forest (its split arrays come from rpf_tree_dump).  Host only. */
typedef struct {
    int64_t heap;
    double split;
    int32_t size, left, chosen, depth;
} rpf_node;

rpf_status rpf_tree_nodes(const rpf_forest *f, int32_t tree, rpf_node *out_host, int64_t cap,
                          int64_t *count_host);

typedef struct {
    int64_t n;               /* points (all data sets of a batched forest)                  */
    int32_t d, n_trees, leaf_size, n_try;
    int32_t depth;           /* split levels (uniform rule: depth of the deepest leaf)       */
    int32_t dist_prec;
    int64_t n_leaves;        /* leaves per tree (uniform rule: of the tree with the most)    */
    uint64_t device_bytes;   /* device memory owned by the forest                           */
    int32_t batch_count;     /* data sets (1 unless built by rpf_build_batched)             */
    int32_t split_rule;      /* rpf_split the forest was grown with                         */
} rpf_info;

rpf_status rpf_forest_info(const rpf_forest *f, rpf_info *out_host);

/* Counters of the last rpf_all_knn / rpf_query on this forest (host, synchronises the
 * stream): rows that fell back to the exhaustive candidate scan because a pruning buffer
 * overflowed, the total number of candidates re-ranked in binary32 / binary64, and the
 * candidate records that reached the final merge (kept from the first trees' leaves, and
 * emitted by the remaining trees below the row's threshold; rows that overflowed count
 * what they attempted), and the rows whose records outgrew the one-wave final merge and were
 * merged by a whole block instead (their results are exact either way).
 * Returns RPF_EINTERNAL when the last call met a candidate index outside [0, n) in its
 * pruning buffers (an internal error: such rows are recomputed by the exhaustive scan,
 * never dereferenced, so the outputs stay correct). */
typedef struct {
    int64_t rows, fallback_rows, reranked32, reranked64;
    int64_t first_phase_kept, second_phase_emitted;
    int64_t block_merged_rows;
} rpf_knn_stats;

rpf_status rpf_last_knn_stats(const rpf_forest *f, rpf_knn_stats *out_host, void *stream);

/* Per-kernel timing with HIP events recorded on the launch stream around every kernel
 * of the library (off by default).  rpf_profile_read copies up to `cap` records. */
typedef struct {
    char name[48];
    int64_t launches;
    double total_ms;
    double algo_bytes;  /* algorithmic bytes moved by these launches (see each kernel) */
    double algo_flops;  /* algorithmic flops of these launches                          */
} rpf_profile_record;

rpf_status rpf_profile_enable(int32_t on);
rpf_status rpf_profile_reset(void);
rpf_status rpf_profile_read(rpf_profile_record *out_host, int32_t cap, int32_t *count);

/* Device bytes one rpf_query call of m queries with this K takes for its workspace (an
 * estimate from above, host only; the serving loop admits batches by it). */
rpf_status rpf_query_workspace_bytes(const rpf_forest *f, int64_t m, int32_t K, uint64_t *bytes_host);

/* ---- Serving loop: continuous batching of query requests over a resident forest.
 *
 * Requests (m query rows, K; Alg. 3 search) are queued by rpf_server_submit and served by
 * `slots` worker threads, each with its own HIP stream.  A free slot takes the oldest
 * waiting request together with every later waiting request of the same K, up to
 * max_batch_rows rows in all, and runs them as one rpf_query batch; requests arriving while
 * batches run wait for the next free slot.  A batch is admitted only while the workspace
 * bytes of the batches in flight (rpf_query_workspace_bytes plus staging) stay within
 * mem_budget_bytes (0 = unlimited); a batch that alone exceeds it still runs when nothing
 * else does.  Each request's result is exactly what rpf_query gives for it alone.
 *
 * Ownership: Q_dev, out_idx_dev and out_dist_dev belong to the caller and must stay valid
 * until the request is collected by rpf_server_poll (done = 1) or rpf_server_wait.  Q_dev
 * is read after the work already queued on the submitting `stream` (an event orders it);
 * the outputs hold the result once the request is collected.  The forest must outlive the
 * server.  All server calls are thread-safe.  Latency = from the submit call to the
 * completion of the request's batch. */
typedef struct rpf_server rpf_server;

typedef struct {
    int32_t slots;            /* worker threads / streams, 1..16                            */
    int32_t reserved;         /* must be 0                                                  */
    int64_t max_batch_rows;   /* rows of one batch (a single larger request runs alone)     */
    int64_t max_queue;        /* waiting requests; rpf_server_submit returns RPF_EBUSY above */
    uint64_t mem_budget_bytes;
} rpf_server_config;

typedef struct {
    int64_t requests, rows, batches;    /* completed since creation or the last reset */
    double mean_batch_rows;
    double p50_s, p99_s, max_s;         /* request latency percentiles (seconds)      */
    double rows_per_s;                  /* rows completed / (last completion - first submit) */
    int64_t failed_requests;            /* requests that ended with an error status   */
    int64_t bad_index_rows;             /* the forest's internal-fault count (see
                                           rpf_all_knn); 0 unless the library is wrong   */
} rpf_server_report;

rpf_status rpf_server_create(const rpf_forest *f, const rpf_server_config *cfg, rpf_server **out);
/* Non-blocking.  RPF_EBUSY when max_queue requests are waiting; RPF_EINVAL for m < 1 or K
 * outside [1, min(n, 256)].  *ticket_host identifies the request. */
rpf_status rpf_server_submit(rpf_server *srv, const float *Q_dev, int64_t m, int32_t K, int32_t *out_idx_dev,
                             float *out_dist_dev, void *stream, uint64_t *ticket_host);
/* RPF_ENOTREADY (done = 0) while the request runs; once done (done = 1) the request's own
 * status is returned and the ticket is released. */
rpf_status rpf_server_poll(rpf_server *srv, uint64_t ticket, int32_t *done_host, double *latency_s_host);
/* Blocks until the request is done; returns its status and releases the ticket. */
rpf_status rpf_server_wait(rpf_server *srv, uint64_t ticket, double *latency_s_host);
rpf_status rpf_server_stats(rpf_server *srv, rpf_server_report *out_host);
/* Device-side span of each batch since creation or the last reset (at most the first 65536):
 * HIP events recorded on the slot's stream before the batch's first launch and after its
 * last, in milliseconds after an event completed when the server was created.  Spans of
 * batches on different slots that intersect show their work in flight on the device at the
 * same time.  Copies up to `cap` records; *count_host = records held.  A span the events
 * could not time holds -1. */
typedef struct {
    int32_t slot, requests;
    int64_t rows;
    double start_ms, end_ms;
} rpf_server_batch;

rpf_status rpf_server_batch_log(rpf_server *srv, rpf_server_batch *out_host, int32_t cap, int32_t *count_host);
rpf_status rpf_server_reset_stats(rpf_server *srv);
/* Serves every waiting request, stops the workers and frees the server (NULL: no-op).
 * Requests not collected are released with it. */
rpf_status rpf_server_destroy(rpf_server *srv);

/* Device memory of forests and of the per-call kNN workspaces comes from a cache kept by
 * the library: blocks obtained from hipMalloc are reused by later calls (a block last used
 * on another stream is ordered behind that use by an event) and are not returned to the
 * runtime when a forest is freed.  This call hipFree's every idle cached block of `device`
 * (device < 0: of every device); blocks in use by live forests or running calls stay.  The
 * cache also empties itself once when an allocation fails, before it reports RPF_ENOMEM. */
rpf_status rpf_release_cached_memory(int32_t device);

const char *rpf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RPF_H */
