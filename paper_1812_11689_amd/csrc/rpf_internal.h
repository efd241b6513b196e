// Internal declarations of the rpForests HIP library (gfx950, wave64).
//
// Canonical arithmetic (the library's reading of Sec. 2 / Alg. 3, which fix no order):
//   projection  p = r.x : 32 partial sums s_c over j = c (mod 32), j ascending, of the exact
//               binary64 products (double)x_j*(double)r_j; a balanced adjacent-pair tree over
//               s_0..s_31; + 0.0.
//   distance    D = |a-b|^2 : the same 32 classes with s_c <- fma(delta, delta, s_c),
//               delta = a_j - b_j rounded in the working precision (binary64 or binary32).
//   sums        canon_sum(v[0..m)) : v padded with +0.0 to a power of two, adjacent pairs
//               added level by level.
// On the GPU eight lanes share one vector: lane g in [0,8) owns classes 4g..4g+3, reads
// the float4 at j = 32k + 4g, and the tree is (s0+s1)+(s2+s3) inside the lane followed by
// butterflies over lane distance 1, 2, 4 -- the same tree, operation for operation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rpf.h"
#include "merge_index.h"

namespace rpf {

constexpr int kLarge = 4096;      // segments above this size use the multi-block path
constexpr int kChunk = 4096;      // positions per block on the multi-block path (power of 2)
constexpr int kDigitBits = 11;    // radix digit of the multi-block median select
constexpr int kDigitBins = 1 << kDigitBits;
constexpr int kNumDigits = 9;     // 96-bit key (p, index): 8 digits of 11 bits + 1 of 8
constexpr int kCandCap = 1024;    // candidates gathered for the final in-block select

// ---------------------------------------------------------------- descriptors

struct SegDesc {      // one internal node of a level (same shape for every tree)
    int64_t off;      // first position in the node-ordered permutation
    int32_t size;     // number of members m
    int32_t heap;     // heap id h (root 1)
    int32_t chunk0;   // multi-block path: first chunk of this segment
    int32_t nchunk;   // multi-block path: number of chunks
};

struct ChunkDesc {
    int64_t start;    // first position
    int32_t len;      // <= kChunk
    int32_t seg;      // segment index within the level
};

struct LeafDesc {
    int64_t off;      // first position of the leaf in the permutation
    int32_t size;
    int32_t heap;
};

// multi-block median select state, one per (tree, segment)
enum : int32_t { SEL_HIST = 0, SEL_COMPACT = 1, SEL_GATHERED = 2, SEL_DONE = 3 };

struct SelState {
    uint64_t pfx_hi;   // prefix of the 96-bit key found so far (top nbits valid)
    uint32_t pfx_lo;
    int32_t nbits;
    int64_t rank;      // rank of the target among the keys that match the prefix
    int64_t cnt;       // number of keys that match the prefix
    int32_t mode;
    int32_t chosen;    // chosen try (Alg. 2)
    double best_s2;    // Alg. 2 running best spread
    double s1;         // Alg. 2 scratch: sum of projections of the current try
    int32_t counted;   // 1: the final step filled the partition's left counts of the chunks
    int32_t pad;
};

struct Ent {           // one pruning candidate: point index and bounds on its squared distance
    int32_t idx;
    float lb;
    float ub;
    int32_t pad;
};


struct LatNorm {       // a point on the 1/255 grid: |k - 128|^2 (exact) and |k| / 255
    int32_t na;
    float ra;
};

struct Cand {          // a key gathered for the in-block median select
    uint64_t hi;
    uint32_t lo;
    uint32_t pad;
};

struct LookDesc {     // the children of one internal node, for projections made a level ahead
    int32_t child_seg[2];   // index among the next level's internal nodes, -1 for a leaf
    int32_t child_heap[2];  // heap ids of the children that are internal nodes, else 0
};

// Two levels from one read of X (one direction per node): the lead level projects every row
// onto its node's direction and onto both children's, and its partition hands each row the
// projection onto the child it moves into, as that level's key at its new position; the fed
// level below starts from those keys and never reads X.
struct LevelLink {
    const LookDesc *look = nullptr;   // lead: per internal node of the level (null: not a lead)
    double2 *ahead = nullptr;         // lead: [T][n] projections onto the two children, by position
    uint64_t *keys_next = nullptr;    // lead: [T][n] keys of the fed level, by its positions
    uint32_t *hist_next = nullptr;    // lead above a multi-block level: its digit-0 histograms
    int nseg_next = 0;
    const uint64_t *keys_in = nullptr;  // fed: keys made by the lead (null: project)
    uint32_t *hist_in = nullptr;        // fed multi-block level: histograms made by the lead
    bool roots = false;  // lead at the roots (identity permutation): one read of X for all trees
    // grid forests: the projections read each row from the int8 copy (k - 128, stride dq)
    // instead of X, a quarter of the bytes for the same binary32 values
    const int8_t *xq = nullptr;
    int dq = 0;
};

struct SubItem {       // an internal node at the first level of the persistent subtree launch
    int64_t off;      // first position in the node-ordered permutation
    int32_t size;     // members (at most the one-block segment size)
    int32_t heap;     // heap id, global (hbase + id within its data set)
    int32_t hbase;    // the data set's first heap slot (0 for a single data set)
    int32_t pad;
};

size_t subtree_lds(int max_m, int d);
void launch_subtree(hipStream_t s, bool vec, const float *X, int d, const float *R, int64_t H, const SubItem *items,
                    int nitems, int T, int n0, const int32_t *pin, int32_t *pout, int64_t n, double *split,
                    int32_t *split_idx, int32_t *chosen, int32_t *err, uint32_t *next, int max_m, int lds_limit);

struct LargeBufs {     // temporaries of the multi-block level path (and of the level links)
    uint64_t *keys;
    uint64_t *keys2;      // keys made one level ahead
    uint32_t *hist2;      // their digit-0 histograms
    double2 *ahead;       // projections onto the children, by position
    double *praw;
    SelState *state;
    uint32_t *hist;
    Cand *cand;
    uint32_t *cand_cnt;
    uint32_t *lcount;
    double *part;
};

struct TileJob {       // one MFMA tile: A rows x B rows (<= 32*MB each) of one tree
    int64_t a_off;     // first A row (position in the per-tree A arrays)
    int64_t b_off;     // first B row (position in the per-tree leaf-ordered arrays)
    int32_t a_rows;
    int32_t b_rows;
    int32_t tree;
    int32_t same;      // 1: A and B are the same positions (all-points diagonal tile)
    int32_t b_pos;     // offset of the first B row inside its leaf
    int32_t leaf_m;    // size of the leaf the B rows belong to
    int32_t leaf;      // index of that leaf (its centroid row)
    int32_t pad;
};

// read-only view of a forest for the kNN launchers
struct ForestView {
    int64_t n, H;
    int d, T, n0, n_try, L, prec, dp, max_leaf, job_mb;
    int sym_prec;  // precision of the all-points tiles (prec, split bfloat16 or the int8 grid over binary32)
    const int8_t *Xq;     // grid forests: [n][dq] k - 128 (zero past d)
    const LatNorm *qn;    // grid forests: [n]
    int dq;
    const float *X, *R, *centroid;
    const double *split;
    const int32_t *chosen, *perm, *leaf_of, *heap_leaf;
    const void *Xc;
    const float2 *nrm;
    const LeafDesc *leaves;
    int64_t nleaf;
    const TileJob *jobs;
    int64_t n_jobs_tree;
    double tile_flops_tree;  // useful Gram flops of one tree's all-points tiles
    unsigned long long *stats;
    unsigned long long *fault;  // sticky count of rows that met an out-of-range candidate index
    // uniform-rule forests: every tree has its own leaves.  The leaf table is [T][leaf_stride]
    // (nleaf == leaf_stride, unused entries of a tree have size 0), leaf_of holds ordinals
    // within the tree and heap_leaf is the identity; tree t's all-points tiles are
    // jobs[job_off[t], job_off[t + 1]) and flops_off[t] is the useful Gram flops of the trees
    // before t (host arrays of T + 1 entries).  Median-rule forests: leaf_stride 0 (one table
    // for every tree), job_off and flops_off null.
    int64_t leaf_stride;
    const int64_t *job_off;
    const double *flops_off;
};
ForestView view(const rpf_forest *f);
// internal-fault counter of a forest: the host mirror (no synchronisation; it lags the device
// by the work still queued), its refresh (an asynchronous copy enqueued on s), and a read of
// the device counter itself (synchronises s)
uint64_t forest_fault_seen(const rpf_forest *f);
void forest_fault_mirror(const rpf_forest *f, hipStream_t s);
uint64_t forest_fault_read(const rpf_forest *f, hipStream_t s);
rpf_status fault_error(const rpf_forest *f, const char *who);
rpf_status search_tail(const rpf_forest *f, hipStream_t s, const char *who);
bool sync_check_on();  // RPF_SYNC_CHECK=1: every launch is followed by a synchronisation

// entry points of the search (knn_kernels.hip), shared by the C ABI and the server
rpf_status knn_all(const rpf_forest *f, int K, int exclude_self, int32_t *out_idx, float *out_dist, hipStream_t s);
rpf_status knn_query(const rpf_forest *f, const float *Q, int64_t m, int K, int32_t *out_idx, float *out_dist,
                     hipStream_t s);
rpf_status route(const rpf_forest *f, const float *Q, int64_t m, int32_t *out_leaf, hipStream_t s);
uint64_t query_workspace_bytes(const rpf_forest *f, int64_t m, int K);
// all-points search of several forests (parts) sharing one persistent workspace (recordable
// launches); maxB[i] bounds the first-phase tree count part i will be launched with
struct KnnShared;
KnnShared *knn_shared_create(const std::vector<const rpf_forest *> &parts, const std::vector<int> &maxB, int K,
                             int exclude_self, hipStream_t s);
int knn_part_first_trees(const rpf_forest *f, int K, int B);
int knn_part_shape_mask(const rpf_forest *f, int K);
int knn_part_bucket_size(const rpf_forest *f, int K, int B);
void knn_part_launch(const KnnShared *p, const rpf_forest *f, int B, int shape, int bucket_S, int32_t *out_idx,
                     float *out_dist, hipStream_t s);
void knn_shared_destroy(KnnShared *p, hipStream_t s);
void fill_u32(void *p, int64_t count, uint32_t value, hipStream_t s);
void fill_u64(void *p, int64_t count, uint64_t value, hipStream_t s);
// the leaf-ordered, centred copy in the tile precision, made on a query's first use (the
// all-points search of leaves that fit one tile stages its rows from X instead)
// (may_make = false: RPF_ENOTREADY instead of allocating them when they do not exist yet)
rpf_status ensure_leaf_copies(const rpf_forest *f, hipStream_t s, bool may_make = true);
// copies tree 0's all-points tiles (jobs[0, njt)) to trees 1 .. T - 1
void replicate_jobs(TileJob *jobs, int64_t njt, int T, hipStream_t s);
int64_t forest_points(const rpf_forest *f);
int32_t forest_dim(const rpf_forest *f);
int32_t forest_batch_count(const rpf_forest *f);
bool forest_uniform(const rpf_forest *f);  // grown by the uniform split rule (leaves per tree)

bool capturing(hipStream_t s);  // a stream capture (graph recording) is active on s
rpf_status fail(rpf_status st, const std::string &msg);
rpf_status check_hip(hipError_t e, const char *what);
void launch_nonfinite(hipStream_t s, const float *x, int64_t count, int32_t *flag);
// records the first failing launch of the calling thread (name + HIP error); with
// RPF_SYNC_CHECK=1 in the environment it also synchronises after every launch
void launch_check(hipStream_t s, const char *name);
// caching device allocator (device_cache.hip): blocks stay with the library and are reused;
// a block returned on one stream is safe to hand to another (event-ordered)
constexpr int kStatSlots = 64;  // kNN counters: [kStatSlots][8] unsigned 64-bit, summed on the host
void *cache_alloc(size_t bytes, hipStream_t s);  // nullptr when the device is out of memory
void cache_free(void *p, hipStream_t s);          // p's last use is the work queued on s
void cache_free_idle(void *p);                    // p has no work queued or running (after a synchronisation)
uint64_t cache_held_bytes(int dev);
void cache_release(int dev);                      // hipFree idle blocks (dev < 0: every device)
std::string take_launch_error();

// ---------------------------------------------------------------- uniform split rule (uniform_kernels.hip)

constexpr int kUniformDepth = 62;  // nodes this deep are not split (heap ids below 2^63)

struct UniSeg {        // one open node of a level of the uniform-rule growth
    int64_t pos;       // first position in the [T][n] permutation (tree * n + offset)
    int64_t heap;      // heap id within its tree (root 1)
    int32_t size;
    int32_t tree;
    int32_t chunk0;    // chunked path: first chunk of the node
    int32_t nchunk;
};

struct UniChunk {
    int64_t pos;       // first position in the [T][n] permutation
    int32_t len;       // <= kChunk
    int32_t seg;       // node index within the chunked list
};

struct UniSplit {      // the split of one node
    double c;          // split value
    int32_t nl;        // left size (0 or the node's size: the node stays whole)
    int32_t chosen;    // direction try (Alg. 2)
};

struct UniBufs {       // temporaries of the chunked path
    double *P = nullptr;        // [n_try][T n] projections
    double *part = nullptr;     // [chunks][n_try] partial canonical sums
    double2 *mm = nullptr;      // [chunks][n_try] (min, max)
    double *mu = nullptr;       // [nodes][n_try] means
    uint32_t *lcount = nullptr; // [chunks] left members
    uint32_t *loff = nullptr;   // [chunks] left members of the node before the chunk
    int32_t *tmp = nullptr;     // [T n] scratch permutation
};

size_t uni_block_lds(int max_m, int d, int n_try);
void launch_uni_block(hipStream_t s, const float *X, int d, int n_try, uint64_t seed, const UniSeg *segs, int nseg,
                      int max_m, int32_t *perm, UniSplit *out);
void launch_uni_chunked(hipStream_t s, const float *X, int d, int n_try, uint64_t seed, const UniSeg *segs, int nseg,
                        const UniChunk *chunks, int nchunk, int32_t *perm, int64_t TN, const UniBufs &b,
                        UniSplit *out);

// ---------------------------------------------------------------- order-preserving keys

__host__ __device__ inline uint64_t key_of(double p) {
    uint64_t b;
    __builtin_memcpy(&b, &p, 8);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__host__ __device__ inline double val_of(uint64_t u) {
    uint64_t b = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
    double p;
    __builtin_memcpy(&p, &b, 8);
    return p;
}

__device__ inline bool key_less(uint64_t hi, uint32_t lo, uint64_t phi, uint32_t plo) {
    return hi < phi || (hi == phi && lo < plo);
}

__device__ inline unsigned __int128 key96(uint64_t hi, uint32_t lo) {
    return ((unsigned __int128)hi << 32) | lo;
}

// ---------------------------------------------------------------- wave helpers

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

__device__ inline int mask_rank(uint64_t mask) {  // set bits of mask below this lane
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

__device__ inline double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }
__device__ inline float shfl_xor_f(float v, int m) { return __shfl_xor(v, m, 64); }

// exclusive scan over a 256-thread block (4 waves); s_w needs 4 words
__device__ inline void block_excl_scan256(uint32_t v, uint32_t *s_w, uint32_t &excl, uint32_t &total) {
    // 256 threads = 4 waves
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint32_t wb = 0, tot = 0;
    for (int k = 0; k < 4; k++) {
        uint32_t c = s_w[k];
        if (k < w) wb += c;
        tot += c;
    }
    excl = wb + x - v;
    total = tot;
    __syncthreads();
}

// exclusive scan over a block of NW waves; s_w needs NW words
template <int NW>
__device__ inline void block_excl_scan_w(uint32_t v, uint32_t *s_w, uint32_t &excl, uint32_t &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint32_t wb = 0, tot = 0;
    for (int k = 0; k < NW; k++) {
        uint32_t c = s_w[k];
        if (k < w) wb += c;
        tot += c;
    }
    excl = wb + x - v;
    total = tot;
    __syncthreads();
}

// ---------------------------------------------------------------- canonical arithmetic

// canon_sum over s[0..m) in place by the whole block (s has room for the power-of-two
// padding P2 >= m); every thread returns the sum
__device__ inline double block_canon_sum(double *s, int m) {
    int P2 = 1;
    while (P2 < m) P2 <<= 1;
    for (int i = m + threadIdx.x; i < P2; i += blockDim.x) s[i] = 0.0;
    __syncthreads();
    for (int h = 1; h < P2; h <<= 1) {
        for (int i = 2 * h * threadIdx.x; i < P2; i += 2 * h * blockDim.x) s[i] = s[i] + s[i + h];
        __syncthreads();
    }
    double r = s[0];
    __syncthreads();
    return r;
}

// Projection of row x onto r (r usually staged in LDS) by an aligned group of 8 lanes;
// every lane of the group returns p.  VEC: d % 4 == 0 and x, r 16-byte aligned.
template <bool VEC>
__device__ inline double group8_dot64(const float *__restrict__ x, const float *__restrict__ r,
                                      int d, int g) {
    // the product of two binary32 values is exact in binary64, so fma(x, r, s) rounds once,
    // exactly as s + x * r does
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (VEC) {
        for (int j = 4 * g; j < d; j += 32) {
            float4 xv = *reinterpret_cast<const float4 *>(x + j);
            float4 rv = *reinterpret_cast<const float4 *>(r + j);
            s0 = __builtin_fma((double)xv.x, (double)rv.x, s0);
            s1 = __builtin_fma((double)xv.y, (double)rv.y, s1);
            s2 = __builtin_fma((double)xv.z, (double)rv.z, s2);
            s3 = __builtin_fma((double)xv.w, (double)rv.w, s3);
        }
    } else {
        for (int j = 4 * g; j < d; j += 32) {
            s0 = __builtin_fma((double)x[j], (double)r[j], s0);
            if (j + 1 < d) s1 = __builtin_fma((double)x[j + 1], (double)r[j + 1], s1);
            if (j + 2 < d) s2 = __builtin_fma((double)x[j + 2], (double)r[j + 2], s2);
            if (j + 3 < d) s3 = __builtin_fma((double)x[j + 3], (double)r[j + 3], s3);
        }
    }
    double v = (s0 + s1) + (s2 + s3);
    v = v + shfl_xor_d(v, 1);
    v = v + shfl_xor_d(v, 2);
    v = v + shfl_xor_d(v, 4);
    return v + 0.0;
}

// Projections of two rows xa, xb onto one direction r (binary32, usually in LDS) from one
// pass, the loads of both rows in flight together; each equals group8_dot64's bit for bit.
template <bool VEC>
__device__ inline void group8_dot64r2(const float *__restrict__ xa, const float *__restrict__ xb,
                                      const float *__restrict__ r, int d, int g, double &pa, double &pb) {
    double s[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    if (VEC) {
        for (int j = 4 * g; j < d; j += 32) {
            const float4 va = *reinterpret_cast<const float4 *>(xa + j);
            const float4 vb = *reinterpret_cast<const float4 *>(xb + j);
            const float4 rv = *reinterpret_cast<const float4 *>(r + j);
            s[0][0] = __builtin_fma((double)va.x, (double)rv.x, s[0][0]);
            s[0][1] = __builtin_fma((double)va.y, (double)rv.y, s[0][1]);
            s[0][2] = __builtin_fma((double)va.z, (double)rv.z, s[0][2]);
            s[0][3] = __builtin_fma((double)va.w, (double)rv.w, s[0][3]);
            s[1][0] = __builtin_fma((double)vb.x, (double)rv.x, s[1][0]);
            s[1][1] = __builtin_fma((double)vb.y, (double)rv.y, s[1][1]);
            s[1][2] = __builtin_fma((double)vb.z, (double)rv.z, s[1][2]);
            s[1][3] = __builtin_fma((double)vb.w, (double)rv.w, s[1][3]);
        }
    } else {
        for (int j = 4 * g; j < d; j += 32) {
#pragma unroll
            for (int e = 0; e < 4; e++) {
                if (e == 0 || j + e < d) {
                    const double rv = (double)r[j + e];
                    s[0][e] = __builtin_fma((double)xa[j + e], rv, s[0][e]);
                    s[1][e] = __builtin_fma((double)xb[j + e], rv, s[1][e]);
                }
            }
        }
    }
    double v[2];
#pragma unroll
    for (int k = 0; k < 2; k++) {
        double w = (s[k][0] + s[k][1]) + (s[k][2] + s[k][3]);
        w = w + shfl_xor_d(w, 1);
        w = w + shfl_xor_d(w, 2);
        w = w + shfl_xor_d(w, 4);
        v[k] = w + 0.0;
    }
    pa = v[0];
    pb = v[1];
}

// Projections of two rows xa, xb onto three directions r, r + rs, r + 2 rs (binary32 values
// held as binary64, converted once per block rather than once per row) from one read of each
// row, every direction value read once for both rows; each projection is computed exactly as
// group8_dot64 computes it.  p[0..2]: row xa, p[3..5]: row xb.
template <bool VEC>
__device__ inline void group8_dot64x3r2(const float *__restrict__ xa, const float *__restrict__ xb,
                                        const double *__restrict__ r, int rs, int d, int g, double p[6]) {
    double s[6][4];
#pragma unroll
    for (int k = 0; k < 6; k++) s[k][0] = s[k][1] = s[k][2] = s[k][3] = 0.0;
    if (VEC) {
        for (int j = 4 * g; j < d; j += 32) {
            const float4 va = *reinterpret_cast<const float4 *>(xa + j);
            const float4 vb = *reinterpret_cast<const float4 *>(xb + j);
            const double a0 = va.x, a1 = va.y, a2 = va.z, a3 = va.w;
            const double b0 = vb.x, b1 = vb.y, b2 = vb.z, b3 = vb.w;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const double2 ra = *reinterpret_cast<const double2 *>(r + k * rs + j);
                const double2 rb = *reinterpret_cast<const double2 *>(r + k * rs + j + 2);
                s[k][0] = __builtin_fma(a0, ra.x, s[k][0]);
                s[k][1] = __builtin_fma(a1, ra.y, s[k][1]);
                s[k][2] = __builtin_fma(a2, rb.x, s[k][2]);
                s[k][3] = __builtin_fma(a3, rb.y, s[k][3]);
                s[k + 3][0] = __builtin_fma(b0, ra.x, s[k + 3][0]);
                s[k + 3][1] = __builtin_fma(b1, ra.y, s[k + 3][1]);
                s[k + 3][2] = __builtin_fma(b2, rb.x, s[k + 3][2]);
                s[k + 3][3] = __builtin_fma(b3, rb.y, s[k + 3][3]);
            }
        }
    } else {
        for (int j = 4 * g; j < d; j += 32) {
#pragma unroll
            for (int e = 0; e < 4; e++) {
                if (e == 0 || j + e < d) {
                    const double ae = (double)xa[j + e], be = (double)xb[j + e];
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        const double rv = r[k * rs + j + e];
                        s[k][e] = __builtin_fma(ae, rv, s[k][e]);
                        s[k + 3][e] = __builtin_fma(be, rv, s[k + 3][e]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 6; k++) {
        double w = (s[k][0] + s[k][1]) + (s[k][2] + s[k][3]);
        w = w + shfl_xor_d(w, 1);
        w = w + shfl_xor_d(w, 2);
        w = w + shfl_xor_d(w, 4);
        p[k] = w + 0.0;
    }
}

// Binary32 coordinate of a grid point from its int8 copy (byte k - 128): the binary64 product
// k * (1/255) rounded to binary32, which equals the correctly rounded quotient k / 255 for
// every k in [0, 255].  The copy holds only coordinates x with float(k) / 255 == x, so this is
// x itself (up to the sign of a zero, which no sum below can see), returned as binary64.
__device__ inline double grid_x(uint32_t k) { return (double)(float)((double)k * (1.0 / 255.0)); }

// group8_dot64 over a row of the int8 grid copy (4-byte aligned, zero-padded past d): the
// same lanes, elements and order as the binary32 forms, so the value is theirs bit for bit.
// VEC: d % 4 == 0 (no element guards, r 16-byte aligned).
template <bool VEC>
__device__ inline double group8_dot64_q8(const int8_t *__restrict__ x, const float *__restrict__ r, int d, int g) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int j = 4 * g; j < d; j += 32) {
        const uint32_t w = *reinterpret_cast<const uint32_t *>(x + j) ^ 0x80808080u;
        if (VEC) {
            const float4 rv = *reinterpret_cast<const float4 *>(r + j);
            s[0] = __builtin_fma(grid_x(w & 255u), (double)rv.x, s[0]);
            s[1] = __builtin_fma(grid_x((w >> 8) & 255u), (double)rv.y, s[1]);
            s[2] = __builtin_fma(grid_x((w >> 16) & 255u), (double)rv.z, s[2]);
            s[3] = __builtin_fma(grid_x(w >> 24), (double)rv.w, s[3]);
        } else {
#pragma unroll
            for (int e = 0; e < 4; e++)
                if (e == 0 || j + e < d) s[e] = __builtin_fma(grid_x((w >> (8 * e)) & 255u), (double)r[j + e], s[e]);
        }
    }
    double v = (s[0] + s[1]) + (s[2] + s[3]);
    v = v + shfl_xor_d(v, 1);
    v = v + shfl_xor_d(v, 2);
    v = v + shfl_xor_d(v, 4);
    return v + 0.0;
}

// group8_dot64x3r2 over two rows of the int8 grid copy; bit for bit the binary32 form's values.
template <bool VEC>
__device__ inline void group8_dot64x3r2_q8(const int8_t *__restrict__ xa, const int8_t *__restrict__ xb,
                                           const double *__restrict__ r, int rs, int d, int g, double p[6]) {
    double s[6][4];
#pragma unroll
    for (int k = 0; k < 6; k++) s[k][0] = s[k][1] = s[k][2] = s[k][3] = 0.0;
#pragma unroll 2
    for (int j = 4 * g; j < d; j += 32) {
        const uint32_t wa = *reinterpret_cast<const uint32_t *>(xa + j) ^ 0x80808080u;
        const uint32_t wb = *reinterpret_cast<const uint32_t *>(xb + j) ^ 0x80808080u;
        if (VEC) {
            double a[4], b[4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                a[e] = grid_x((wa >> (8 * e)) & 255u);
                b[e] = grid_x((wb >> (8 * e)) & 255u);
            }
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const double2 r0 = *reinterpret_cast<const double2 *>(r + k * rs + j);
                const double2 r1 = *reinterpret_cast<const double2 *>(r + k * rs + j + 2);
                s[k][0] = __builtin_fma(a[0], r0.x, s[k][0]);
                s[k][1] = __builtin_fma(a[1], r0.y, s[k][1]);
                s[k][2] = __builtin_fma(a[2], r1.x, s[k][2]);
                s[k][3] = __builtin_fma(a[3], r1.y, s[k][3]);
                s[k + 3][0] = __builtin_fma(b[0], r0.x, s[k + 3][0]);
                s[k + 3][1] = __builtin_fma(b[1], r0.y, s[k + 3][1]);
                s[k + 3][2] = __builtin_fma(b[2], r1.x, s[k + 3][2]);
                s[k + 3][3] = __builtin_fma(b[3], r1.y, s[k + 3][3]);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; e++) {
                if (e == 0 || j + e < d) {
                    const double ae = grid_x((wa >> (8 * e)) & 255u), be = grid_x((wb >> (8 * e)) & 255u);
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        const double rv = r[k * rs + j + e];
                        s[k][e] = __builtin_fma(ae, rv, s[k][e]);
                        s[k + 3][e] = __builtin_fma(be, rv, s[k + 3][e]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 6; k++) {
        double w = (s[k][0] + s[k][1]) + (s[k][2] + s[k][3]);
        w = w + shfl_xor_d(w, 1);
        w = w + shfl_xor_d(w, 2);
        w = w + shfl_xor_d(w, 4);
        p[k] = w + 0.0;
    }
}

template <bool VEC>
__device__ inline double group8_dist64(const float *__restrict__ a, const float *__restrict__ b,
                                       int d, int g) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int j = 4 * g; j < d; j += 32) {
        if (VEC) {
            float4 av = *reinterpret_cast<const float4 *>(a + j);
            float4 bv = *reinterpret_cast<const float4 *>(b + j);
            double e0 = (double)av.x - (double)bv.x, e1 = (double)av.y - (double)bv.y;
            double e2 = (double)av.z - (double)bv.z, e3 = (double)av.w - (double)bv.w;
            s0 = __builtin_fma(e0, e0, s0);
            s1 = __builtin_fma(e1, e1, s1);
            s2 = __builtin_fma(e2, e2, s2);
            s3 = __builtin_fma(e3, e3, s3);
        } else {
            double e0 = (double)a[j] - (double)b[j];
            s0 = __builtin_fma(e0, e0, s0);
            if (j + 1 < d) { double e = (double)a[j + 1] - (double)b[j + 1]; s1 = __builtin_fma(e, e, s1); }
            if (j + 2 < d) { double e = (double)a[j + 2] - (double)b[j + 2]; s2 = __builtin_fma(e, e, s2); }
            if (j + 3 < d) { double e = (double)a[j + 3] - (double)b[j + 3]; s3 = __builtin_fma(e, e, s3); }
        }
    }
    double v = (s0 + s1) + (s2 + s3);
    v = v + shfl_xor_d(v, 1);
    v = v + shfl_xor_d(v, 2);
    v = v + shfl_xor_d(v, 4);
    return v;
}

template <bool VEC>
__device__ inline float group8_dist32(const float *__restrict__ a, const float *__restrict__ b,
                                      int d, int g) {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    for (int j = 4 * g; j < d; j += 32) {
        if (VEC) {
            float4 av = *reinterpret_cast<const float4 *>(a + j);
            float4 bv = *reinterpret_cast<const float4 *>(b + j);
            float e0 = av.x - bv.x, e1 = av.y - bv.y, e2 = av.z - bv.z, e3 = av.w - bv.w;
            s0 = __builtin_fmaf(e0, e0, s0);
            s1 = __builtin_fmaf(e1, e1, s1);
            s2 = __builtin_fmaf(e2, e2, s2);
            s3 = __builtin_fmaf(e3, e3, s3);
        } else {
            float e0 = a[j] - b[j];
            s0 = __builtin_fmaf(e0, e0, s0);
            if (j + 1 < d) { float e = a[j + 1] - b[j + 1]; s1 = __builtin_fmaf(e, e, s1); }
            if (j + 2 < d) { float e = a[j + 2] - b[j + 2]; s2 = __builtin_fmaf(e, e, s2); }
            if (j + 3 < d) { float e = a[j + 3] - b[j + 3]; s3 = __builtin_fmaf(e, e, s3); }
        }
    }
    float v = (s0 + s1) + (s2 + s3);
    v = v + shfl_xor_f(v, 1);
    v = v + shfl_xor_f(v, 2);
    v = v + shfl_xor_f(v, 4);
    return v;
}

// both canonical distances from one read of the two rows (binary32 and binary64 classes)
template <bool VEC>
__device__ inline void group8_dist32_64(const float *__restrict__ a, const float *__restrict__ b, int d, int g,
                                        float &D32, double &D64) {
    float f0 = 0.f, f1 = 0.f, f2 = 0.f, f3 = 0.f;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int j = 4 * g; j < d; j += 32) {
        float4 av, bv;
        if (VEC) {
            av = *reinterpret_cast<const float4 *>(a + j);
            bv = *reinterpret_cast<const float4 *>(b + j);
        } else {
            av.x = a[j];
            bv.x = b[j];
            av.y = j + 1 < d ? a[j + 1] : 0.f;
            bv.y = j + 1 < d ? b[j + 1] : 0.f;
            av.z = j + 2 < d ? a[j + 2] : 0.f;
            bv.z = j + 2 < d ? b[j + 2] : 0.f;
            av.w = j + 3 < d ? a[j + 3] : 0.f;
            bv.w = j + 3 < d ? b[j + 3] : 0.f;
        }
        const float e0 = av.x - bv.x, e1 = av.y - bv.y, e2 = av.z - bv.z, e3 = av.w - bv.w;
        f0 = __builtin_fmaf(e0, e0, f0);
        f1 = __builtin_fmaf(e1, e1, f1);
        f2 = __builtin_fmaf(e2, e2, f2);
        f3 = __builtin_fmaf(e3, e3, f3);
        const double d0 = (double)av.x - (double)bv.x, d1 = (double)av.y - (double)bv.y;
        const double d2 = (double)av.z - (double)bv.z, d3 = (double)av.w - (double)bv.w;
        s0 = __builtin_fma(d0, d0, s0);
        s1 = __builtin_fma(d1, d1, s1);
        s2 = __builtin_fma(d2, d2, s2);
        s3 = __builtin_fma(d3, d3, s3);
    }
    float v = (f0 + f1) + (f2 + f3);
    v = v + shfl_xor_f(v, 1);
    v = v + shfl_xor_f(v, 2);
    v = v + shfl_xor_f(v, 4);
    D32 = v;
    double u = (s0 + s1) + (s2 + s3);
    u = u + shfl_xor_d(u, 1);
    u = u + shfl_xor_d(u, 2);
    u = u + shfl_xor_d(u, 4);
    D64 = u;
}

// The same two distances from a to two rows b0, b1 (d % 4 == 0, 16-byte aligned), with the
// row loads of four steps issued before their arithmetic: the eight lanes of a group then
// wait on memory once per 256 columns of both rows, not once per 32.  Each distance is
// computed exactly as group8_dist32_64 computes it.
__device__ inline void group8_dist32_64x2(const float *__restrict__ a, const float *__restrict__ b0,
                                          const float *__restrict__ b1, int d, int g, float (&D32)[2],
                                          double (&D64)[2]) {
    float f[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    double s[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    auto step = [&](const float4 av, const float4 bv, int r) {
        const float e0 = av.x - bv.x, e1 = av.y - bv.y, e2 = av.z - bv.z, e3 = av.w - bv.w;
        f[r][0] = __builtin_fmaf(e0, e0, f[r][0]);
        f[r][1] = __builtin_fmaf(e1, e1, f[r][1]);
        f[r][2] = __builtin_fmaf(e2, e2, f[r][2]);
        f[r][3] = __builtin_fmaf(e3, e3, f[r][3]);
        const double d0 = (double)av.x - (double)bv.x, d1 = (double)av.y - (double)bv.y;
        const double d2 = (double)av.z - (double)bv.z, d3 = (double)av.w - (double)bv.w;
        s[r][0] = __builtin_fma(d0, d0, s[r][0]);
        s[r][1] = __builtin_fma(d1, d1, s[r][1]);
        s[r][2] = __builtin_fma(d2, d2, s[r][2]);
        s[r][3] = __builtin_fma(d3, d3, s[r][3]);
    };
    int j = 4 * g;
    for (; j + 96 < d; j += 128) {  // four steps of both rows in flight
        float4 x0[4], x1[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            x0[k] = *reinterpret_cast<const float4 *>(b0 + j + 32 * k);
            x1[k] = *reinterpret_cast<const float4 *>(b1 + j + 32 * k);
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const float4 av = *reinterpret_cast<const float4 *>(a + j + 32 * k);
            step(av, x0[k], 0);
            step(av, x1[k], 1);
        }
    }
    if (j < d) {  // the last one to three steps, their loads in flight together: a step past d
                  // reads a clamped address and adds fma(0, 0, s) = s (the sums are never -0)
        float4 x0[3], x1[3], av[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const int jk = j + 32 * k < d ? j + 32 * k : j;
            x0[k] = *reinterpret_cast<const float4 *>(b0 + jk);
            x1[k] = *reinterpret_cast<const float4 *>(b1 + jk);
            av[k] = *reinterpret_cast<const float4 *>(a + jk);
        }
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const bool ok = j + 32 * k < d;
            step(av[k], ok ? x0[k] : av[k], 0);
            step(av[k], ok ? x1[k] : av[k], 1);
        }
    }
#pragma unroll
    for (int r = 0; r < 2; r++) {
        float v = (f[r][0] + f[r][1]) + (f[r][2] + f[r][3]);
        v = v + shfl_xor_f(v, 1);
        v = v + shfl_xor_f(v, 2);
        v = v + shfl_xor_f(v, 4);
        D32[r] = v;
        double u = (s[r][0] + s[r][1]) + (s[r][2] + s[r][3]);
        u = u + shfl_xor_d(u, 1);
        u = u + shfl_xor_d(u, 2);
        u = u + shfl_xor_d(u, 4);
        D64[r] = u;
    }
}

// The binary64 distances alone of group8_dist32_64x2 (the same operations, in the same order).
__device__ inline void group8_dist64x2(const float *__restrict__ a, const float *__restrict__ b0,
                                       const float *__restrict__ b1, int d, int g, double (&D64)[2]) {
    double s[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    auto step = [&](const float4 av, const float4 bv, int r) {
        const double d0 = (double)av.x - (double)bv.x, d1 = (double)av.y - (double)bv.y;
        const double d2 = (double)av.z - (double)bv.z, d3 = (double)av.w - (double)bv.w;
        s[r][0] = __builtin_fma(d0, d0, s[r][0]);
        s[r][1] = __builtin_fma(d1, d1, s[r][1]);
        s[r][2] = __builtin_fma(d2, d2, s[r][2]);
        s[r][3] = __builtin_fma(d3, d3, s[r][3]);
    };
    int j = 4 * g;
    for (; j + 96 < d; j += 128) {  // four steps of both rows in flight
        float4 x0[4], x1[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            x0[k] = *reinterpret_cast<const float4 *>(b0 + j + 32 * k);
            x1[k] = *reinterpret_cast<const float4 *>(b1 + j + 32 * k);
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const float4 av = *reinterpret_cast<const float4 *>(a + j + 32 * k);
            step(av, x0[k], 0);
            step(av, x1[k], 1);
        }
    }
    if (j < d) {  // the last one to three steps, their loads in flight together: a step past d
                  // reads a clamped address and adds fma(0, 0, s) = s (the sums are never -0)
        float4 x0[3], x1[3], av[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const int jk = j + 32 * k < d ? j + 32 * k : j;
            x0[k] = *reinterpret_cast<const float4 *>(b0 + jk);
            x1[k] = *reinterpret_cast<const float4 *>(b1 + jk);
            av[k] = *reinterpret_cast<const float4 *>(a + jk);
        }
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const bool ok = j + 32 * k < d;
            step(av[k], ok ? x0[k] : av[k], 0);
            step(av[k], ok ? x1[k] : av[k], 1);
        }
    }
#pragma unroll
    for (int r = 0; r < 2; r++) {
        double u = (s[r][0] + s[r][1]) + (s[r][2] + s[r][3]);
        u = u + shfl_xor_d(u, 1);
        u = u + shfl_xor_d(u, 2);
        u = u + shfl_xor_d(u, 4);
        D64[r] = u;
    }
}

// The binary64 distances of four rows at once (the same operations, in the same order, as
// group8_dist32_64 computes D64): sixteen 16-byte loads in flight per lane for d = 128.
__device__ inline void group8_dist64x4(const float *__restrict__ a, const float *const (&b)[4], int d, int g,
                                       double (&D64)[4]) {
    double s[4][4];
#pragma unroll
    for (int r = 0; r < 4; r++) s[r][0] = s[r][1] = s[r][2] = s[r][3] = 0.0;
    auto step = [&](const float4 av, const float4 bv, int r) {
        const double d0 = (double)av.x - (double)bv.x, d1 = (double)av.y - (double)bv.y;
        const double d2 = (double)av.z - (double)bv.z, d3 = (double)av.w - (double)bv.w;
        s[r][0] = __builtin_fma(d0, d0, s[r][0]);
        s[r][1] = __builtin_fma(d1, d1, s[r][1]);
        s[r][2] = __builtin_fma(d2, d2, s[r][2]);
        s[r][3] = __builtin_fma(d3, d3, s[r][3]);
    };
    int j = 4 * g;
    for (; j + 96 < d; j += 128) {  // four steps of all four rows in flight
        float4 x[4][4];
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int k = 0; k < 4; k++) x[r][k] = *reinterpret_cast<const float4 *>(b[r] + j + 32 * k);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const float4 av = *reinterpret_cast<const float4 *>(a + j + 32 * k);
#pragma unroll
            for (int r = 0; r < 4; r++) step(av, x[r][k], r);
        }
    }
    if (j < d) {  // the last one to three steps, their loads in flight together: a step past d
                  // reads a clamped address and adds fma(0, 0, s) = s (the sums are never -0)
        float4 x[4][3], av[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const int jk = j + 32 * k < d ? j + 32 * k : j;
#pragma unroll
            for (int r = 0; r < 4; r++) x[r][k] = *reinterpret_cast<const float4 *>(b[r] + jk);
            av[k] = *reinterpret_cast<const float4 *>(a + jk);
        }
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const bool ok = j + 32 * k < d;
#pragma unroll
            for (int r = 0; r < 4; r++) step(av[k], ok ? x[r][k] : av[k], r);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; r++) {
        double u = (s[r][0] + s[r][1]) + (s[r][2] + s[r][3]);
        u = u + shfl_xor_d(u, 1);
        u = u + shfl_xor_d(u, 2);
        u = u + shfl_xor_d(u, 4);
        D64[r] = u;
    }
}

// ---------------------------------------------------------------- host-side launch helpers

struct Prof;  // per-kernel event timing (rpf_api.hip)
void prof_begin(hipStream_t s, const char *name, double bytes, double flops, void **tok);
void prof_end(hipStream_t s, void *tok);

struct ProfScope {
    hipStream_t s;
    void *tok = nullptr;
    ProfScope(hipStream_t s_, const char *name, double bytes = 0, double flops = 0) : s(s_) {
        prof_begin(s, name, bytes, flops, &tok);
    }
    ~ProfScope() { prof_end(s, tok); }
};

}  // namespace rpf
