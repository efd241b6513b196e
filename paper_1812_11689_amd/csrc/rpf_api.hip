// C ABI of the rpForests library: argument checks, the closed-form tree plan, device
// memory, and the launch sequences of rpf_build / rpf_all_knn / rpf_query.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "rpf_internal.h"

namespace rpf {

// ---- launchers defined in build_kernels.hip / knn_kernels.hip
size_t cand_bytes();
size_t level_small_lds(int max_m, int d, int n_try);
void launch_level_small(hipStream_t s, bool vec, const float *X, int d, const float *R, int64_t H, int n_try,
                        const SegDesc *segs, int nseg, int max_m, int T, const int32_t *pin, int32_t *pout,
                        int64_t n, double *split, int32_t *split_idx, int32_t *chosen, int32_t *err,
                        const LevelLink &lk);
void launch_level_large(hipStream_t s, bool vec, const float *X, int d, const float *R, int64_t H, int n_try,
                        const SegDesc *segs, int nseg, const ChunkDesc *chunks, int nchunk, int T,
                        const int32_t *pin, int32_t *pout, int64_t n, double *split, int32_t *split_idx,
                        int32_t *chosen, int32_t *err, const LargeBufs &b, double proj_bytes,
                        const LevelLink &lk);
void launch_copy_segments(hipStream_t s, const LeafDesc *segs, int nseg, int T, const int32_t *in, int32_t *out,
                          int64_t n);
void launch_iota(hipStream_t s, int32_t *perm, int64_t n, int T);
void launch_leaf_finalize(hipStream_t s, int prec, const float *X, int d, int dp, const LeafDesc *leaves,
                          int nleaf, int T, const int32_t *perm, int64_t n, int32_t *leaf_of, float *centroid,
                          void *Xc, float2 *nrm, int max_leaf, int lds_limit);
void launch_leaf_copy(hipStream_t s, int prec, const float *X, int d, int dp, const LeafDesc *leaves, int nleaf,
                      int ntree, const int32_t *perm, int64_t n, const float *centroid, void *Xc);
void launch_leaf_stats(hipStream_t s, int prec, const float *X, int d, int dp, const LeafDesc *leaves, int nleaf,
                       int ntree, const int32_t *perm, int64_t n, int32_t *leaf_of, float *centroid, float2 *nrm,
                       int max_leaf);
void launch_nonfinite(hipStream_t s, const float *x, int64_t count, int32_t *flag);
void launch_localize(int32_t *idx, int64_t rows, int K, const int64_t *off, int count, hipStream_t s);


// ---------------------------------------------------------------- errors

static thread_local std::string g_err;

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

rpf_status fail(rpf_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

rpf_status check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return RPF_OK;
    return fail(e == hipErrorOutOfMemory ? RPF_ENOMEM : RPF_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

static thread_local std::string g_launch_err;

bool sync_check_on() {
    static const bool sync = [] {
        const char *e = getenv("RPF_SYNC_CHECK");
        return e && e[0] == '1';
    }();
    return sync;
}

void launch_check(hipStream_t s, const char *name) {
    const bool sync = sync_check_on();
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && sync && !capturing(s)) e = hipStreamSynchronize(s);
    if (e != hipSuccess && g_launch_err.empty()) g_launch_err = std::string(name) + ": " + hipGetErrorString(e);
}

std::string take_launch_error() {
    std::string r;
    r.swap(g_launch_err);
    return r;
}

// ---------------------------------------------------------------- profiling

struct ProfRec {
    int64_t launches = 0;
    double ms = 0, bytes = 0, flops = 0;
};
struct Pending {
    std::string name;
    hipEvent_t a, b;
    double bytes, flops;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::map<std::string, ProfRec> g_prof;
static std::vector<Pending> g_pending;
static std::vector<hipEvent_t> g_event_pool;

static hipEvent_t get_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    hipEventCreate(&e);
    return e;
}

void prof_begin(hipStream_t s, const char *name, double bytes, double flops, void **tok) {
    *tok = nullptr;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on || capturing(s)) return;  // a recorded graph carries no timing events
    Pending *p = new Pending{name, get_event(), get_event(), bytes, flops};
    hipEventRecord(p->a, s);
    *tok = p;
}

void prof_end(hipStream_t s, void *tok) {
    if (!tok) return;
    Pending *p = static_cast<Pending *>(tok);
    hipEventRecord(p->b, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_pending.push_back(*p);
    delete p;
}

static void prof_drain() {
    for (auto &p : g_pending) {
        hipEventSynchronize(p.b);
        float ms = 0;
        hipEventElapsedTime(&ms, p.a, p.b);
        ProfRec &r = g_prof[p.name];
        r.launches++;
        r.ms += ms;
        r.bytes += p.bytes;
        r.flops += p.flops;
        g_event_pool.push_back(p.a);
        g_event_pool.push_back(p.b);
    }
    g_pending.clear();
}

// ---------------------------------------------------------------- validation kernels

// *flag |= 1 when x holds a NaN or an infinity.  VEC: x 16-byte aligned, four values per access.
template <bool VEC>
__global__ void k_nonfinite(const float *__restrict__ x, int64_t count, int32_t *flag) {
    int bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (VEC) {
        const int64_t c4 = count >> 2;
        const float4 *x4 = reinterpret_cast<const float4 *>(x);
        for (int64_t j = i; j < c4; j += stride) {
            const float4 v = x4[j];
            bad |= (int)!isfinite(v.x) | (int)!isfinite(v.y) | (int)!isfinite(v.z) | (int)!isfinite(v.w);
        }
        i += c4 << 2;  // the last count % 4 values
        if (i < count) bad |= !isfinite(x[i]);
    } else {
        for (; i < count; i += stride) bad |= !isfinite(x[i]);
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(flag, 1);
}

void launch_nonfinite(hipStream_t s, const float *x, int64_t count, int32_t *flag) {
    if (count <= 0) return;
    const bool vec = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    const int64_t per = vec ? 1024 : 256;
    const int64_t blocks = std::min<int64_t>((count + per - 1) / per, 16384);
    if (vec)
        hipLaunchKernelGGL(k_nonfinite<true>, dim3((unsigned)blocks), dim3(256), 0, s, x, count, flag);
    else
        hipLaunchKernelGGL(k_nonfinite<false>, dim3((unsigned)blocks), dim3(256), 0, s, x, count, flag);
}

// The input copy and its check in one pass: dst = src, and *flag |= 1 when src holds a NaN or
// an infinity.  VEC: both pointers 16-byte aligned, four values per access.
template <bool VEC>
__global__ void k_copy_nonfinite(const float *__restrict__ src, float *__restrict__ dst, int64_t count,
                                 int32_t *flag) {
    int bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (VEC) {
        const int64_t c4 = count >> 2;
        const float4 *s4 = reinterpret_cast<const float4 *>(src);
        float4 *d4 = reinterpret_cast<float4 *>(dst);
        for (int64_t j = i; j < c4; j += stride) {
            const float4 v = s4[j];
            bad |= (int)!isfinite(v.x) | (int)!isfinite(v.y) | (int)!isfinite(v.z) | (int)!isfinite(v.w);
            d4[j] = v;
        }
        i += c4 << 2;  // the last count % 4 values, one per thread of the first threads
        if (i < count) {
            const float v = src[i];
            bad |= !isfinite(v);
            dst[i] = v;
        }
    } else {
        for (; i < count; i += stride) {
            const float v = src[i];
            bad |= !isfinite(v);
            dst[i] = v;
        }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(flag, 1);
}

void launch_copy_nonfinite(hipStream_t s, const float *src, float *dst, int64_t count, int32_t *flag) {
    if (count <= 0) return;
    const bool vec = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0;
    const int64_t per = vec ? 1024 : 256;  // values one 256-thread block covers per sweep
    const int64_t blocks = std::min<int64_t>((count + per - 1) / per, 16384);
    if (vec)
        hipLaunchKernelGGL(k_copy_nonfinite<true>, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, count, flag);
    else
        hipLaunchKernelGGL(k_copy_nonfinite<false>, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, count, flag);
}

// Points on the 1/255 grid: for each coordinate x, k = rint(255 x) must lie in [0, 255] with
// float(k) / 255.0f == x (so -0 counts as k = 0); the row is stored as int8 k - 128 (zero from
// d to dq) with |k - 128|^2 (exact) and |k| / 255.  One wave per row; any coordinate off the
// grid sets *flag.
__global__ __launch_bounds__(256) void k_grid_quantise(const float *__restrict__ X, int64_t n, int d, int dq,
                                                       int8_t *__restrict__ Xq, LatNorm *__restrict__ qn,
                                                       int32_t *__restrict__ flag) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    int32_t na = 0, kk = 0;
    bool ok = true;
    for (int c = lane; c < dq; c += 64) {
        int v = 0;
        if (c < d) {
            const float x = X[row * d + c];
            const int k = (int)rintf(x * 255.f);
            ok &= k >= 0 && k <= 255 && (float)k / 255.f == x;
            const int kc = k < 0 ? 0 : k > 255 ? 255 : k;
            v = kc - 128;
            na += v * v;
            kk += kc * kc;
        }
        Xq[row * dq + c] = (int8_t)v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        na += __shfl_xor(na, o, 64);
        kk += __shfl_xor(kk, o, 64);
    }
    if (lane == 0) qn[row] = LatNorm{na, sqrtf((float)kk) / 255.f};
    if (__ballot(!ok) && lane == 0) atomicOr(flag, 1);
}

// leaf_of alone: the heap id of every point's leaf, from the leaf table and the final order
__global__ __launch_bounds__(256) void k_leaf_ids(const LeafDesc *__restrict__ leaves, const int32_t *__restrict__ perm,
                                                  int64_t n, int32_t *__restrict__ leaf_of) {
    const LeafDesc lf = leaves[blockIdx.x];
    const int64_t t = blockIdx.y;
    for (int i = threadIdx.x; i < lf.size; i += blockDim.x)
        leaf_of[t * n + perm[t * n + lf.off + i]] = lf.heap;
}

void launch_leaf_ids(hipStream_t s, const LeafDesc *leaves, int nleaf, int T, const int32_t *perm, int64_t n,
                     int32_t *leaf_of) {
    if (nleaf <= 0) return;
    hipLaunchKernelGGL(k_leaf_ids, dim3((unsigned)nleaf, (unsigned)T), dim3(256), 0, s, leaves, perm, n, leaf_of);
}

void launch_grid_quantise(hipStream_t s, const float *X, int64_t n, int d, int dq, int8_t *Xq, LatNorm *qn,
                          int32_t *flag) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_grid_quantise, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, X, n, d, dq, Xq, qn, flag);
    launch_check(s, "k_grid_quantise");
}

}  // namespace rpf

using namespace rpf;

// ---------------------------------------------------------------- the forest

namespace rpf {
struct LevelPlan {
    std::vector<SegDesc> segs;     // internal nodes
    std::vector<ChunkDesc> chunks; // multi-block path
    std::vector<LeafDesc> copy;    // leaves formed at or before this level (carried over)
    std::vector<LookDesc> look;    // per internal node: its children at the next level
    std::vector<int32_t> hbase;    // per internal node: its data set's first heap slot
    int max_m = 0;
    bool large = false;
    bool lead = false, fed = false;  // linked pair: the lead also makes the fed level's keys
    int64_t seg_off = 0, chunk_off = 0, copy_off = 0;  // offsets into the device descriptor arrays
};
}  // namespace rpf

struct rpf_forest {
    int64_t n = 0;
    int32_t d = 0, T = 0, n0 = 0, n_try = 0, L = 0, prec = 0, dp = 0;
    int32_t tile_prec = 0;  // as asked (rpf_dist_prec); prec is that of the copies and norms
    int8_t *Xq = nullptr;       // grid forests: [n][dq] int8 k - 128
    rpf::LatNorm *qn = nullptr; // grid forests: [n]
    int32_t dq = 0;
    int64_t H = 0;
    int device = 0;
    // persistent device arrays
    float *X = nullptr;          // [n][d]
    float *R = nullptr;          // [T][H][n_try][d]
    double *split = nullptr;     // [T][H]
    int32_t *split_idx = nullptr;
    int32_t *chosen = nullptr;
    int32_t *perm[2] = {nullptr, nullptr};
    int final_buf = 0;
    int32_t *leaf_of = nullptr;  // [T][n]
    float *centroid = nullptr;   // [T][nleaf][d]
    void *Xc = nullptr;          // [T][n][dp] leaf-ordered, centred, tile precision
    float2 *nrm = nullptr;       // [T][n] (|Xc row|^2, |x - mu|)
    int32_t *err = nullptr;      // device error flags of the build kernels
    int32_t *heap_leaf = nullptr;  // heap id -> leaf index
    // descriptors
    SegDesc *d_segs = nullptr;
    ChunkDesc *d_chunks = nullptr;
    LeafDesc *d_leaves = nullptr;
    LeafDesc *d_copy = nullptr;
    LookDesc *d_look = nullptr;  // per internal node of every level, indexed like d_segs
    TileJob *d_jobs = nullptr;   // all-points tile jobs
    int64_t n_jobs_tree = 0;     // jobs per tree
    int job_mb = 8;
    double tile_flops_tree = 0;
    std::vector<LeafDesc> leaves;
    int max_leaf = 0;
    uint64_t bytes = 0;
    // the closed-form plan of the build, kept so the build launches can be replayed
    std::vector<rpf::LevelPlan> levels;
    rpf::LargeBufs lb{};         // temporaries of the multi-block levels
    std::vector<void *> tmps;    // their blocks (released after a one-shot build)
    int lds_max = 0;
    // persistent subtree schedule (RPF_BUILD_SUBTREES): levels sub_level .. L-1 in one launch
    int sub_level = -1;          // -1: not available for this forest
    bool subtree_on = false;     // the schedule build_launches uses
    int sub_max_m = 0;
    int64_t n_sub_items = 0;
    rpf::SubItem *d_sub_items = nullptr;
    uint32_t *sub_next = nullptr;  // the launch's work counter
    // batched forests: one root per data set (a single data set is the one-root case)
    std::vector<rpf_batch_entry> batch;
    int64_t *d_batch_off = nullptr;       // [count + 1] first point of every data set, then n
    // stats of the last kNN call
    unsigned long long *stats = nullptr;  // [kStatSlots][8]
    // rows whose pruning buffers met an index outside [0, n) since the build (an internal
    // error; never cleared): device counter (the word after the stats), and its host mirror
    // in pinned memory, refreshed by an asynchronous copy at the end of every search call
    unsigned long long *fault = nullptr;
    int pin_slot = -1;
    mutable std::mutex mu;
    // the leaf copies (Xc) when made after the build, on a query's first use
    std::mutex xc_mu;
    hipEvent_t xc_ev = nullptr;  // recorded after the copy kernel
    // uniform split rule: every tree has its own leaves (table [T][leaf_stride], leaf_of holds
    // ordinals within the tree), its own tile jobs and its own node list
    int32_t split_rule = RPF_SPLIT_MEDIAN;
    uint64_t seed = 0;
    int64_t leaf_stride = 0;
    std::vector<int32_t> tree_nleaf;       // leaves of each tree
    std::vector<int64_t> job_off;          // [T + 1]
    std::vector<double> flops_off;         // [T + 1]
    std::vector<std::vector<rpf_node>> nodes;
};

namespace rpf {



static int depth_of(int64_t n, int64_t n0) {
    int L = 0;
    while ((n + ((int64_t)1 << L) - 1) >> L > n0) L++;
    return L;
}

static int lds_limit(int dev) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) v = 65536;
    return v;
}

}  // namespace rpf

extern "C" {

int32_t rpf_depth(int64_t n, int32_t leaf_size) {
    if (n < 1 || leaf_size < 1) return -1;
    return depth_of(n, leaf_size);
}

const char *rpf_last_error(void) { return g_err.c_str(); }

rpf_status rpf_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return RPF_OK;
}

rpf_status rpf_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain();
    g_prof.clear();
    return RPF_OK;
}

rpf_status rpf_profile_read(rpf_profile_record *out, int32_t cap, int32_t *count) {
    if (!count || (cap > 0 && !out)) return fail(RPF_EINVAL, "rpf_profile_read: null pointer");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain();
    int32_t k = 0;
    for (auto &kv : g_prof) {
        if (k < cap) {
            memset(&out[k], 0, sizeof(out[k]));
            strncpy(out[k].name, kv.first.c_str(), sizeof(out[k].name) - 1);
            out[k].launches = kv.second.launches;
            out[k].total_ms = kv.second.ms;
            out[k].algo_bytes = kv.second.bytes;
            out[k].algo_flops = kv.second.flops;
        }
        k++;
    }
    *count = k;
    return RPF_OK;
}

// Host mirrors of the forests' internal-fault counters: one pinned page for the process
// (allocated once, never freed), a word per live forest.  A forest that finds no free word
// reports its faults at synchronising calls only.
constexpr int kPinSlots = 4096;
static std::mutex g_pin_mu;
static unsigned long long *g_pin = nullptr;
static std::vector<int> g_pin_free;

static int pin_take() {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    if (!g_pin) {
        void *p = nullptr;
        if (hipHostMalloc(&p, kPinSlots * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess || !p) {
            hipGetLastError();
            return -1;
        }
        g_pin = static_cast<unsigned long long *>(p);
        for (int i = kPinSlots - 1; i >= 0; i--) g_pin_free.push_back(i);
    }
    if (g_pin_free.empty()) return -1;
    const int k = g_pin_free.back();
    g_pin_free.pop_back();
    __atomic_store_n(&g_pin[k], 0ull, __ATOMIC_RELAXED);
    return k;
}

static void pin_give(int k) {
    if (k < 0) return;
    std::lock_guard<std::mutex> lk(g_pin_mu);
    g_pin_free.push_back(k);
}

// forest arrays come from the library's caching allocator, so repeated build / free
// cycles reuse device blocks instead of mapping fresh pages; callers synchronise first
static void free_forest_memory(rpf_forest *f) {
    void *ptrs[] = {f->X, f->R, f->split, f->split_idx, f->chosen, f->perm[0], f->perm[1], f->leaf_of,
                    f->centroid, f->Xc, f->nrm, f->err, f->heap_leaf, f->d_segs, f->d_chunks, f->d_leaves,
                    f->d_copy, f->d_look, f->d_jobs, f->stats, f->d_batch_off, f->Xq, f->qn, f->d_sub_items,
                    f->sub_next};
    for (void *p : ptrs) cache_free_idle(p);
    pin_give(f->pin_slot);
    f->pin_slot = -1;
    for (void *p : f->tmps) cache_free_idle(p);
    f->tmps.clear();
    if (f->xc_ev) hipEventDestroy(f->xc_ev);
    f->xc_ev = nullptr;
}

rpf_status rpf_free(rpf_forest *f) {
    if (!f) return RPF_OK;
    hipDeviceSynchronize();
    free_forest_memory(f);
    delete f;
    return RPF_OK;
}

}  // extern "C"

// Grow the forest over `count` data sets concatenated in X ([sum n_i][d]); every data set is
// an independent root whose trees advance with all the others, level by level, in the same
// launches.  Internal node h (heap id, root 1) of data set i has the global id hbase_i + h,
// with hbase_i = sum over j < i of (2^L_j - 1): the direction and split arrays are
// [T][sum H_i] and the kernels index them as for one tree.  Leaf h of data set i has the id
// lbase_i + h, lbase_i = sum over j < i of 2^(L_j + 1), in leaf_of and in the leaf table.
static rpf_status prepare_forest(const int64_t *sizes, int count, int32_t d, const rpf_params *p, void *stream,
                                 rpf_forest **out, bool need_directions = true) {
    if (out) *out = nullptr;
    if (!out) return fail(RPF_EINVAL, "rpf_build: out is NULL");
    if (!p) return fail(RPF_EINVAL, "rpf_build: params is NULL");
    if (!sizes || count < 1) return fail(RPF_EINVAL, "rpf_build: no data set");
    int64_t n = 0;
    for (int i = 0; i < count; i++) {
        if (sizes[i] < 1) return fail(RPF_EINVAL, "rpf_build: every data set needs n >= 1");
        n += sizes[i];
        if (n >= ((int64_t)1 << 31)) return fail(RPF_EINVAL, "rpf_build: n must be in [1, 2^31)");
    }
    if (d < 1) return fail(RPF_EINVAL, "rpf_build: d must be >= 1");
    if (d > 4096) return fail(RPF_EINVAL, "rpf_build: d above 4096 is not supported (per-block staging)");
    if (p->n_trees < 1 || p->n_trees > 65535) return fail(RPF_EINVAL, "rpf_build: n_trees must be in [1, 65535]");
    if (p->leaf_size < 1) return fail(RPF_EINVAL, "rpf_build: leaf_size must be >= 1");
    if (p->n_try < 1) return fail(RPF_EINVAL, "rpf_build: n_try must be >= 1");
    if (p->split_rule != RPF_SPLIT_MEDIAN)
        return fail(RPF_EINVAL, p->split_rule == RPF_SPLIT_UNIFORM
                                    ? "the uniform split rule grows one data set per forest (rpf_build), not batches or plans"
                                    : "rpf_build: unknown split_rule");
    if (p->dist_prec < RPF_DIST_FP32 || p->dist_prec > RPF_DIST_U8GRID)
        return fail(RPF_EINVAL, "rpf_build: unknown dist_prec");
    if (p->build_flags & ~RPF_BUILD_SUBTREES) return fail(RPF_EINVAL, "rpf_build: unknown build_flags");
    std::vector<rpf_batch_entry> roots(count);
    int L = 0;
    int64_t H = 0, LB = 0;
    for (int i = 0; i < count; i++) {
        rpf_batch_entry &r = roots[i];
        r.offset = i ? roots[i - 1].offset + roots[i - 1].n : 0;
        r.n = sizes[i];
        r.depth = depth_of(sizes[i], p->leaf_size);
        if (r.depth > 30) return fail(RPF_EINVAL, "rpf_build: tree deeper than 30 levels");
        r.reserved = 0;
        r.heap_base = H;
        r.leaf_heap_base = LB;
        H += ((int64_t)1 << r.depth) - 1;
        LB += (int64_t)2 << r.depth;
        L = std::max(L, (int)r.depth);
    }
    if (H >= ((int64_t)1 << 31) || LB >= ((int64_t)1 << 31)) return fail(RPF_EINVAL, "rpf_build: too many tree nodes");
    if (need_directions && H > 0 && !p->directions_dev) return fail(RPF_EINVAL, "rpf_build: directions_dev is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int T = p->n_trees, n0 = p->leaf_size, n_try = p->n_try;

    int dev = 0;
    hipGetDevice(&dev);

    // ---- plan (closed form: the median rule makes the shape data-independent)
    std::vector<LevelPlan> levels(L);
    std::vector<LeafDesc> leaves;
    {
        struct Node { int64_t heap, off, size; int root; };  // heap: id within its data set
        std::vector<Node> cur;
        for (int i = 0; i < count; i++) cur.push_back({1, roots[i].offset, roots[i].n, i});
        std::vector<LeafDesc> formed;
        for (int l = 0; l <= L; l++) {
            std::vector<Node> next;
            std::vector<int32_t> node_seg(cur.size(), -1);  // internal node index of each node of `cur`
            for (size_t q = 0; q < cur.size(); q++) {
                const Node &nd = cur[q];
                const rpf_batch_entry &r = roots[nd.root];
                if (nd.size > n0 && l < r.depth) {
                    node_seg[q] = (int32_t)levels[l].segs.size();
                    levels[l].segs.push_back(SegDesc{nd.off, (int32_t)nd.size, (int32_t)(r.heap_base + nd.heap), 0, 0});
                    levels[l].hbase.push_back((int32_t)r.heap_base);
                    levels[l].max_m = std::max<int>(levels[l].max_m, (int)nd.size);
                    next.push_back({2 * nd.heap, nd.off, nd.size / 2, nd.root});
                    next.push_back({2 * nd.heap + 1, nd.off + nd.size / 2, nd.size - nd.size / 2, nd.root});
                } else {
                    formed.push_back(LeafDesc{nd.off, (int32_t)nd.size, (int32_t)(r.leaf_heap_base + nd.heap)});
                }
            }
            if (l > 0 && l <= L) {  // children of level l - 1's nodes: pushed in pairs, in node order
                auto &up = levels[l - 1];
                up.look.resize(up.segs.size());
                for (size_t k = 0; k < up.segs.size(); k++)
                    for (int b = 0; b < 2; b++) {
                        const int32_t cs = l < L ? node_seg[2 * k + b] : -1;
                        up.look[k].child_seg[b] = cs;
                        up.look[k].child_heap[b] = cs >= 0 ? levels[l].segs[cs].heap : 0;
                    }
            }
            if (l < L) levels[l].copy = formed;  // leaves carried into this level's output
            cur.swap(next);
        }
        leaves = formed;
        std::sort(leaves.begin(), leaves.end(), [](const LeafDesc &a, const LeafDesc &b) { return a.off < b.off; });
    }
    const int lds_max = lds_limit(dev);
    int small_max = kLarge;
    while (small_max > 2 && level_small_lds(small_max, d, n_try) > (size_t)lds_max) small_max /= 2;
    int64_t max_seg_large = 0, max_chunk_large = 0;
    int64_t nseg_tot = 0, nchunk_tot = 0, ncopy_tot = 0;
    for (auto &lv : levels) {
        lv.large = lv.max_m > small_max;
        lv.seg_off = nseg_tot;
        lv.copy_off = ncopy_tot;
        lv.chunk_off = nchunk_tot;
        if (lv.large) {
            for (auto &sg : lv.segs) {
                sg.chunk0 = (int32_t)lv.chunks.size();
                sg.nchunk = (int32_t)((sg.size + kChunk - 1) / kChunk);
                for (int q = 0; q < sg.nchunk; q++) {
                    int64_t st = sg.off + (int64_t)q * kChunk;
                    int32_t len = (int32_t)std::min<int64_t>(kChunk, sg.off + sg.size - st);
                    lv.chunks.push_back(ChunkDesc{st, len, (int32_t)(&sg - lv.segs.data())});
                }
            }
            max_seg_large = std::max<int64_t>(max_seg_large, (int64_t)lv.segs.size());
            max_chunk_large = std::max<int64_t>(max_chunk_large, (int64_t)lv.chunks.size());
        }
        nseg_tot += lv.segs.size();
        nchunk_tot += lv.chunks.size();
        ncopy_tot += lv.copy.size();
    }

    // ---- level links: with one direction per node, pair each level with the next (the lead
    // projects onto the children too); a multi-block level is never fed by a one-block one
    bool any_link = false, any_large_fed = false;
    if (n_try == 1 && d <= 1024)
        for (int l = 0; l + 1 < L; l++) {
            LevelPlan &a = levels[l], &b = levels[l + 1];
            if (a.fed || a.segs.empty() || b.segs.empty() || (b.large && !a.large)) continue;
            a.lead = b.fed = true;
            any_link = true;
            any_large_fed |= b.large;
        }

    // ---- the persistent subtree schedule: from the first level after which every level fits
    // one workgroup (a fed level stays level-synchronous: its keys come from the level above),
    // when at least two levels remain
    int sub_level = -1;
    if (n_try == 1) {
        int l0 = L;
        while (l0 > 0 && !levels[l0 - 1].large) l0--;
        if (l0 < L && levels[l0].fed) l0++;
        int mm = 0;
        for (int l = l0; l < L; l++) mm = std::max(mm, levels[l].max_m);
        if (l0 + 2 <= L && !levels[l0].segs.empty() && (int64_t)levels[l0].segs.size() * T < ((int64_t)1 << 31) &&
            subtree_lds(mm, d) <= (size_t)lds_max)
            sub_level = l0;
    }

    // ---- memory plan
    // split bfloat16 and int8 grid tiles run beside binary32 copies and norms: the forest is a
    // binary32 one
    const bool grid = p->dist_prec == RPF_DIST_U8GRID;
    const int prec = (p->dist_prec == RPF_DIST_BF16X3 || grid) ? RPF_DIST_FP32 : p->dist_prec;
    const int dq = grid ? (d + 63) & ~63 : 0;
    const int dp = (d + 7) & ~7;
    const size_t esz = prec == RPF_DIST_FP32 ? 4 : 2;
    const int64_t nleaf = (int64_t)leaves.size();
    int max_leaf = 0;
    for (auto &lf : leaves) max_leaf = std::max(max_leaf, (int)lf.size);
    // the all-points search stages leaves of one tile (at most 256 points) straight from X;
    // larger leaves read the leaf-ordered centred copy, made here; queries make it on first use
    const bool xc_eager = max_leaf > 256 && !grid;  // grid tiles read the int8 copy
    const uint64_t xc_bytes = (uint64_t)T * n * dp * esz;
    uint64_t bytes = 0;
    bytes += (uint64_t)n * d * 4;                        // X
    bytes += (uint64_t)T * H * n_try * d * 4;            // R
    bytes += (uint64_t)T * H * (8 + 4 + 4);              // split, split_idx, chosen
    bytes += (uint64_t)2 * T * n * 4;                    // perm x2
    bytes += (uint64_t)T * n * 4;                        // leaf_of
    bytes += (uint64_t)T * nleaf * d * 4;                // centroid
    bytes += (uint64_t)T * n * dp * esz;                 // Xc
    bytes += (uint64_t)T * n * 8;                        // nrm
    uint64_t tmp_bytes = 0;
    if (max_seg_large > 0) {
        tmp_bytes += (uint64_t)T * n * 8;                                      // keys
        if (n_try > 1) tmp_bytes += (uint64_t)T * n * 8;                       // praw
        tmp_bytes += (uint64_t)T * max_seg_large * (sizeof(SelState) + 4 * kDigitBins + cand_bytes() * kCandCap + 4);
        tmp_bytes += (uint64_t)T * max_chunk_large * (4 + 8);
    }
    if (any_link) tmp_bytes += (uint64_t)T * n * (16 + 8);                    // ahead, keys2
    if (any_large_fed) tmp_bytes += (uint64_t)T * max_seg_large * 4 * kDigitBins;  // hist2
    if (p->mem_budget_bytes && bytes + tmp_bytes > p->mem_budget_bytes)
        return fail(RPF_ENOMEM, "rpf_build: forest needs " + std::to_string(bytes + tmp_bytes) +
                                    " bytes, over mem_budget_bytes");

    rpf_forest *f = new rpf_forest();
    f->n = n; f->d = d; f->T = T; f->n0 = n0; f->n_try = n_try; f->L = L; f->H = H;
    f->prec = prec; f->tile_prec = p->dist_prec; f->dp = dp; f->device = dev; f->leaves = leaves; f->max_leaf = max_leaf;
    f->bytes = bytes - (xc_eager ? 0 : xc_bytes);
    f->batch = roots;

    auto bail = [&](rpf_status st) {
        hipStreamSynchronize(s);
        free_forest_memory(f);
        delete f;
        return st;
    };
#define RPF_ALLOC(ptr, sz)                                                                            \
    do {                                                                                              \
        size_t _sz = (size_t)(sz);                                                                    \
        if (_sz) {                                                                                    \
            (ptr) = static_cast<std::remove_reference_t<decltype(ptr)>>(cache_alloc(_sz, s));                                \
            if (!(ptr)) {                                                                             \
                fail(RPF_ENOMEM, "rpf_build: device allocation of " #ptr " failed");                 \
                return bail(RPF_ENOMEM);                                                              \
            }                                                                                         \
        }                                                                                             \
    } while (0)

    RPF_ALLOC(f->X, (size_t)n * d * 4);
    RPF_ALLOC(f->R, (size_t)T * H * n_try * d * 4);
    RPF_ALLOC(f->split, (size_t)T * H * 8);
    RPF_ALLOC(f->split_idx, (size_t)T * H * 4);
    RPF_ALLOC(f->chosen, (size_t)T * H * 4);
    RPF_ALLOC(f->perm[0], (size_t)T * n * 4);
    RPF_ALLOC(f->perm[1], (size_t)T * n * 4);
    RPF_ALLOC(f->leaf_of, (size_t)T * n * 4);
    RPF_ALLOC(f->centroid, (size_t)T * nleaf * d * 4);
    if (xc_eager) RPF_ALLOC(f->Xc, (size_t)xc_bytes);
    RPF_ALLOC(f->nrm, (size_t)T * n * 8);
    if (grid) {
        RPF_ALLOC(f->Xq, (size_t)n * dq);
        RPF_ALLOC(f->qn, (size_t)n * sizeof(LatNorm));
        f->dq = dq;
        f->bytes += (size_t)n * dq + (size_t)n * sizeof(LatNorm);
    }
    RPF_ALLOC(f->err, 64);
    RPF_ALLOC(f->stats, kStatSlots * 8 * 8 + 256);
    f->fault = f->stats + kStatSlots * 8;
    fill_u64(f->fault, 1, 0, s);
    f->pin_slot = pin_take();
    RPF_ALLOC(f->heap_leaf, ((size_t)LB + 1) * sizeof(int32_t));  // leaf ids < lbase + 2^(L+1)
    RPF_ALLOC(f->d_batch_off, ((size_t)count + 1) * sizeof(int64_t));
    if (nseg_tot) RPF_ALLOC(f->d_segs, nseg_tot * sizeof(SegDesc));
    if (nchunk_tot) RPF_ALLOC(f->d_chunks, nchunk_tot * sizeof(ChunkDesc));
    RPF_ALLOC(f->d_leaves, nleaf * sizeof(LeafDesc));
    if (ncopy_tot) RPF_ALLOC(f->d_copy, ncopy_tot * sizeof(LeafDesc));
    if (nseg_tot && any_link) RPF_ALLOC(f->d_look, nseg_tot * sizeof(LookDesc));
    std::vector<SubItem> sub_items;
    if (sub_level >= 0) {
        const LevelPlan &lv = levels[sub_level];
        for (size_t k = 0; k < lv.segs.size(); k++)
            sub_items.push_back(SubItem{lv.segs[k].off, lv.segs[k].size, lv.segs[k].heap, lv.hbase[k], 0});
        int mm = 0;
        for (int l = sub_level; l < L; l++) mm = std::max(mm, levels[l].max_m);
        RPF_ALLOC(f->d_sub_items, sub_items.size() * sizeof(SubItem));
        RPF_ALLOC(f->sub_next, 16);
        f->sub_level = sub_level;
        f->sub_max_m = mm;
        f->n_sub_items = (int64_t)sub_items.size();
        f->subtree_on = (p->build_flags & RPF_BUILD_SUBTREES) != 0;
        hipMemcpyAsync(f->d_sub_items, sub_items.data(), sub_items.size() * sizeof(SubItem), hipMemcpyHostToDevice, s);
    }

    // ---- descriptors (host copies stay alive until the synchronisation below)
    std::vector<SegDesc> all_segs;
    std::vector<ChunkDesc> all_chunks;
    std::vector<LeafDesc> all_copy;
    std::vector<LookDesc> all_look;
    for (auto &lv : levels) {
        all_segs.insert(all_segs.end(), lv.segs.begin(), lv.segs.end());
        lv.look.resize(lv.segs.size(), LookDesc{{-1, -1}, {0, 0}});
        all_look.insert(all_look.end(), lv.look.begin(), lv.look.end());
        all_chunks.insert(all_chunks.end(), lv.chunks.begin(), lv.chunks.end());
        all_copy.insert(all_copy.end(), lv.copy.begin(), lv.copy.end());
    }
    std::vector<int32_t> hl((size_t)LB + 1, -1);
    for (size_t i = 0; i < leaves.size(); i++) hl[leaves[i].heap] = (int32_t)i;
    std::vector<int64_t> boff((size_t)count + 1);
    for (int i = 0; i < count; i++) boff[i] = roots[i].offset;
    boff[count] = n;
    hipMemcpyAsync(f->d_batch_off, boff.data(), boff.size() * 8, hipMemcpyHostToDevice, s);
    if (nseg_tot) hipMemcpyAsync(f->d_segs, all_segs.data(), nseg_tot * sizeof(SegDesc), hipMemcpyHostToDevice, s);
    if (nchunk_tot)
        hipMemcpyAsync(f->d_chunks, all_chunks.data(), nchunk_tot * sizeof(ChunkDesc), hipMemcpyHostToDevice, s);
    if (ncopy_tot) hipMemcpyAsync(f->d_copy, all_copy.data(), ncopy_tot * sizeof(LeafDesc), hipMemcpyHostToDevice, s);
    if (f->d_look) hipMemcpyAsync(f->d_look, all_look.data(), nseg_tot * sizeof(LookDesc), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(f->d_leaves, leaves.data(), nleaf * sizeof(LeafDesc), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(f->heap_leaf, hl.data(), hl.size() * 4, hipMemcpyHostToDevice, s);
    fill_u64(f->split, (int64_t)T * H, 0x7ff8000000000000ull, s);  // binary64 quiet NaN
    fill_u32(f->split_idx, (int64_t)T * H, 0xffffffffu, s);
    fill_u32(f->chosen, (int64_t)T * H, 0xffffffffu, s);
    launch_check(s, "descriptor upload");

    // ---- temporaries of the multi-block path (kept by the forest until released)
    LargeBufs &lb = f->lb;
    auto talloc = [&](void **ptr, size_t sz) -> bool {
        if (!sz) { *ptr = nullptr; return true; }
        *ptr = cache_alloc(sz, s);
        if (!*ptr) return false;
        f->tmps.push_back(*ptr);
        return true;
    };
    bool ok = true;
    if (max_seg_large > 0) {
        ok &= talloc((void **)&lb.keys, (size_t)T * n * 8);
        if (n_try > 1) ok &= talloc((void **)&lb.praw, (size_t)T * n * 8);
        ok &= talloc((void **)&lb.state, (size_t)T * max_seg_large * sizeof(SelState));
        ok &= talloc((void **)&lb.hist, (size_t)T * max_seg_large * 4 * kDigitBins);
        ok &= talloc((void **)&lb.cand, (size_t)T * max_seg_large * cand_bytes() * kCandCap);
        ok &= talloc((void **)&lb.cand_cnt, (size_t)T * max_seg_large * 4);
        ok &= talloc((void **)&lb.lcount, (size_t)T * max_chunk_large * 4);
        ok &= talloc((void **)&lb.part, (size_t)T * max_chunk_large * 8);
    }
    if (any_link) {
        ok &= talloc((void **)&lb.ahead, (size_t)T * n * 16);
        ok &= talloc((void **)&lb.keys2, (size_t)T * n * 8);
    }
    if (any_large_fed) ok &= talloc((void **)&lb.hist2, (size_t)T * max_seg_large * 4 * kDigitBins);
    if (!ok) {
        fail(RPF_ENOMEM, "rpf_build: temporary allocation failed");
        return bail(RPF_ENOMEM);
    }
    f->levels = levels;
    f->lds_max = lds_max;

    // all-points tile jobs (same leaf shapes in every tree)
    {
        int MB = 8;
        if (max_leaf <= 32) MB = 1;
        else if (max_leaf <= 64) MB = 2;
        else if (max_leaf <= 128) MB = 4;
        const int TR = 32 * MB;
        std::vector<TileJob> jobs;  // tree 0; the device copies them to the other trees
        for (size_t li = 0; li < leaves.size(); li++) {
            const LeafDesc &lf = leaves[li];
            const int nt = (lf.size + TR - 1) / TR;
            for (int I = 0; I < nt; I++)
                for (int J = 0; J < nt; J++) {
                    TileJob j;
                    j.a_off = lf.off + (int64_t)I * TR;
                    j.b_off = lf.off + (int64_t)J * TR;
                    j.a_rows = std::min(TR, lf.size - I * TR);
                    j.b_rows = std::min(TR, lf.size - J * TR);
                    j.tree = 0;
                    j.same = I == J;
                    j.b_pos = J * TR;
                    j.leaf_m = lf.size;
                    j.leaf = (int32_t)li;
                    j.pad = 0;
                    jobs.push_back(j);
                }
        }
        f->n_jobs_tree = (int64_t)jobs.size();
        for (auto &lf : leaves) f->tile_flops_tree += 2.0 * d * (double)lf.size * (double)lf.size;
        f->job_mb = MB;
        RPF_ALLOC(f->d_jobs, (size_t)T * jobs.size() * sizeof(TileJob));
        hipMemcpyAsync(f->d_jobs, jobs.data(), jobs.size() * sizeof(TileJob), hipMemcpyHostToDevice, s);
        replicate_jobs(f->d_jobs, f->n_jobs_tree, T, s);
        hipStreamSynchronize(s);  // the host job list and descriptors die with this scope
        f->bytes += (size_t)T * jobs.size() * sizeof(TileJob);
    }
#undef RPF_ALLOC
    *out = f;
    return RPF_OK;
}

// The build proper: launches only (no allocation, no synchronisation, no memset), so a
// stream capture can record it.  X and the directions must be in place.
static void build_launches(rpf_forest *f, hipStream_t s) {
    const int64_t n = f->n, H = f->H;
    const int d = f->d, T = f->T, n_try = f->n_try, dp = f->dp, prec = f->prec;
    const double esz = prec == RPF_DIST_FP32 ? 4.0 : 2.0;
    const int64_t nleaf = (int64_t)f->leaves.size();
    const bool vec = (d % 4) == 0;
    launch_iota(s, f->perm[0], n, T);
    launch_check(s, "iota");
    int cur = 0;
    for (size_t l = 0; l < f->levels.size(); l++) {
        LevelPlan &lv = f->levels[l];
        const int32_t *pin = f->perm[cur];
        int32_t *pout = f->perm[cur ^ 1];
        launch_copy_segments(s, f->d_copy + lv.copy_off, (int)lv.copy.size(), T, pin, pout, n);
        launch_check(s, "copy_segments");
        if (f->subtree_on && (int)l == f->sub_level) {
            // this level and every one below it: one persistent launch, leaf order in pout
            double bytes = 0;
            for (size_t k = l; k < f->levels.size(); k++)
                for (auto &sg : f->levels[k].segs) bytes += (double)T * sg.size * (4.0 * d + 4 + 8);
            ProfScope ps(s, "subtree_levels", bytes, 0);
            launch_subtree(s, vec, f->X, d, f->R, H, f->d_sub_items, (int)f->n_sub_items, T, f->n0, pin, pout, n,
                           f->split, f->split_idx, f->chosen, f->err, f->sub_next, f->sub_max_m, f->lds_max);
            launch_check(s, "subtree");
            cur ^= 1;
            break;
        }
        int64_t members = 0;
        for (auto &sg : lv.segs) members += sg.size;
        LevelLink lk;
        if (lv.lead) {
            lk.look = f->d_look + lv.seg_off;
            lk.ahead = f->lb.ahead;
            lk.keys_next = f->lb.keys2;
            if (f->levels[l + 1].large) {
                lk.hist_next = f->lb.hist2;
                lk.nseg_next = (int)f->levels[l + 1].segs.size();
            }
        }
        if (lv.fed) {
            lk.keys_in = f->lb.keys2;
            if (lv.large) lk.hist_in = f->lb.hist2;
        }
        // the roots: identity permutation in every tree, so one read of X serves all trees
        lk.roots = l == 0 && lv.lead && lv.large && vec && d <= 128;
        // grid forests: the rows come from the int8 copy (one byte a coordinate)
        lk.xq = f->Xq;
        lk.dq = f->dq;
        const double xb = f->Xq ? (double)f->dq : 4.0 * d;  // bytes of a row read
        // algorithmic bytes: X rows (none on a fed level), ids and keys, the children's
        // projections out and back on a lead level
        const double row_bytes = (lv.fed ? 8.0 : xb + 8) + 4 + (lv.lead ? 16.0 : 0.0);
        const double proj_bytes = lk.roots ? members * (4.0 * d) + (double)T * members * (8 + 16)
                                           : (double)T * members * (xb + 4 + 8 + (lv.lead ? 16.0 : 0.0));
        if (!lv.large) {
            ProfScope ps(s, "level_small", (double)T * members * row_bytes, 0);
            launch_level_small(s, vec, f->X, d, f->R, H, n_try, f->d_segs + lv.seg_off, (int)lv.segs.size(),
                               lv.max_m, T, pin, pout, n, f->split, f->split_idx, f->chosen, f->err, lk);
            launch_check(s, "level_small");
        } else {
            launch_level_large(s, vec, f->X, d, f->R, H, n_try, f->d_segs + lv.seg_off, (int)lv.segs.size(),
                               f->d_chunks + lv.chunk_off, (int)lv.chunks.size(), T, pin, pout, n, f->split,
                               f->split_idx, f->chosen, f->err, f->lb, proj_bytes, lk);
            launch_check(s, "level_large");
        }
        cur ^= 1;
    }
    f->final_buf = cur;
    if (f->Xc) {  // leaves above one tile: the all-points search reads the centred copy
        ProfScope ps(s, "leaf_finalize", (double)T * n * (8.0 * d + dp * esz + 16), 0);
        launch_leaf_finalize(s, prec, f->X, d, dp, f->d_leaves, (int)nleaf, T, f->perm[cur], n, f->leaf_of,
                             f->centroid, f->Xc, f->nrm, f->max_leaf, f->lds_max);
        launch_check(s, "leaf_finalize");
    } else if (f->Xq && f->max_leaf > 256) {
        // grid forest with leaves above one tile: the all-points tiles read the int8 copy and
        // its norms; leaf_of is all they need.  Centroids, norms and the query copies are made
        // together by the first query (rpf::ensure_leaf_copies)
        ProfScope ps(s, "leaf_finalize", (double)T * n * 12.0, 0);
        launch_leaf_ids(s, f->d_leaves, (int)nleaf, T, f->perm[cur], n, f->leaf_of);
        launch_check(s, "leaf_ids");
    } else {  // centroids and norms only: the tiles centre the rows as they stage them
        ProfScope ps(s, "leaf_finalize", (double)T * n * (4.0 * d + 16), 0);
        launch_leaf_stats(s, prec, f->X, d, dp, f->d_leaves, (int)nleaf, T, f->perm[cur], n, f->leaf_of, f->centroid,
                          f->nrm, f->max_leaf);
        launch_check(s, "leaf_stats");
    }
}

// The leaf-ordered centred copy for queries, made once, on the first call that needs it:
// later callers on other streams wait for the event recorded after the copy kernel.
rpf_status rpf::ensure_leaf_copies(const rpf_forest *cf, hipStream_t s, bool may_make) {
    rpf_forest *f = const_cast<rpf_forest *>(cf);
    if (f->split_rule == RPF_SPLIT_UNIFORM)
        return fail(RPF_EINVAL, "queries need a median-rule forest (a uniform-rule forest has no query copies)");
    std::lock_guard<std::mutex> lk(f->xc_mu);
    if (f->Xc) return f->xc_ev ? check_hip(hipStreamWaitEvent(s, f->xc_ev, 0), "leaf copies: wait") : RPF_OK;
    if (!may_make)
        return fail(RPF_ENOTREADY, "the forest's query copies do not exist yet: they are made (allocated) by its "
                                   "first rpf_query call or by rpf_server_create");
    if (capturing(s))
        return fail(RPF_EINVAL, "the forest's query copies are made on its first query, which cannot be recorded: "
                                "run one query before the capture");
    const size_t bytes = (size_t)f->T * f->n * f->dp * (f->prec == RPF_DIST_FP32 ? 4 : 2);
    void *p = cache_alloc(bytes, s);
    if (!p) return fail(RPF_ENOMEM, "device allocation of the forest's query copies failed");
    if (f->Xq && f->max_leaf > 256)  // grid forest: centroids and norms were left to this call
        launch_leaf_finalize(s, f->prec, f->X, f->d, f->dp, f->d_leaves, (int)f->leaves.size(), f->T,
                             f->perm[f->final_buf], f->n, f->leaf_of, f->centroid, p, f->nrm, f->max_leaf, f->lds_max);
    else
        launch_leaf_copy(s, f->prec, f->X, f->d, f->dp, f->d_leaves, (int)f->leaves.size(), f->T,
                         f->perm[f->final_buf], f->n, f->centroid, p);
    const std::string le = take_launch_error();
    if (!le.empty()) {
        cache_free(p, s);
        return fail(RPF_EDEVICE, "leaf copies: " + le);
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, s) != hipSuccess) {
        if (ev) hipEventDestroy(ev);
        ev = nullptr;
        const rpf_status st = check_hip(hipStreamSynchronize(s), "leaf copies");  // no event: finish them here
        if (st != RPF_OK) {
            cache_free_idle(p);
            return st;
        }
    }
    f->xc_ev = ev;
    f->Xc = p;
    f->bytes += bytes;
    return RPF_OK;
}

static void release_temporaries(rpf_forest *f, hipStream_t s) {
    for (void *q : f->tmps) cache_free(q, s);
    f->tmps.clear();
    f->lb = LargeBufs{};
}

static rpf_status build_impl(const float *X, const int64_t *sizes, int count, int32_t d, const rpf_params *p,
                             void *stream, rpf_forest **out) {
    if (out) *out = nullptr;
    if (!X) return fail(RPF_EINVAL, "rpf_build: X is NULL");
    rpf_forest *f = nullptr;
    rpf_status st = prepare_forest(sizes, count, d, p, stream, &f);
    if (st != RPF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    auto bail = [&](rpf_status e) {
        hipStreamSynchronize(s);
        free_forest_memory(f);
        delete f;
        return e;
    };
    const int64_t n = f->n, H = f->H;
    const int T = f->T, n_try = f->n_try;
    // ---- inputs: copy, then reject non-finite values (one synchronisation)
    fill_u32(f->err, 16, 0, s);
    fill_u32(f->stats, kStatSlots * 8 * 2, 0, s);
    launch_copy_nonfinite(s, X, f->X, n * d, f->err);
    if (H > 0) launch_copy_nonfinite(s, p->directions_dev, f->R, T * H * n_try * d, f->err + 1);
    if (f->Xq) launch_grid_quantise(s, f->X, n, d, f->dq, f->Xq, f->qn, f->err + 4);
    launch_check(s, "input copy and check");
    int32_t flags[5] = {0, 0, 0, 0, 0};
    if ((st = check_hip(hipMemcpyAsync(flags, f->err, 20, hipMemcpyDeviceToHost, s), "read flags")) != RPF_OK) return bail(st);
    if ((st = check_hip(hipStreamSynchronize(s), "rpf_build input check")) != RPF_OK) return bail(st);
    if (flags[0]) { fail(RPF_EINVAL, "rpf_build: X holds NaN or Inf"); return bail(RPF_EINVAL); }
    if (flags[1]) { fail(RPF_EINVAL, "rpf_build: directions hold NaN or Inf"); return bail(RPF_EINVAL); }
    if (flags[4]) {
        fail(RPF_EINVAL, "rpf_build: RPF_DIST_U8GRID needs every coordinate of X to be float(k) / 255 for an integer "
                         "k in [0, 255]");
        return bail(RPF_EINVAL);
    }
    fill_u32(f->err, 16, 0, s);
    build_launches(f, s);
    release_temporaries(f, s);
    launch_check(s, "rpf_build tail");
    const std::string le = take_launch_error();
    if (!le.empty()) {
        fail(RPF_EDEVICE, "rpf_build: " + le);
        return bail(RPF_EDEVICE);
    }
    *out = f;
    return RPF_OK;
}

// ---------------------------------------------------------------- uniform split rule

// Leaf pass of a uniform-rule forest: each tree has its own leaf table (row t of the
// [T][leaf_stride] table), so the leaf kernels run once per tree on that tree's slices.
static void uniform_leaf_pass(rpf_forest *f, hipStream_t s) {
    const int64_t n = f->n, ls = f->leaf_stride;
    const int d = f->d, dp = f->dp, prec = f->prec;
    const size_t esz = prec == RPF_DIST_FP32 ? 4 : 2;
    const int32_t *perm = f->perm[f->final_buf];
    for (int t = 0; t < f->T; t++) {
        const LeafDesc *lv = f->d_leaves + (int64_t)t * ls;
        const int nl = f->tree_nleaf[t];
        const int32_t *pt = perm + (int64_t)t * n;
        int32_t *lo = f->leaf_of + (int64_t)t * n;
        float *cen = f->centroid + (int64_t)t * ls * d;
        float2 *nr = f->nrm + (int64_t)t * n;
        if (f->Xc)
            launch_leaf_finalize(s, prec, f->X, d, dp, lv, nl, 1, pt, n, lo, cen,
                                 static_cast<uint8_t *>(f->Xc) + (size_t)t * n * dp * esz, nr, f->max_leaf, f->lds_max);
        else if (f->Xq && f->max_leaf > 256)
            launch_leaf_ids(s, lv, nl, 1, pt, n, lo);
        else
            launch_leaf_stats(s, prec, f->X, d, dp, lv, nl, 1, pt, n, lo, cen, nr, f->max_leaf);
    }
    launch_check(s, "uniform leaf pass");
}

// Grow a forest by the uniform split rule: a host-driven level loop over the open nodes of
// every tree (the shapes depend on the data), then the same leaf pass and all-points tile
// jobs as the median rule, per tree.  Synchronises the stream once per level.
static rpf_status build_uniform(const float *X, int64_t n, int32_t d, const rpf_params *p, void *stream,
                                rpf_forest **out) {
    if (out) *out = nullptr;
    if (!out) return fail(RPF_EINVAL, "rpf_build: out is NULL");
    if (!X) return fail(RPF_EINVAL, "rpf_build: X is NULL");
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(RPF_EINVAL, "rpf_build: n must be in [1, 2^31)");
    if (d < 1) return fail(RPF_EINVAL, "rpf_build: d must be >= 1");
    if (d > 4096) return fail(RPF_EINVAL, "rpf_build: d above 4096 is not supported (per-block staging)");
    if (p->n_trees < 1 || p->n_trees > 65535) return fail(RPF_EINVAL, "rpf_build: n_trees must be in [1, 65535]");
    if (p->leaf_size < 1) return fail(RPF_EINVAL, "rpf_build: leaf_size must be >= 1");
    if (p->n_try < 1) return fail(RPF_EINVAL, "rpf_build: n_try must be >= 1");
    if (p->dist_prec < RPF_DIST_FP32 || p->dist_prec > RPF_DIST_U8GRID)
        return fail(RPF_EINVAL, "rpf_build: unknown dist_prec");
    if (p->build_flags & ~RPF_BUILD_SUBTREES) return fail(RPF_EINVAL, "rpf_build: unknown build_flags");
    const int64_t T = p->n_trees, TN = T * n;
    if (TN >= ((int64_t)1 << 40)) return fail(RPF_EINVAL, "rpf_build: n_trees * n too large");
    const int n0 = p->leaf_size, n_try = p->n_try;
    const uint64_t seed = p->seed;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    hipGetDevice(&dev);
    const bool grid = p->dist_prec == RPF_DIST_U8GRID;
    const int prec = (p->dist_prec == RPF_DIST_BF16X3 || grid) ? RPF_DIST_FP32 : p->dist_prec;
    const int dq = grid ? (d + 63) & ~63 : 0;
    const int dp = (d + 7) & ~7;
    const size_t esz = prec == RPF_DIST_FP32 ? 4 : 2;
    const int lds_max = lds_limit(dev);
    int small_max = kChunk;
    while (small_max > 2 && uni_block_lds(small_max, d, n_try) > (size_t)lds_max) small_max /= 2;
    const bool chunked = n > small_max;  // only nodes above small_max take the chunked path
    // open nodes are larger than n0, chunked ones larger than small_max
    const int64_t seg_cap = TN / (n0 + 1) + T + 1;
    const int64_t lseg_cap = chunked ? TN / (small_max + 1) + T + 1 : 0;
    const int64_t chunk_cap = chunked ? TN / kChunk + lseg_cap + 1 : 0;

    uint64_t bytes = (uint64_t)n * d * 4 + (uint64_t)TN * (4 + 4 + 8);  // X, perm, leaf_of, nrm
    if (grid) bytes += (uint64_t)n * dq + (uint64_t)n * sizeof(LatNorm);
    uint64_t tmp_bytes = (uint64_t)seg_cap * (sizeof(UniSeg) + sizeof(UniSplit));
    if (chunked)
        tmp_bytes += (uint64_t)n_try * TN * 8 + (uint64_t)TN * 4 + (uint64_t)chunk_cap * (sizeof(UniChunk) + n_try * 24 + 8) +
                     (uint64_t)lseg_cap * (sizeof(UniSeg) + sizeof(UniSplit) + n_try * 8);
    if (p->mem_budget_bytes && bytes + tmp_bytes > p->mem_budget_bytes)
        return fail(RPF_ENOMEM, "rpf_build: forest needs " + std::to_string(bytes + tmp_bytes) +
                                    " bytes, over mem_budget_bytes");

    rpf_forest *f = new rpf_forest();
    f->n = n; f->d = d; f->T = (int32_t)T; f->n0 = n0; f->n_try = n_try; f->L = 0; f->H = 0;
    f->prec = prec; f->tile_prec = p->dist_prec; f->dp = dp; f->device = dev; f->lds_max = lds_max;
    f->split_rule = RPF_SPLIT_UNIFORM; f->seed = seed;
    rpf_batch_entry root{};
    root.offset = 0; root.n = n;
    f->batch = {root};
    f->bytes = bytes;
    std::vector<void *> temps;
    auto bail = [&](rpf_status st) {
        hipStreamSynchronize(s);
        for (void *q : temps) cache_free_idle(q);
        free_forest_memory(f);
        delete f;
        return st;
    };
    auto dalloc = [&](size_t sz) -> void * { return sz ? cache_alloc(sz, s) : nullptr; };
#define RPF_UALLOC(ptr, sz)                                                                   \
    do {                                                                                      \
        const size_t _sz = (size_t)(sz);                                                      \
        (ptr) = static_cast<std::remove_reference_t<decltype(ptr)>>(dalloc(_sz));            \
        if (_sz && !(ptr)) {                                                                  \
            fail(RPF_ENOMEM, "rpf_build: device allocation of " #ptr " failed");             \
            return bail(RPF_ENOMEM);                                                          \
        }                                                                                     \
    } while (0)
#define RPF_UTEMP(ptr, sz)                                                                    \
    do {                                                                                      \
        RPF_UALLOC(ptr, sz);                                                                  \
        if (ptr) temps.push_back((void *)(ptr));                                              \
    } while (0)

    RPF_UALLOC(f->X, (size_t)n * d * 4);
    RPF_UALLOC(f->perm[0], (size_t)TN * 4);
    RPF_UALLOC(f->leaf_of, (size_t)TN * 4);
    RPF_UALLOC(f->nrm, (size_t)TN * 8);
    RPF_UALLOC(f->err, 64);
    RPF_UALLOC(f->stats, kStatSlots * 8 * 8 + 256);
    f->fault = f->stats + kStatSlots * 8;
    fill_u64(f->fault, 1, 0, s);
    f->pin_slot = pin_take();
    if (grid) {
        RPF_UALLOC(f->Xq, (size_t)n * dq);
        RPF_UALLOC(f->qn, (size_t)n * sizeof(LatNorm));
        f->dq = dq;
    }
    UniSeg *d_seg = nullptr, *d_lseg = nullptr;
    UniSplit *d_split = nullptr, *d_lsplit = nullptr;
    UniChunk *d_chunk = nullptr;
    UniBufs ub;
    RPF_UTEMP(d_seg, (size_t)seg_cap * sizeof(UniSeg));
    RPF_UTEMP(d_split, (size_t)seg_cap * sizeof(UniSplit));
    if (chunked) {
        RPF_UTEMP(d_lseg, (size_t)lseg_cap * sizeof(UniSeg));
        RPF_UTEMP(d_lsplit, (size_t)lseg_cap * sizeof(UniSplit));
        RPF_UTEMP(d_chunk, (size_t)chunk_cap * sizeof(UniChunk));
        RPF_UTEMP(ub.P, (size_t)n_try * TN * 8);
        RPF_UTEMP(ub.part, (size_t)chunk_cap * n_try * 8);
        RPF_UTEMP(ub.mm, (size_t)chunk_cap * n_try * sizeof(double2));
        RPF_UTEMP(ub.mu, (size_t)lseg_cap * n_try * 8);
        RPF_UTEMP(ub.lcount, (size_t)chunk_cap * 4);
        RPF_UTEMP(ub.loff, (size_t)chunk_cap * 4);
        RPF_UTEMP(ub.tmp, (size_t)TN * 4);
    }

    // ---- inputs: copy, then reject non-finite values (one synchronisation)
    fill_u32(f->err, 16, 0, s);
    fill_u32(f->stats, kStatSlots * 8 * 2, 0, s);
    launch_copy_nonfinite(s, X, f->X, n * d, f->err);
    if (f->Xq) launch_grid_quantise(s, f->X, n, d, dq, f->Xq, f->qn, f->err + 4);
    launch_iota(s, f->perm[0], n, (int)T);
    launch_check(s, "input copy and check");
    int32_t flags[5] = {0, 0, 0, 0, 0};
    rpf_status st;
    if ((st = check_hip(hipMemcpyAsync(flags, f->err, 20, hipMemcpyDeviceToHost, s), "read flags")) != RPF_OK) return bail(st);
    if ((st = check_hip(hipStreamSynchronize(s), "rpf_build input check")) != RPF_OK) return bail(st);
    if (flags[0]) { fail(RPF_EINVAL, "rpf_build: X holds NaN or Inf"); return bail(RPF_EINVAL); }
    if (flags[4]) {
        fail(RPF_EINVAL, "rpf_build: RPF_DIST_U8GRID needs every coordinate of X to be float(k) / 255 for an integer "
                         "k in [0, 255]");
        return bail(RPF_EINVAL);
    }

    // ---- growth, level by level
    struct Open { int64_t pos, heap; int32_t size, tree, depth; };
    std::vector<Open> open;
    std::vector<std::vector<LeafDesc>> tleaves(T);
    f->nodes.assign(T, {});
    int max_depth = 0;
    auto close_leaf = [&](const Open &o) {
        tleaves[o.tree].push_back(LeafDesc{o.pos - (int64_t)o.tree * n, o.size, 0});
        max_depth = std::max(max_depth, (int)o.depth);
    };
    for (int64_t t = 0; t < T; t++) {
        const Open r{t * n, 1, (int32_t)n, (int32_t)t, 0};
        if (n > n0) open.push_back(r);
        else close_leaf(r);
    }
    std::vector<UniSeg> hs, hl;
    std::vector<UniChunk> hc;
    std::vector<int64_t> is_small, is_large;  // indices into `open`
    std::vector<UniSplit> rs, rl;
    while (!open.empty()) {
        hs.clear(); hl.clear(); hc.clear(); is_small.clear(); is_large.clear();
        int max_small = 2;
        for (int64_t k = 0; k < (int64_t)open.size(); k++) {
            const Open &o = open[k];
            UniSeg g{o.pos, o.heap, o.size, o.tree, 0, 0};
            if (o.size <= small_max) {
                hs.push_back(g);
                is_small.push_back(k);
                max_small = std::max(max_small, (int)o.size);
            } else {
                g.chunk0 = (int32_t)hc.size();
                g.nchunk = (int32_t)((o.size + kChunk - 1) / kChunk);
                for (int q = 0; q < g.nchunk; q++) {
                    const int64_t st0 = o.pos + (int64_t)q * kChunk;
                    hc.push_back(UniChunk{st0, (int32_t)std::min<int64_t>(kChunk, o.pos + o.size - st0),
                                          (int32_t)hl.size()});
                }
                hl.push_back(g);
                is_large.push_back(k);
            }
        }
        if ((int64_t)hs.size() > seg_cap || (int64_t)hl.size() > lseg_cap || (int64_t)hc.size() > chunk_cap) {
            fail(RPF_EINTERNAL, "rpf_build: uniform growth outgrew its node capacity");
            return bail(RPF_EINTERNAL);
        }
        if (!hs.empty()) {
            hipMemcpyAsync(d_seg, hs.data(), hs.size() * sizeof(UniSeg), hipMemcpyHostToDevice, s);
            ProfScope ps(s, "uniform_level_block", 0, 0);
            launch_uni_block(s, f->X, d, n_try, seed, d_seg, (int)hs.size(), max_small, f->perm[0], d_split);
        }
        if (!hl.empty()) {
            hipMemcpyAsync(d_lseg, hl.data(), hl.size() * sizeof(UniSeg), hipMemcpyHostToDevice, s);
            hipMemcpyAsync(d_chunk, hc.data(), hc.size() * sizeof(UniChunk), hipMemcpyHostToDevice, s);
            ProfScope ps(s, "uniform_level_chunked", 0, 0);
            launch_uni_chunked(s, f->X, d, n_try, seed, d_lseg, (int)hl.size(), d_chunk, (int)hc.size(), f->perm[0], TN,
                               ub, d_lsplit);
        }
        rs.resize(hs.size());
        rl.resize(hl.size());
        if (!rs.empty()) hipMemcpyAsync(rs.data(), d_split, rs.size() * sizeof(UniSplit), hipMemcpyDeviceToHost, s);
        if (!rl.empty()) hipMemcpyAsync(rl.data(), d_lsplit, rl.size() * sizeof(UniSplit), hipMemcpyDeviceToHost, s);
        if ((st = check_hip(hipStreamSynchronize(s), "rpf_build uniform level")) != RPF_OK) return bail(st);
        {
            const std::string le = take_launch_error();
            if (!le.empty()) {
                fail(RPF_EDEVICE, "rpf_build: " + le);
                return bail(RPF_EDEVICE);
            }
        }
        std::vector<Open> next;
        auto settle = [&](const Open &o, const UniSplit &r) -> bool {
            if (r.nl < 0 || r.nl > o.size || r.chosen < 0 || r.chosen >= n_try) return false;
            f->nodes[o.tree].push_back(rpf_node{o.heap, r.c, o.size, r.nl, r.chosen, o.depth});
            if (r.nl == 0 || r.nl == o.size) {  // an empty child: the node stays whole
                close_leaf(o);
                return true;
            }
            const Open kids[2] = {{o.pos, 2 * o.heap, r.nl, o.tree, o.depth + 1},
                                  {o.pos + r.nl, 2 * o.heap + 1, o.size - r.nl, o.tree, o.depth + 1}};
            for (const Open &c : kids) {
                if (c.size > n0 && c.depth < kUniformDepth) next.push_back(c);
                else close_leaf(c);
            }
            return true;
        };
        bool ok = true;
        for (size_t k = 0; k < hs.size(); k++) ok &= settle(open[is_small[k]], rs[k]);
        for (size_t k = 0; k < hl.size(); k++) ok &= settle(open[is_large[k]], rl[k]);
        if (!ok) {
            fail(RPF_EINTERNAL, "rpf_build: a uniform split came back out of range");
            return bail(RPF_EINTERNAL);
        }
        open.swap(next);
    }
    for (void *q : temps) cache_free(q, s);
    temps.clear();

    // ---- leaves: left to right within each tree (ordinal = leaf id), one padded table
    int64_t stride = 0;
    int max_leaf = 0;
    f->tree_nleaf.resize(T);
    for (int64_t t = 0; t < T; t++) {
        auto &lv = tleaves[t];
        std::sort(lv.begin(), lv.end(), [](const LeafDesc &a, const LeafDesc &b) { return a.off < b.off; });
        int64_t at = 0;
        for (size_t i = 0; i < lv.size(); i++) {
            if (lv[i].off != at) {
                fail(RPF_EINTERNAL, "rpf_build: uniform leaves do not tile the permutation");
                return bail(RPF_EINTERNAL);
            }
            at += lv[i].size;
            lv[i].heap = (int32_t)i;
            max_leaf = std::max(max_leaf, (int)lv[i].size);
        }
        if (at != n) {
            fail(RPF_EINTERNAL, "rpf_build: uniform leaves do not tile the permutation");
            return bail(RPF_EINTERNAL);
        }
        f->tree_nleaf[t] = (int32_t)lv.size();
        stride = std::max<int64_t>(stride, (int64_t)lv.size());
    }
    f->leaf_stride = stride;
    f->max_leaf = max_leaf;
    f->L = max_depth;
    f->batch[0].depth = max_depth;
    int MB = 8;
    if (max_leaf <= 32) MB = 1;
    else if (max_leaf <= 64) MB = 2;
    else if (max_leaf <= 128) MB = 4;
    const int TR = 32 * MB;
    f->job_mb = MB;
    std::vector<TileJob> jobs;
    f->job_off.assign(T + 1, 0);
    f->flops_off.assign(T + 1, 0.0);
    for (int64_t t = 0; t < T; t++) {
        double fl = 0;
        for (size_t li = 0; li < tleaves[t].size(); li++) {
            const LeafDesc &lf = tleaves[t][li];
            const int nt = (lf.size + TR - 1) / TR;
            for (int I = 0; I < nt; I++)
                for (int J = 0; J < nt; J++) {
                    TileJob j;
                    j.a_off = lf.off + (int64_t)I * TR;
                    j.b_off = lf.off + (int64_t)J * TR;
                    j.a_rows = std::min(TR, lf.size - I * TR);
                    j.b_rows = std::min(TR, lf.size - J * TR);
                    j.tree = (int32_t)t;
                    j.same = I == J;
                    j.b_pos = J * TR;
                    j.leaf_m = lf.size;
                    j.leaf = (int32_t)li;
                    j.pad = 0;
                    jobs.push_back(j);
                }
            fl += 2.0 * d * (double)lf.size * (double)lf.size;
        }
        f->job_off[t + 1] = (int64_t)jobs.size();
        f->flops_off[t + 1] = f->flops_off[t] + fl;
    }
    f->n_jobs_tree = 0;
    f->tile_flops_tree = f->flops_off[T] / (double)T;
    std::vector<LeafDesc> table((size_t)(T * stride), LeafDesc{0, 0, -1});
    for (int64_t t = 0; t < T; t++)
        std::copy(tleaves[t].begin(), tleaves[t].end(), table.begin() + t * stride);
    const bool xc_eager = max_leaf > 256 && !grid;
    const uint64_t more = (uint64_t)T * stride * (d * 4 + sizeof(LeafDesc)) + (uint64_t)(stride + 1) * 4 +
                          (uint64_t)jobs.size() * sizeof(TileJob) + (xc_eager ? (uint64_t)TN * dp * esz : 0);
    if (p->mem_budget_bytes && f->bytes + more > p->mem_budget_bytes) {
        fail(RPF_ENOMEM, "rpf_build: forest needs " + std::to_string(f->bytes + more) + " bytes, over mem_budget_bytes");
        return bail(RPF_ENOMEM);
    }
    RPF_UALLOC(f->d_leaves, table.size() * sizeof(LeafDesc));
    RPF_UALLOC(f->heap_leaf, (size_t)(stride + 1) * 4);
    RPF_UALLOC(f->centroid, (size_t)T * stride * d * 4);
    RPF_UALLOC(f->d_jobs, jobs.size() * sizeof(TileJob));
    if (xc_eager) RPF_UALLOC(f->Xc, (size_t)TN * dp * esz);
    f->bytes += more;
    std::vector<int32_t> ident((size_t)stride + 1);
    for (int64_t i = 0; i <= stride; i++) ident[i] = (int32_t)i;
    hipMemcpyAsync(f->d_leaves, table.data(), table.size() * sizeof(LeafDesc), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(f->heap_leaf, ident.data(), ident.size() * 4, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(f->d_jobs, jobs.data(), jobs.size() * sizeof(TileJob), hipMemcpyHostToDevice, s);
    f->final_buf = 0;
    {
        ProfScope ps(s, "leaf_finalize", (double)TN * (4.0 * d + 16), 0);
        uniform_leaf_pass(f, s);
    }
    if ((st = check_hip(hipStreamSynchronize(s), "rpf_build uniform leaves")) != RPF_OK) return bail(st);
    const std::string le = take_launch_error();
    if (!le.empty()) {
        fail(RPF_EDEVICE, "rpf_build: " + le);
        return bail(RPF_EDEVICE);
    }
#undef RPF_UTEMP
#undef RPF_UALLOC
    *out = f;
    return RPF_OK;
}

extern "C" {

rpf_status rpf_build(const float *X, int64_t n, int32_t d, const rpf_params *p, void *stream, rpf_forest **out) {
    if (p && p->split_rule == RPF_SPLIT_UNIFORM) return build_uniform(X, n, d, p, stream, out);
    return build_impl(X, &n, 1, d, p, stream, out);
}

rpf_status rpf_build_batched(const float *X, const int64_t *n_host, int32_t count, int32_t d, const rpf_params *p,
                             void *stream, rpf_forest **out) {
    if (out) *out = nullptr;
    if (!n_host || count < 1) return fail(RPF_EINVAL, "rpf_build_batched: need count >= 1 sizes");
    return build_impl(X, n_host, count, d, p, stream, out);
}

}  // extern "C"

// A build and all-points search of fixed shapes recorded once as a HIP graph.  The data
// sets are grouped by dimension and each group is cut into parts of bounded size (data sets
// are never split); every part is one forest over its data sets.  One graph launch runs,
// part after part, the input checks, every level of every tree, the leaf pass, the
// candidate stage (one workspace shared by all parts) and the index localisation.
struct PlanPart {
    rpf_forest *f = nullptr;
    std::vector<int> sets;     // data set indices, in order
    int32_t *out_idx = nullptr;
    float *out_dist = nullptr;
    int B = 0;                 // first-phase trees (0: default rule; set by the tuner)
    int shape = 0;             // Phase II symmetric tile shape (set by the tuner)
    int S = 0;                 // Phase II bucket size (0: default rule; set by the tuner)
};

struct rpf_plan {
    std::vector<PlanPart> parts;
    std::vector<rpf_plan_entry> entries;
    KnnShared *knn = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int K = 0, excl = 0, count = 0;
};

constexpr int kTuneB[] = {2, 3, 4, 6, 8};  // first-phase tree counts the tuner tries

// The tuner's choices, per part shape: kept for the process, written to and read from a
// file (rpf_tune_save / rpf_tune_load), and applied by rpf_plan_create to every part whose
// shape has an entry.  A part's shape: d, largest leaf, tile precision, K, T and
// floor(log2 n).
struct TuneKey {
    int d, max_leaf, prec, K, T, nlog2;
    bool operator<(const TuneKey &o) const {
        return std::tie(d, max_leaf, prec, K, T, nlog2) < std::tie(o.d, o.max_leaf, o.prec, o.K, o.T, o.nlog2);
    }
};
struct TuneVal {
    int B, shape, S, subtree;
};
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneVal> g_tune;

static TuneKey tune_key(const rpf_forest *f, int K) {
    int lg = 0;
    while (((int64_t)2 << lg) <= f->n) lg++;
    return TuneKey{f->d, f->max_leaf, f->tile_prec, K, f->T, lg};
}

static void plan_free(rpf_plan *pl) {
    if (!pl) return;
    hipDeviceSynchronize();
    if (pl->exec) hipGraphExecDestroy(pl->exec);
    if (pl->graph) hipGraphDestroy(pl->graph);
    if (pl->cap) hipStreamDestroy(pl->cap);
    knn_shared_destroy(pl->knn, nullptr);
    for (auto &pt : pl->parts) {
        cache_free(pt.out_idx, nullptr);
        cache_free(pt.out_dist, nullptr);
        if (pt.f) {
            free_forest_memory(pt.f);
            delete pt.f;
        }
    }
    delete pl;
}

static rpf_status plan_record(rpf_plan *pl) {
    if (pl->exec) hipGraphExecDestroy(pl->exec);
    if (pl->graph) hipGraphDestroy(pl->graph);
    pl->exec = nullptr;
    pl->graph = nullptr;
    take_launch_error();
    hipStream_t c = pl->cap;
    rpf_status st = check_hip(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal), "begin capture");
    if (st != RPF_OK) return st;
    for (auto &pt : pl->parts) {
        rpf_forest *f = pt.f;
        fill_u32(f->err, 16, 0, c);
        launch_nonfinite(c, f->X, f->n * f->d, f->err + 2);
        launch_nonfinite(c, f->R, (int64_t)f->T * f->H * f->n_try * f->d, f->err + 3);
        if (f->Xq) launch_grid_quantise(c, f->X, f->n, f->d, f->dq, f->Xq, f->qn, f->err + 4);
        build_launches(f, c);
        knn_part_launch(pl->knn, f, pt.B, pt.shape, pt.S, pt.out_idx, pt.out_dist, c);
        if (pt.sets.size() > 1) launch_localize(pt.out_idx, f->n, pl->K, f->d_batch_off, (int)pt.sets.size(), c);
    }
    const hipError_t ec = hipStreamEndCapture(c, &pl->graph);
    const std::string le = take_launch_error();
    if (ec != hipSuccess || !le.empty() || !pl->graph)
        return fail(RPF_EDEVICE, "rpf_plan: recording failed: " + (le.empty() ? std::string(hipGetErrorString(ec)) : le));
    return check_hip(hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0), "graph instantiate");
}

extern "C" {

rpf_status rpf_plan_create(const int64_t *n_host, const int32_t *d_host, int32_t count, const rpf_params *p, int32_t K,
                           int32_t exclude_self, int64_t max_part_points, void *stream, rpf_plan **out) {
    if (out) *out = nullptr;
    if (!out || !n_host || !d_host || !p || count < 1)
        return fail(RPF_EINVAL, "rpf_plan_create: NULL pointer or count < 1");
    if (exclude_self != 0 && exclude_self != 1) return fail(RPF_EINVAL, "rpf_plan_create: exclude_self must be 0 or 1");
    if (K < 1 || K > 256) return fail(RPF_EINVAL, "rpf_plan_create: K must be in [1, 256]");
    for (int i = 0; i < count; i++)
        if (n_host[i] < 1 || d_host[i] < 1) return fail(RPF_EINVAL, "rpf_plan_create: every data set needs n, d >= 1");
    if (max_part_points <= 0) max_part_points = (int64_t)4 << 20;
    hipStream_t s = (hipStream_t)stream;
    rpf_plan *pl = new rpf_plan();
    pl->K = K;
    pl->excl = exclude_self;
    pl->count = count;
    // group by d (first appearance), then cut each group into parts of <= max_part_points
    std::vector<int32_t> dims;
    for (int i = 0; i < count; i++)
        if (std::find(dims.begin(), dims.end(), d_host[i]) == dims.end()) dims.push_back(d_host[i]);
    for (int32_t d : dims) {
        PlanPart cur;
        int64_t pts = 0;
        for (int i = 0; i < count; i++) {
            if (d_host[i] != d) continue;
            if (!cur.sets.empty() && pts + n_host[i] > max_part_points) {
                pl->parts.push_back(cur);
                cur = PlanPart();
                pts = 0;
            }
            cur.sets.push_back(i);
            pts += n_host[i];
        }
        if (!cur.sets.empty()) pl->parts.push_back(cur);
    }
    pl->entries.resize(count);
    std::vector<const rpf_forest *> fs;
    std::vector<int> maxB;
    for (size_t k = 0; k < pl->parts.size(); k++) {
        PlanPart &pt = pl->parts[k];
        std::vector<int64_t> sizes;
        for (int i : pt.sets) sizes.push_back(n_host[i]);
        const int32_t d = d_host[pt.sets[0]];
        rpf_status st = prepare_forest(sizes.data(), (int)sizes.size(), d, p, stream, &pt.f, false);
        if (st != RPF_OK) {
            plan_free(pl);
            return st;
        }
        if (K > pt.f->n - exclude_self) {
            plan_free(pl);
            return fail(RPF_EINVAL, "rpf_plan_create: K must be <= n - exclude_self of every part");
        }
        pt.out_idx = static_cast<int32_t *>(cache_alloc((size_t)pt.f->n * K * 4, s));
        pt.out_dist = static_cast<float *>(cache_alloc((size_t)pt.f->n * K * 4, s));
        if (!pt.out_idx || !pt.out_dist) {
            plan_free(pl);
            return fail(RPF_ENOMEM, "rpf_plan_create: device allocation failed");
        }
        for (size_t j = 0; j < pt.sets.size(); j++) {
            const rpf_batch_entry &e = pt.f->batch[j];
            rpf_plan_entry &pe = pl->entries[pt.sets[j]];
            pe.part = (int32_t)k;
            pe.index_in_part = (int32_t)j;
            pe.d = d;
            pe.reserved = 0;
            pe.n = e.n;
            pe.row = e.offset;
            pe.heap_base = e.heap_base;
            pe.n_nodes = ((int64_t)1 << e.depth) - 1;
        }
        {  // the tuner's earlier choices for a part of this shape, if any
            std::lock_guard<std::mutex> lk(g_tune_mu);
            const auto it = g_tune.find(tune_key(pt.f, K));
            if (it != g_tune.end()) {
                pt.B = it->second.B;
                pt.shape = it->second.shape & knn_part_shape_mask(pt.f, K);
                pt.S = it->second.S;
                pt.f->subtree_on = it->second.subtree && pt.f->sub_level >= 0;
            }
        }
        fs.push_back(pt.f);
        maxB.push_back(knn_part_first_trees(pt.f, K, kTuneB[sizeof(kTuneB) / sizeof(kTuneB[0]) - 1]));
    }
    pl->knn = knn_shared_create(fs, maxB, K, exclude_self, s);
    if (!pl->knn) {
        plan_free(pl);
        return fail(RPF_ENOMEM, "rpf_plan_create: kNN workspace allocation failed");
    }
    rpf_status st;
    if ((st = check_hip(hipStreamSynchronize(s), "rpf_plan_create")) != RPF_OK ||
        (st = check_hip(hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking), "rpf_plan_create stream")) != RPF_OK ||
        (st = plan_record(pl)) != RPF_OK) {
        plan_free(pl);
        return st;
    }
    *out = pl;
    return RPF_OK;
}

rpf_status rpf_plan_info(const rpf_plan *pl, int32_t *n_parts, int32_t *count) {
    if (!pl) return fail(RPF_EINVAL, "rpf_plan_info: NULL plan");
    if (n_parts) *n_parts = (int32_t)pl->parts.size();
    if (count) *count = pl->count;
    return RPF_OK;
}

rpf_status rpf_plan_part(const rpf_plan *pl, int32_t k, rpf_plan_part_info *out) {
    if (!pl || !out) return fail(RPF_EINVAL, "rpf_plan_part: NULL pointer");
    if (k < 0 || k >= (int32_t)pl->parts.size()) return fail(RPF_EINVAL, "rpf_plan_part: part out of range");
    const PlanPart &pt = pl->parts[k];
    out->rows = pt.f->n;
    out->d = pt.f->d;
    out->n_sets = (int32_t)pt.sets.size();
    out->n_nodes = pt.f->H;
    out->X_dev = pt.f->X;
    out->directions_dev = pt.f->R;
    out->out_idx_dev = pt.out_idx;
    out->out_dist_dev = pt.out_dist;
    out->forest = pt.f;
    out->first_trees = knn_part_first_trees(pt.f, pl->K, pt.B);
    out->tile_shape = pt.shape;
    out->bucket_size = pt.S ? pt.S : knn_part_bucket_size(pt.f, pl->K, out->first_trees);
    out->subtrees = pt.f->subtree_on ? 1 : 0;
    return RPF_OK;
}

rpf_status rpf_plan_entry_of(const rpf_plan *pl, int32_t i, rpf_plan_entry *out) {
    if (!pl || !out) return fail(RPF_EINVAL, "rpf_plan_entry_of: NULL pointer");
    if (i < 0 || i >= pl->count) return fail(RPF_EINVAL, "rpf_plan_entry_of: data set out of range");
    *out = pl->entries[i];
    return RPF_OK;
}

rpf_status rpf_plan_launch(rpf_plan *pl, void *stream) {
    if (!pl) return fail(RPF_EINVAL, "rpf_plan_launch: NULL plan");
    return check_hip(hipGraphLaunch(pl->exec, (hipStream_t)stream), "rpf_plan_launch");
}

rpf_status rpf_plan_check(rpf_plan *pl, void *stream) {
    if (!pl) return fail(RPF_EINVAL, "rpf_plan_check: NULL plan");
    std::vector<int32_t> flags(5 * pl->parts.size(), 0);
    for (size_t k = 0; k < pl->parts.size(); k++)
        hipMemcpyAsync(&flags[5 * k], pl->parts[k].f->err, 20, hipMemcpyDeviceToHost, (hipStream_t)stream);
    const rpf_status st = check_hip(hipStreamSynchronize((hipStream_t)stream), "rpf_plan_check");
    if (st != RPF_OK) return st;
    for (size_t k = 0; k < pl->parts.size(); k++) {
        if (flags[5 * k + 2]) return fail(RPF_EINVAL, "rpf_plan_check: X holds NaN or Inf (part " + std::to_string(k) + ")");
        if (flags[5 * k + 3])
            return fail(RPF_EINVAL, "rpf_plan_check: directions hold NaN or Inf (part " + std::to_string(k) + ")");
        if (flags[5 * k + 4])
            return fail(RPF_EINVAL, "rpf_plan_check: X is off the 1/255 grid (part " + std::to_string(k) + ")");
        if (flags[5 * k]) return fail(RPF_EINTERNAL, "rpf_plan_check: build kernels flagged error " + std::to_string(flags[5 * k]));
        if (const uint64_t flt = forest_fault_read(pl->parts[k].f, (hipStream_t)stream))
            return fail(RPF_EINTERNAL, "rpf_plan_check: " + std::to_string(flt) + " rows of part " + std::to_string(k) +
                                           " met a candidate index outside the data set");
    }
    return RPF_OK;
}

rpf_status rpf_plan_tune(rpf_plan *pl, void *stream, double *tuned_ms) {
    if (!pl) return fail(RPF_EINVAL, "rpf_plan_tune: NULL plan");
    hipStream_t s = (hipStream_t)stream;
    rpf_status st = rpf_plan_launch(pl, stream);  // forests built from the current inputs
    if (st != RPF_OK || (st = rpf_plan_check(pl, stream)) != RPF_OK) return st;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    // the best of two timed runs after one warm-up run
    auto timed = [&](auto &&run) {
        double ms = 1e300;
        for (int rep = 0; rep < 3; rep++) {
            hipEventRecord(e0, s);
            run();
            hipEventRecord(e1, s);
            hipEventSynchronize(e1);
            float t = 0;
            hipEventElapsedTime(&t, e0, e1);
            if (rep) ms = std::min(ms, (double)t);
        }
        return ms;
    };
    double total = 0;
    for (auto &pt : pl->parts) {
        auto cand = [&](int B, int shape, int S) {
            return timed([&] { knn_part_launch(pl->knn, pt.f, B, shape, S, pt.out_idx, pt.out_dist, s); });
        };
        // 1. first-phase trees, default tile shape and bucket size
        double best = 1e300;
        int bestB = pt.B;
        std::vector<int> tried;
        for (int b : kTuneB) {
            const int B = knn_part_first_trees(pt.f, pl->K, b);
            if (std::find(tried.begin(), tried.end(), B) != tried.end()) continue;
            tried.push_back(B);
            const double ms = cand(B, 0, 0);
            if (ms < best) {
                best = ms;
                bestB = B;
            }
        }
        // 2. Phase II tile shape: k-chunk, queue length, waves per block
        const int mask = knn_part_shape_mask(pt.f, pl->K);
        int bestShape = 0;
        for (int sh = 1; sh <= mask; sh++) {
            if ((sh & mask) != sh) continue;
            const double ms = cand(bestB, sh, 0);
            if (ms < best) {
                best = ms;
                bestShape = sh;
            }
        }
        // 3. Phase II bucket size: the default rule's, or half of it
        int bestS = 0;
        const int S0 = knn_part_bucket_size(pt.f, pl->K, bestB);
        if (S0 >= 8) {
            const double ms = cand(bestB, bestShape, S0 / 2);
            if (ms < best) {
                best = ms;
                bestS = S0 / 2;
            }
        }
        pt.B = bestB;
        pt.shape = bestShape;
        pt.S = bestS;
        // 4. build schedule: level by level, or the small levels in one persistent launch
        if (pt.f->sub_level >= 0) {
            double ms_sched[2];
            for (int on = 0; on < 2; on++) {
                pt.f->subtree_on = on != 0;
                ms_sched[on] = timed([&] { build_launches(pt.f, s); });
            }
            pt.f->subtree_on = ms_sched[1] < ms_sched[0];
            best += std::min(ms_sched[0], ms_sched[1]);
        }
        total += best;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(pt.f, pl->K)] = TuneVal{pt.B, pt.shape, pt.S, pt.f->subtree_on ? 1 : 0};
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    const std::string le = take_launch_error();
    if (!le.empty()) return fail(RPF_EDEVICE, "rpf_plan_tune: " + le);
    if (tuned_ms) *tuned_ms = total;
    return plan_record(pl);  // the outputs are recomputed by the next launch
}

rpf_status rpf_tune_save(const char *path) {
    if (!path) return fail(RPF_EINVAL, "rpf_tune_save: NULL path");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *fp = fopen(path, "w");
    if (!fp) return fail(RPF_EINVAL, std::string("rpf_tune_save: cannot open ") + path);
    for (const auto &kv : g_tune) {
        const TuneKey &k = kv.first;
        const TuneVal &v = kv.second;
        fprintf(fp,
                "{\"d\": %d, \"max_leaf\": %d, \"prec\": %d, \"K\": %d, \"T\": %d, \"n_log2\": %d, "
                "\"first_trees\": %d, \"tile_shape\": %d, \"bucket_size\": %d, \"subtrees\": %d}\n",
                k.d, k.max_leaf, k.prec, k.K, k.T, k.nlog2, v.B, v.shape, v.S, v.subtree);
    }
    const bool ok = fclose(fp) == 0;
    return ok ? RPF_OK : fail(RPF_EINVAL, std::string("rpf_tune_save: write failed: ") + path);
}

rpf_status rpf_tune_load(const char *path, int32_t *entries) {
    if (!path) return fail(RPF_EINVAL, "rpf_tune_load: NULL path");
    FILE *fp = fopen(path, "r");
    if (!fp) return fail(RPF_EINVAL, std::string("rpf_tune_load: cannot open ") + path);
    std::map<TuneKey, TuneVal> got;
    char line[512];
    int lineno = 0;
    bool bad = false;
    while (fgets(line, sizeof line, fp)) {
        lineno++;
        bool blank = true;
        for (const char *c = line; *c; c++) blank &= (*c == ' ' || *c == '\t' || *c == '\n' || *c == '\r');
        if (blank) continue;
        TuneKey k;
        TuneVal v;
        int used = 0;
        const int got_n = sscanf(line,
                                 " {\"d\": %d, \"max_leaf\": %d, \"prec\": %d, \"K\": %d, \"T\": %d, \"n_log2\": %d, "
                                 "\"first_trees\": %d, \"tile_shape\": %d, \"bucket_size\": %d, \"subtrees\": %d}%n",
                                 &k.d, &k.max_leaf, &k.prec, &k.K, &k.T, &k.nlog2, &v.B, &v.shape, &v.S, &v.subtree,
                                 &used);
        if (got_n != 10 || used == 0 || v.B < 0 || v.shape < 0 || v.shape > 7 || v.S < 0 || v.S > 64 ||
            (v.subtree != 0 && v.subtree != 1)) {
            bad = true;
            break;
        }
        got[k] = v;
    }
    fclose(fp);
    if (bad) return fail(RPF_EINVAL, "rpf_tune_load: malformed entry on line " + std::to_string(lineno));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : got) g_tune[kv.first] = kv.second;
    if (entries) *entries = (int32_t)g_tune.size();
    return RPF_OK;
}

rpf_status rpf_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return RPF_OK;
}

rpf_status rpf_plan_destroy(rpf_plan *pl) {
    plan_free(pl);
    return RPF_OK;
}

}  // extern "C"

namespace rpf {
rpf_status fault_error(const rpf_forest *f, const char *who) {
    return fail(RPF_EINTERNAL, std::string(who) + ": " + std::to_string(forest_fault_seen(f)) +
                                   " rows of an earlier search on this forest met a candidate index outside the "
                                   "data set (recomputed exhaustively; an internal error)");
}

// end of a search call: the fault counter's host mirror is refreshed behind the call's work;
// when every launch is synchronised (RPF_SYNC_CHECK=1) the call itself reports a fault
rpf_status search_tail(const rpf_forest *f, hipStream_t s, const char *who) {
    forest_fault_mirror(f, s);
    if (!sync_check_on()) return RPF_OK;
    const rpf_status st = check_hip(hipStreamSynchronize(s), who);
    if (st != RPF_OK) return st;
    return forest_fault_seen(f) ? fault_error(f, who) : RPF_OK;
}
}  // namespace rpf

extern "C" {

rpf_status rpf_batch_info(const rpf_forest *f, int32_t i, rpf_batch_entry *out) {
    if (!f || !out) return fail(RPF_EINVAL, "rpf_batch_info: NULL pointer");
    if (i < 0 || i >= (int32_t)f->batch.size()) return fail(RPF_EINVAL, "rpf_batch_info: data set out of range");
    *out = f->batch[i];
    return RPF_OK;
}

rpf_status rpf_all_knn(const rpf_forest *f, int32_t K, int32_t exclude_self, int32_t *out_idx, float *out_dist,
                       void *stream) {
    if (!f) return fail(RPF_EINVAL, "rpf_all_knn: forest is NULL");
    if (!out_idx || !out_dist) return fail(RPF_EINVAL, "rpf_all_knn: output is NULL");
    if (exclude_self != 0 && exclude_self != 1) return fail(RPF_EINVAL, "rpf_all_knn: exclude_self must be 0 or 1");
    if (K < 1 || K > f->n - exclude_self) return fail(RPF_EINVAL, "rpf_all_knn: K must be in [1, n - exclude_self]");
    if (K > 256) return fail(RPF_EINVAL, "rpf_all_knn: K above 256 is not supported");
    if (forest_fault_seen(f)) return fault_error(f, "rpf_all_knn");
    hipStream_t s = (hipStream_t)stream;
    rpf_status st = knn_all(f, K, exclude_self, out_idx, out_dist, s);
    if (st != RPF_OK) return st;
    if (f->batch.size() >= 2) {
        launch_localize(out_idx, f->n, K, f->d_batch_off, (int)f->batch.size(), s);
        const std::string le = take_launch_error();
        if (!le.empty()) return fail(RPF_EDEVICE, "rpf_all_knn: " + le);
    }
    return search_tail(f, s, "rpf_all_knn");
}

rpf_status rpf_query(const rpf_forest *f, const float *Q, int64_t m, int32_t K, int32_t *out_idx, float *out_dist,
                     void *stream) {
    if (!f) return fail(RPF_EINVAL, "rpf_query: forest is NULL");
    if (m < 0) return fail(RPF_EINVAL, "rpf_query: m must be >= 0");
    if (m == 0) return RPF_OK;
    if (!Q || !out_idx || !out_dist) return fail(RPF_EINVAL, "rpf_query: NULL pointer");
    if (K < 1 || K > f->n) return fail(RPF_EINVAL, "rpf_query: K must be in [1, n]");
    if (K > 256) return fail(RPF_EINVAL, "rpf_query: K above 256 is not supported");
    if (f->batch.size() > 1) return fail(RPF_EINVAL, "rpf_query: the forest holds several data sets");
    if (f->split_rule == RPF_SPLIT_UNIFORM) return fail(RPF_EINVAL, "rpf_query: queries need a median-rule forest");
    if (forest_fault_seen(f)) return fault_error(f, "rpf_query");
    const rpf_status st = knn_query(f, Q, m, K, out_idx, out_dist, (hipStream_t)stream);
    return st != RPF_OK ? st : search_tail(f, (hipStream_t)stream, "rpf_query");
}

rpf_status rpf_query_workspace_bytes(const rpf_forest *f, int64_t m, int32_t K, uint64_t *bytes) {
    if (!f || !bytes) return fail(RPF_EINVAL, "rpf_query_workspace_bytes: NULL pointer");
    if (m < 0 || K < 1 || K > 256) return fail(RPF_EINVAL, "rpf_query_workspace_bytes: m >= 0 and 1 <= K <= 256");
    *bytes = m == 0 ? 0 : query_workspace_bytes(f, m, K);
    return RPF_OK;
}

rpf_status rpf_route(const rpf_forest *f, const float *Q, int64_t m, int32_t *out_leaf, void *stream) {
    if (!f) return fail(RPF_EINVAL, "rpf_route: forest is NULL");
    if (f->batch.size() > 1) return fail(RPF_EINVAL, "rpf_route: the forest holds several data sets");
    if (f->split_rule == RPF_SPLIT_UNIFORM) return fail(RPF_EINVAL, "rpf_route: routing needs a median-rule forest");
    if (m < 0) return fail(RPF_EINVAL, "rpf_route: m must be >= 0");
    if (m == 0) return RPF_OK;
    if (!Q || !out_leaf) return fail(RPF_EINVAL, "rpf_route: NULL pointer");
    return route(f, Q, m, out_leaf, (hipStream_t)stream);
}

rpf_status rpf_tree_dump(const rpf_forest *f, int32_t tree, double *split, int32_t *split_idx, int32_t *chosen,
                         int32_t *perm, int32_t *leaf_of, void *stream) {
    if (!f) return fail(RPF_EINVAL, "rpf_tree_dump: forest is NULL");
    if (tree < 0 || tree >= f->T) return fail(RPF_EINVAL, "rpf_tree_dump: tree out of range");
    if (f->split_rule == RPF_SPLIT_UNIFORM && (split || split_idx || chosen))
        return fail(RPF_EINVAL, "rpf_tree_dump: a uniform-rule forest has no split arrays (rpf_tree_nodes lists its nodes)");
    hipStream_t s = (hipStream_t)stream;
    const int64_t H = f->H, n = f->n;
    if (split && H) hipMemcpyAsync(split, f->split + tree * H, H * 8, hipMemcpyDeviceToDevice, s);
    if (split_idx && H) hipMemcpyAsync(split_idx, f->split_idx + tree * H, H * 4, hipMemcpyDeviceToDevice, s);
    if (chosen && H) hipMemcpyAsync(chosen, f->chosen + tree * H, H * 4, hipMemcpyDeviceToDevice, s);
    if (perm) hipMemcpyAsync(perm, f->perm[f->final_buf] + tree * n, n * 4, hipMemcpyDeviceToDevice, s);
    if (leaf_of) hipMemcpyAsync(leaf_of, f->leaf_of + tree * n, n * 4, hipMemcpyDeviceToDevice, s);
    return check_hip(hipGetLastError(), "rpf_tree_dump");
}

rpf_status rpf_tree_nodes(const rpf_forest *f, int32_t tree, rpf_node *out, int64_t cap, int64_t *count) {
    if (!f || !count) return fail(RPF_EINVAL, "rpf_tree_nodes: NULL pointer");
    if (f->split_rule != RPF_SPLIT_UNIFORM) return fail(RPF_EINVAL, "rpf_tree_nodes: not a uniform-rule forest");
    if (tree < 0 || tree >= f->T) return fail(RPF_EINVAL, "rpf_tree_nodes: tree out of range");
    if (cap < 0 || (cap > 0 && !out)) return fail(RPF_EINVAL, "rpf_tree_nodes: bad output capacity");
    const std::vector<rpf_node> &v = f->nodes[tree];
    const int64_t k = std::min<int64_t>(cap, (int64_t)v.size());
    if (k > 0) std::copy(v.begin(), v.begin() + k, out);
    *count = (int64_t)v.size();
    return RPF_OK;
}

rpf_status rpf_forest_info(const rpf_forest *f, rpf_info *out) {
    if (!f || !out) return fail(RPF_EINVAL, "rpf_forest_info: NULL pointer");
    out->n = f->n;
    out->d = f->d;
    out->n_trees = f->T;
    out->leaf_size = f->n0;
    out->n_try = f->n_try;
    out->depth = f->L;
    out->dist_prec = f->tile_prec;
    out->n_leaves = f->split_rule == RPF_SPLIT_UNIFORM ? f->leaf_stride : (int64_t)f->leaves.size();
    out->device_bytes = f->bytes;
    out->batch_count = (int32_t)f->batch.size();
    out->split_rule = f->split_rule;
    int32_t err = 0;
    hipDeviceSynchronize();
    hipMemcpy(&err, f->err, 4, hipMemcpyDeviceToHost);
    if (err) return fail(RPF_EINTERNAL, "rpf_forest_info: build kernels flagged error " + std::to_string(err));
    unsigned long long flt = 0;
    hipMemcpy(&flt, f->fault, sizeof(flt), hipMemcpyDeviceToHost);
    if (flt)
        return fail(RPF_EINTERNAL, "rpf_forest_info: " + std::to_string(flt) +
                                       " rows of a search met a candidate index outside the data set");
    return RPF_OK;
}

rpf_status rpf_last_knn_stats(const rpf_forest *f, rpf_knn_stats *out, void *stream) {
    if (!f || !out) return fail(RPF_EINVAL, "rpf_last_knn_stats: NULL pointer");
    unsigned long long slots[kStatSlots * 8], v[8] = {};
    hipMemcpyAsync(slots, f->stats, sizeof(slots), hipMemcpyDeviceToHost, (hipStream_t)stream);
    rpf_status st = check_hip(hipStreamSynchronize((hipStream_t)stream), "rpf_last_knn_stats");
    if (st != RPF_OK) return st;
    for (int k = 0; k < kStatSlots; k++)
        for (int i = 0; i < 8; i++) v[i] += slots[k * 8 + i];
    if (v[4] != 0)
        return fail(RPF_EINTERNAL, "rpf_last_knn_stats: " + std::to_string(v[4]) +
                                       " rows met a candidate index outside the data set (recomputed exhaustively)");
    if (const uint64_t flt = forest_fault_read(f, (hipStream_t)stream))
        return fail(RPF_EINTERNAL, "rpf_last_knn_stats: " + std::to_string(flt) +
                                       " rows of an earlier search met a candidate index outside the data set");
    out->rows = (int64_t)v[0] + (int64_t)v[1];
    out->fallback_rows = (int64_t)v[1];
    out->reranked32 = (int64_t)v[2];
    out->reranked64 = (int64_t)v[3];
    out->first_phase_kept = (int64_t)v[5];
    out->second_phase_emitted = (int64_t)v[6];
    out->block_merged_rows = (int64_t)v[7];
    return RPF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- read-only view for the kNN launchers
namespace rpf {
int64_t forest_points(const rpf_forest *f) { return f->n; }
int32_t forest_dim(const rpf_forest *f) { return f->d; }
int32_t forest_batch_count(const rpf_forest *f) { return (int32_t)f->batch.size(); }

ForestView view(const rpf_forest *f) {
    ForestView v;
    v.n = f->n; v.H = f->H; v.d = f->d; v.T = f->T; v.n0 = f->n0; v.n_try = f->n_try; v.L = f->L;
    v.prec = f->prec; v.dp = f->dp; v.max_leaf = f->max_leaf; v.job_mb = f->job_mb;
    v.sym_prec = f->tile_prec;
    v.Xq = f->Xq; v.qn = f->qn; v.dq = f->dq;
    v.X = f->X; v.R = f->R; v.centroid = f->centroid; v.split = f->split; v.chosen = f->chosen;
    v.perm = f->perm[f->final_buf]; v.leaf_of = f->leaf_of; v.heap_leaf = f->heap_leaf; v.Xc = f->Xc;
    v.nrm = f->nrm; v.leaves = f->d_leaves; v.jobs = f->d_jobs;
    v.nleaf = f->leaf_stride ? f->leaf_stride : (int64_t)f->leaves.size();
    v.n_jobs_tree = f->n_jobs_tree; v.tile_flops_tree = f->tile_flops_tree; v.stats = f->stats;
    v.fault = f->fault;
    v.leaf_stride = f->leaf_stride;
    v.job_off = f->job_off.empty() ? nullptr : f->job_off.data();
    v.flops_off = f->flops_off.empty() ? nullptr : f->flops_off.data();
    return v;
}

bool forest_uniform(const rpf_forest *f) { return f->split_rule == RPF_SPLIT_UNIFORM; }

uint64_t forest_fault_seen(const rpf_forest *f) {
    return f->pin_slot < 0 ? 0 : __atomic_load_n(&g_pin[f->pin_slot], __ATOMIC_RELAXED);
}

void forest_fault_mirror(const rpf_forest *f, hipStream_t s) {
    if (f->pin_slot >= 0)
        hipMemcpyAsync(&g_pin[f->pin_slot], f->fault, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
}

// the device counter read after a synchronisation of s (a failed read counts as no fault:
// the failure itself surfaces as a device error)
uint64_t forest_fault_read(const rpf_forest *f, hipStream_t s) {
    unsigned long long v = 0;
    if (hipMemcpyAsync(&v, f->fault, sizeof(v), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return 0;
    return v;
}
}  // namespace rpf
