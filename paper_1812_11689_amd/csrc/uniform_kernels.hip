// Tree growth by the uniform split rule that Alg. 1 prints: at a node W the split point c is
// drawn uniformly between a = min and b = max of the members' projections onto the node's
// direction (Alg. 2 picks that direction among nTry random ones), W_L = {p < c} and
// W_R = {p >= c}.  The shape of a tree now depends on the data, so growth is
// level-synchronous over a frontier the host keeps: one level splits every open node of
// every tree in a handful of launches, and the host reads back the left sizes to open the
// next level.
//
// Random numbers.  A node's draws cannot be laid out in advance as the median rule's
// direction array is, so they come from a counter-based generator keyed by (seed, tree, heap
// id of the node): SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014), whose stream with seed s has the outputs
// out(s, i) = mix64(s + (i + 1) GAMMA).  The node's stream has the seed out(out(seed, t), h);
// its draw 0 gives the split fraction u = (draw >> 11) 2^-53 in [0, 1), and coordinate j of
// direction try i is (sum of the 32-bit halves of draws 1 + 6 (i d + j) + q, q < 6) 2^-32 - 6,
// exact in binary64 and rounded once to binary32 (Irwin-Hall: mean 0, variance 1).
// c = RN(a + RN(u RN(b - a))).  A node with an empty child stays whole, as a leaf; nodes at
// depth kUniformDepth are not split (heap ids stay below 2^63).
//
// Two paths per level, both writing the node's permutation range in place (stable: both
// children keep ascending original index):
//   - nodes of at most kChunk members: one block per node does the whole step in LDS
//     (k_uni_block);
//   - larger nodes: chunks of kChunk positions, aligned at the node's first position, with
//     projections stored in binary64 ([n_try][T n]), the canonical sums of Alg. 2 combined
//     from aligned power-of-two chunk partials (the same balanced tree as one canonical sum),
//     then a stable count / offsets / scatter partition through a scratch permutation.
#include "rpf_internal.h"

namespace rpf {

// ---------------------------------------------------------------- the generator

constexpr uint64_t kSmGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t sm64_at(uint64_t seed, uint64_t i) { return sm64_mix(seed + (i + 1) * kSmGamma); }

__host__ __device__ inline uint64_t uni_node_seed(uint64_t seed, int t, int64_t heap) {
    return sm64_at(sm64_at(seed, (uint64_t)t), (uint64_t)heap);
}

__device__ inline double uni_fraction(uint64_t key) { return (double)(sm64_at(key, 0) >> 11) * 0x1p-53; }

__device__ inline float uni_coord(uint64_t key, int tr, int d, int j) {
    const uint64_t base = 1 + 6 * ((uint64_t)tr * (uint64_t)d + (uint64_t)j);
    uint64_t s = 0;
#pragma unroll
    for (int q = 0; q < 6; q++) {
        const uint64_t w = sm64_at(key, base + q);
        s += (w >> 32) + (w & 0xffffffffull);
    }
    // (double)s is exact (s < 12 * 2^32), the scaling and the shift by 6 too
    return (float)__dsub_rn(__dmul_rn((double)s, 0x1p-32), 6.0);
}

__device__ inline double uni_split_point(double a, double b, double u) {
    return __dadd_rn(a, __dmul_rn(u, __dsub_rn(b, a)));
}

// ---------------------------------------------------------------- block helpers

// exclusive scan of one flag per thread over an NT-thread block (NT a multiple of 64);
// s_w needs NT / 64 words
template <int NT>
__device__ inline void block_flag_scan(bool f, uint32_t *s_w, uint32_t &excl, uint32_t &total) {
    const uint64_t b = __ballot(f);
    const uint32_t inw = (uint32_t)mask_rank(b);
    if (NT == 64) {
        excl = inw;
        total = (uint32_t)__popcll(b);
        return;
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s_w[w] = (uint32_t)__popcll(b);
    __syncthreads();
    uint32_t wb = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; k++) {
        const uint32_t c = s_w[k];
        if (k < w) wb += c;
        tot += c;
    }
    excl = wb + inw;
    total = tot;
    __syncthreads();
}

// min and max over the block (exact in any order); s_r needs 2 NT / 64 doubles
template <int NT>
__device__ inline void block_minmax(double &lo, double &hi, double *s_r) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, shfl_xor_d(lo, o));
        hi = fmax(hi, shfl_xor_d(hi, o));
    }
    if (NT == 64) return;
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_r[w] = lo;
        s_r[NT / 64 + w] = hi;
    }
    __syncthreads();
    lo = s_r[0];
    hi = s_r[NT / 64];
#pragma unroll
    for (int k = 1; k < NT / 64; k++) {
        lo = fmin(lo, s_r[k]);
        hi = fmax(hi, s_r[NT / 64 + k]);
    }
    __syncthreads();
}

template <int NT>
__device__ inline uint32_t block_count(uint32_t v, uint32_t *s_w) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (NT == 64) return v;
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s_w[w] = v;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; k++) t += s_w[k];
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------- nodes of at most kChunk members

size_t uni_block_lds(int max_m, int d, int n_try) {
    int P2 = 2;
    while (P2 < max_m) P2 <<= 1;
    const size_t ds = (size_t)((d + 3) & ~3);
    return (size_t)P2 * 8 * (n_try > 1 ? 3 : 1) + ds * 4 + (size_t)((max_m + 3) & ~3) * 4 + 256;
}

// LDS: p[P2] | (nTry > 1) work[P2], best[P2] | direction[ds] | ids[m] | reductions
template <int NT, bool VEC>
__global__ __launch_bounds__(NT) void k_uni_block(const float *__restrict__ X, int d, int n_try, uint64_t seed,
                                                  const UniSeg *__restrict__ segs, int32_t *__restrict__ perm,
                                                  UniSplit *__restrict__ out) {
    extern __shared__ __align__(16) uint8_t smem[];
    const UniSeg sg = segs[blockIdx.x];
    const int m = sg.size, tid = threadIdx.x;
    int P2 = 2;
    while (P2 < m) P2 <<= 1;
    const int ds = (d + 3) & ~3;
    double *s_p = reinterpret_cast<double *>(smem);
    double *s_work = s_p + P2;
    double *s_best = s_work + P2;
    float *s_dir = reinterpret_cast<float *>(n_try > 1 ? s_best + P2 : s_p + P2);
    int32_t *s_ids = reinterpret_cast<int32_t *>(s_dir + ds);
    double *s_red = reinterpret_cast<double *>(s_ids + ((m + 3) & ~3));
    uint32_t *s_w = reinterpret_cast<uint32_t *>(s_red + 2 * (NT / 64));

    int32_t *pg = perm + sg.pos;
    for (int i = tid; i < m; i += NT) s_ids[i] = pg[i];
    const uint64_t key = uni_node_seed(seed, sg.tree, sg.heap);
    const int g = tid & 7, pt = tid >> 3;
    double best = 0.0;
    int best_i = -1;
    for (int tr = 0; tr < n_try; tr++) {
        __syncthreads();  // the previous try is done with the direction
        for (int j = tid; j < ds; j += NT) s_dir[j] = j < d ? uni_coord(key, tr, d, j) : 0.f;
        __syncthreads();
        for (int base = 0; base < m; base += NT / 4) {  // rows base + pt and base + NT / 8 + pt
            const int ia = base + pt, ib = ia + NT / 8;
            double pa, pb;
            group8_dot64r2<VEC>(X + (int64_t)s_ids[ia < m ? ia : 0] * d, X + (int64_t)s_ids[ib < m ? ib : 0] * d,
                                s_dir, d, g, pa, pb);
            if (g == 0 && ia < m) s_p[ia] = pa;
            if (g == 0 && ib < m) s_p[ib] = pb;
        }
        __syncthreads();
        if (n_try == 1) break;
        // Alg. 2: keep the try with the largest spread S2 (the first wins ties; try 0 when no
        // try has any spread)
        for (int i = tid; i < m; i += NT) s_work[i] = s_p[i];
        const double mu = block_canon_sum(s_work, m) / (double)m;
        for (int i = tid; i < m; i += NT) {
            const double dev = __dsub_rn(s_p[i], mu);
            s_work[i] = __dmul_rn(dev, dev);
        }
        const double s2 = block_canon_sum(s_work, m);
        if (tr == 0 || s2 > best)
            for (int i = tid; i < m; i += NT) s_best[i] = s_p[i];
        if (s2 > best) {
            best = s2;
            best_i = tr;
        }
    }
    __syncthreads();
    const double *P = n_try > 1 ? s_best : s_p;
    double lo = INFINITY, hi = -INFINITY;
    for (int i = tid; i < m; i += NT) {
        lo = fmin(lo, P[i]);
        hi = fmax(hi, P[i]);
    }
    block_minmax<NT>(lo, hi, s_red);
    const double c = uni_split_point(lo, hi, uni_fraction(key));
    uint32_t nl = 0;
    for (int i = tid; i < m; i += NT) nl += P[i] < c ? 1u : 0u;
    nl = block_count<NT>(nl, s_w);
    uint32_t lefts = 0;
    for (int base = 0; base < m; base += NT) {
        const int i = base + tid;
        const bool valid = i < m;
        const bool left = valid && P[i] < c;
        uint32_t excl, total;
        block_flag_scan<NT>(left, s_w, excl, total);
        if (valid) {
            const uint32_t lb = lefts + excl;
            pg[left ? lb : nl + (uint32_t)i - lb] = s_ids[i];
        }
        lefts += total;
    }
    if (tid == 0) out[blockIdx.x] = UniSplit{c, (int32_t)nl, best_i < 0 ? 0 : best_i};
}

// ---------------------------------------------------------------- nodes above kChunk members

// projections of a chunk onto every try (stored), the chunk's min / max per try and, with
// more than one try, its partial canonical sum per try
template <bool VEC>
__global__ __launch_bounds__(256) void k_uni_proj(const float *__restrict__ X, int d, int n_try, uint64_t seed,
                                                  const UniSeg *__restrict__ segs,
                                                  const UniChunk *__restrict__ chunks,
                                                  const int32_t *__restrict__ perm, int64_t TN,
                                                  double *__restrict__ P, double *__restrict__ part,
                                                  double2 *__restrict__ mm) {
    __shared__ __align__(16) float s_dir[4096];
    __shared__ double s_red[8];
    extern __shared__ double s_p[];  // kChunk projections of the chunk, only for several tries
    const UniChunk c = chunks[blockIdx.x];
    const UniSeg sg = segs[c.seg];
    const int tid = threadIdx.x, g = tid & 7, pt = tid >> 3;
    const int ds = (d + 3) & ~3;
    const uint64_t key = uni_node_seed(seed, sg.tree, sg.heap);
    for (int tr = 0; tr < n_try; tr++) {
        __syncthreads();
        for (int j = tid; j < ds; j += 256) s_dir[j] = j < d ? uni_coord(key, tr, d, j) : 0.f;
        __syncthreads();
        double lo = INFINITY, hi = -INFINITY;
        for (int base = 0; base < c.len; base += 64) {  // rows base + pt and base + 32 + pt
            const int ia = base + pt, ib = ia + 32;
            const int32_t ida = perm[c.pos + (ia < c.len ? ia : 0)];
            const int32_t idb = perm[c.pos + (ib < c.len ? ib : 0)];
            double p2[2];
            group8_dot64r2<VEC>(X + (int64_t)ida * d, X + (int64_t)idb * d, s_dir, d, g, p2[0], p2[1]);
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int i = h ? ib : ia;
                const double p = p2[h];
                if (g == 0 && i < c.len) {
                    P[(int64_t)tr * TN + c.pos + i] = p;
                    if (n_try > 1) s_p[i] = p;
                    lo = fmin(lo, p);
                    hi = fmax(hi, p);
                }
            }
        }
        block_minmax<256>(lo, hi, s_red);
        if (tid == 0) mm[(int64_t)blockIdx.x * n_try + tr] = make_double2(lo, hi);
        if (n_try > 1) {
            const double sum = block_canon_sum(s_p, c.len);  // syncs before reading s_p
            if (tid == 0) part[(int64_t)blockIdx.x * n_try + tr] = sum;
        }
    }
}

// in-place balanced tree over the partials v[0], v[stride], ... of nc chunks: the canonical
// sum of the whole node (a missing right operand is the +0.0 padding)
__device__ inline double chunk_tree(double *v, int nc, int stride) {
    for (int h = 1; h < nc; h <<= 1)
        for (int i = 0; i + h < nc; i += 2 * h) v[(int64_t)i * stride] = v[(int64_t)i * stride] + v[(int64_t)(i + h) * stride];
    return v[0];
}

// per (node, try): the mean of the projections
__global__ void k_uni_mean(const UniSeg *__restrict__ segs, int nseg, int n_try, double *__restrict__ part,
                           double *__restrict__ mu) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)nseg * n_try) return;
    const int sgi = (int)(k / n_try), tr = (int)(k % n_try);
    const UniSeg sg = segs[sgi];
    const double s1 = chunk_tree(part + (int64_t)sg.chunk0 * n_try + tr, sg.nchunk, n_try);
    mu[k] = s1 / (double)sg.size;
}

// partial canonical sums of (p - mean)^2 per (chunk, try)
__global__ __launch_bounds__(256) void k_uni_disp(const UniSeg *__restrict__ segs, const UniChunk *__restrict__ chunks,
                                                  int n_try, int64_t TN, const double *__restrict__ P,
                                                  const double *__restrict__ mu, double *__restrict__ part) {
    __shared__ double s_v[kChunk];
    const UniChunk c = chunks[blockIdx.x];
    for (int tr = 0; tr < n_try; tr++) {
        const double m = mu[(int64_t)c.seg * n_try + tr];
        __syncthreads();
        for (int i = threadIdx.x; i < c.len; i += 256) {
            const double dev = __dsub_rn(P[(int64_t)tr * TN + c.pos + i], m);
            s_v[i] = __dmul_rn(dev, dev);
        }
        const double sum = block_canon_sum(s_v, c.len);
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * n_try + tr] = sum;
    }
}

// per node: the try (Alg. 2), a and b of its projections, and the split point
__global__ void k_uni_decide(const UniSeg *__restrict__ segs, int nseg, int n_try, uint64_t seed,
                             double *__restrict__ part, const double2 *__restrict__ mm, UniSplit *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nseg) return;
    const UniSeg sg = segs[k];
    int ch = 0;
    if (n_try > 1) {
        double best = 0.0;
        int best_i = -1;
        for (int tr = 0; tr < n_try; tr++) {
            const double s2 = chunk_tree(part + (int64_t)sg.chunk0 * n_try + tr, sg.nchunk, n_try);
            if (s2 > best) {
                best = s2;
                best_i = tr;
            }
        }
        ch = best_i < 0 ? 0 : best_i;
    }
    double lo = INFINITY, hi = -INFINITY;
    for (int q = 0; q < sg.nchunk; q++) {
        const double2 v = mm[(int64_t)(sg.chunk0 + q) * n_try + ch];
        lo = fmin(lo, v.x);
        hi = fmax(hi, v.y);
    }
    const uint64_t key = uni_node_seed(seed, sg.tree, sg.heap);
    out[k] = UniSplit{uni_split_point(lo, hi, uni_fraction(key)), 0, ch};
}

__global__ __launch_bounds__(256) void k_uni_count(const UniChunk *__restrict__ chunks, int64_t TN,
                                                   const double *__restrict__ P, const UniSplit *__restrict__ sp,
                                                   uint32_t *__restrict__ lcount) {
    __shared__ uint32_t s_w[4];
    const UniChunk c = chunks[blockIdx.x];
    const UniSplit q = sp[c.seg];
    const double *p = P + (int64_t)q.chosen * TN + c.pos;
    uint32_t v = 0;
    for (int i = threadIdx.x; i < c.len; i += 256) v += p[i] < q.c ? 1u : 0u;
    v = block_count<256>(v, s_w);
    if (threadIdx.x == 0) lcount[blockIdx.x] = v;
}

// per node: left positions before each chunk, and the node's left size
__global__ void k_uni_offsets(const UniSeg *__restrict__ segs, int nseg, const uint32_t *__restrict__ lcount,
                              uint32_t *__restrict__ loff, UniSplit *__restrict__ sp) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nseg) return;
    const UniSeg sg = segs[k];
    uint32_t run = 0;
    for (int q = 0; q < sg.nchunk; q++) {
        loff[sg.chunk0 + q] = run;
        run += lcount[sg.chunk0 + q];
    }
    sp[k].nl = (int32_t)run;
}

// stable partition of a chunk into the scratch permutation
__global__ __launch_bounds__(256) void k_uni_scatter(const UniSeg *__restrict__ segs,
                                                     const UniChunk *__restrict__ chunks, int64_t TN,
                                                     const double *__restrict__ P, const UniSplit *__restrict__ sp,
                                                     const uint32_t *__restrict__ loff, const int32_t *__restrict__ perm,
                                                     int32_t *__restrict__ tmp) {
    __shared__ uint32_t s_w[4];
    const UniChunk c = chunks[blockIdx.x];
    const UniSeg sg = segs[c.seg];
    const UniSplit q = sp[c.seg];
    const double *p = P + (int64_t)q.chosen * TN + c.pos;
    const int64_t within = c.pos - sg.pos;  // chunk's first position inside the node
    const uint32_t lo0 = loff[blockIdx.x];
    uint32_t lefts = 0;
    for (int base = 0; base < c.len; base += 256) {
        const int i = base + threadIdx.x;
        const bool valid = i < c.len;
        const bool left = valid && p[i] < q.c;
        uint32_t excl, total;
        block_flag_scan<256>(left, s_w, excl, total);
        if (valid) {
            const int64_t lb = (int64_t)lo0 + lefts + excl;  // lefts before this element in the node
            const int64_t dst = left ? lb : (int64_t)q.nl + within + i - lb;
            tmp[sg.pos + dst] = perm[c.pos + i];
        }
        lefts += total;
    }
}

__global__ __launch_bounds__(256) void k_uni_copy(const UniChunk *__restrict__ chunks, const int32_t *__restrict__ tmp,
                                                  int32_t *__restrict__ perm) {
    const UniChunk c = chunks[blockIdx.x];
    for (int i = threadIdx.x; i < c.len; i += 256) perm[c.pos + i] = tmp[c.pos + i];
}

// ---------------------------------------------------------------- launches of one level

void launch_uni_block(hipStream_t s, const float *X, int d, int n_try, uint64_t seed, const UniSeg *segs, int nseg,
                      int max_m, int32_t *perm, UniSplit *out) {
    if (nseg <= 0) return;
    const size_t lds = uni_block_lds(max_m, d, n_try);
    const bool vec = d % 4 == 0;
    auto go = [&](auto kern, int nt) {
        hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3((unsigned)nseg), dim3(nt), lds, s, X, d, n_try, seed, segs, perm, out);
    };
    if (max_m <= 128) {  // one wave per node
        if (vec) go(k_uni_block<64, true>, 64);
        else go(k_uni_block<64, false>, 64);
    } else {
        if (vec) go(k_uni_block<256, true>, 256);
        else go(k_uni_block<256, false>, 256);
    }
    launch_check(s, "k_uni_block");
}

void launch_uni_chunked(hipStream_t s, const float *X, int d, int n_try, uint64_t seed, const UniSeg *segs, int nseg,
                        const UniChunk *chunks, int nchunk, int32_t *perm, int64_t TN, const UniBufs &b,
                        UniSplit *out) {
    if (nseg <= 0) return;
    const bool vec = d % 4 == 0;
    if (vec)
        hipLaunchKernelGGL(k_uni_proj<true>, dim3(nchunk), dim3(256), n_try > 1 ? kChunk * sizeof(double) : 0, s, X,
                           d, n_try, seed, segs, chunks, perm, TN, b.P, b.part, b.mm);
    else
        hipLaunchKernelGGL(k_uni_proj<false>, dim3(nchunk), dim3(256), n_try > 1 ? kChunk * sizeof(double) : 0, s, X,
                           d, n_try, seed, segs, chunks, perm, TN, b.P, b.part, b.mm);
    launch_check(s, "k_uni_proj");
    if (n_try > 1) {
        const int64_t items = (int64_t)nseg * n_try;
        hipLaunchKernelGGL(k_uni_mean, dim3((unsigned)((items + 63) / 64)), dim3(64), 0, s, segs, nseg, n_try, b.part,
                           b.mu);
        hipLaunchKernelGGL(k_uni_disp, dim3(nchunk), dim3(256), 0, s, segs, chunks, n_try, TN, b.P, b.mu, b.part);
        launch_check(s, "k_uni_disp");
    }
    hipLaunchKernelGGL(k_uni_decide, dim3((nseg + 63) / 64), dim3(64), 0, s, segs, nseg, n_try, seed, b.part, b.mm,
                       out);
    hipLaunchKernelGGL(k_uni_count, dim3(nchunk), dim3(256), 0, s, chunks, TN, b.P, out, b.lcount);
    hipLaunchKernelGGL(k_uni_offsets, dim3((nseg + 63) / 64), dim3(64), 0, s, segs, nseg, b.lcount, b.loff, out);
    hipLaunchKernelGGL(k_uni_scatter, dim3(nchunk), dim3(256), 0, s, segs, chunks, TN, b.P, out, b.loff, perm, b.tmp);
    hipLaunchKernelGGL(k_uni_copy, dim3(nchunk), dim3(256), 0, s, chunks, b.tmp, perm);
    launch_check(s, "uniform chunked level");
}

}  // namespace rpf
