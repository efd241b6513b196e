// Tree growth (Alg. 1 with the median split point of Sec. 2, direction choice of Alg. 2),
// level-synchronous over all trees: at level l every internal node of every tree is a
// contiguous segment of that tree's permutation, and one launch processes all of them
// (grid.y = tree).  Per node: project the members onto the node's direction (binary64,
// canonical order), select the member of rank floor(m/2) in (p, index) order, and
// partition stably so that both children stay in ascending original index.
//
// Two paths:
//   - segments of at most kLarge members: one workgroup per (segment, tree) does the whole
//     step in LDS (k_level_small);
//   - larger segments: chunked projection with a fused first-digit histogram, radix
//     passes narrowing an 11-bit digit of the 96-bit key (p, index) per pass until at most
//     kCandCap candidates remain, an in-block select over the candidates, then a stable
//     chunked partition (count, scan, scatter).
#include "rpf_internal.h"

namespace rpf {

// ================================================================ small segments: fused level

template <bool VEC>
__device__ inline void project_segment(const float *__restrict__ X, int d, const float *s_r,
                                       const int32_t *s_perm, int m, double *s_p) {
    const int g = threadIdx.x & 7, pt = threadIdx.x >> 3;
    const int per = blockDim.x >> 3;
    for (int base = 0; base < m; base += per) {
        int i = base + pt;
        int ii = i < m ? i : 0;
        double p = group8_dot64<VEC>(X + (int64_t)s_perm[ii] * d, s_r, d, g);
        if (g == 0 && i < m) s_p[i] = p;
    }
}

// LDS layout: perm[m] int32 | key[m] u64 | dir[d] | hist[256] | misc ; nTry>1 adds p[m], tree[P2]
// Q8: the node projections read rows from the int8 grid copy Xq (stride dq); the same values
template <bool VEC, bool LEAD, bool Q8 = false>
__global__ __launch_bounds__(256) void k_level_small(
    const float *__restrict__ X, int d, const float *__restrict__ R, int64_t H, int n_try,
    const SegDesc *__restrict__ segs, const int32_t *__restrict__ perm_in,
    int32_t *__restrict__ perm_out, int64_t n, double *__restrict__ split,
    int32_t *__restrict__ split_idx, int32_t *__restrict__ chosen, int32_t *__restrict__ err,
    const LookDesc *__restrict__ look, double2 *__restrict__ ahead, uint64_t *__restrict__ keys_next,
    const uint64_t *__restrict__ keys_in, const int8_t *__restrict__ Xq, int dq) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int t = blockIdx.y;
    const SegDesc sg = segs[blockIdx.x];
    const int m = sg.size;
    const int tid = threadIdx.x;
    const int ds = (d + 3) & ~3;
    int32_t *s_perm = reinterpret_cast<int32_t *>(smem);
    uint64_t *s_key = reinterpret_cast<uint64_t *>(smem + ((4 * m + 15) & ~15));
    // the node's direction (binary32); on a lead level it and its children's, as binary64
    uint8_t *s_dir = smem + ((((4 * m + 15) & ~15) + 8 * m + 15) & ~15);  // 16-byte aligned
    float *s_r = reinterpret_cast<float *>(s_dir);
    double *s_rd = reinterpret_cast<double *>(s_dir);
    uint32_t *s_hist = reinterpret_cast<uint32_t *>(s_rd + 3 * ds);
    uint32_t *s_misc = s_hist + 256;  // 16 words
    double *s_p = reinterpret_cast<double *>(s_misc + 16);
    int P2 = 1;
    while (P2 < m) P2 <<= 1;
    double *s_tree = s_p + m;

    const int32_t *pin = perm_in + (int64_t)t * n + sg.off;
    for (int i = tid; i < m; i += blockDim.x) s_perm[i] = pin[i];
    const float *Rn = R + ((int64_t)t * H + (sg.heap - 1)) * n_try * (int64_t)d;

    int ch = 0;
    if (n_try > 1) {  // Alg. 2: keep the try with the largest spread S2 (first wins ties)
        double best = 0.0;
        int best_i = -1;
        for (int k = 0; k < n_try; k++) {
            __syncthreads();
            for (int j = tid; j < d; j += blockDim.x) s_r[j] = Rn[(int64_t)k * d + j];
            __syncthreads();
            project_segment<VEC>(X, d, s_r, s_perm, m, s_p);
            __syncthreads();
            for (int i = tid; i < m; i += blockDim.x) s_tree[i] = s_p[i];
            double s1 = block_canon_sum(s_tree, m);
            double mu = s1 / (double)m;
            for (int i = tid; i < m; i += blockDim.x) {
                double dev = s_p[i] - mu;
                s_tree[i] = __dmul_rn(dev, dev);
            }
            double s2 = block_canon_sum(s_tree, m);
            if (s2 > best) { best = s2; best_i = k; }
        }
        ch = best_i < 0 ? 0 : best_i;
    }
    __syncthreads();
    if (keys_in) {  // fed level: the keys were made by the partition of the level above
        for (int i = tid; i < m; i += blockDim.x) s_key[i] = keys_in[(int64_t)t * n + sg.off + i];
    } else if (LEAD) {  // lead level: the children's projections from the same read of X
        const LookDesc lk = look[blockIdx.x];
        for (int j = tid; j < d; j += blockDim.x) {
            s_rd[j] = Rn[j];
#pragma unroll
            for (int b = 0; b < 2; b++)  // a leaf child has no direction: project onto zero
                s_rd[ds * (b + 1) + j] =
                    lk.child_heap[b] > 0 ? R[((int64_t)t * H + (lk.child_heap[b] - 1)) * (int64_t)d + j] : 0.f;
        }
        __syncthreads();
        const int g = tid & 7, pt = tid >> 3;
        for (int base = 0; base < m; base += 64) {  // rows base + pt and base + 32 + pt
            const int ia = base + pt, ib = ia + 32;
            double p[6];
            if constexpr (Q8)
                group8_dot64x3r2_q8<VEC>(Xq + (int64_t)s_perm[ia < m ? ia : 0] * dq, Xq + (int64_t)s_perm[ib < m ? ib : 0] * dq,
                                    s_rd, ds, d, g, p);
            else
                group8_dot64x3r2<VEC>(X + (int64_t)s_perm[ia < m ? ia : 0] * d, X + (int64_t)s_perm[ib < m ? ib : 0] * d,
                                      s_rd, ds, d, g, p);
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int i = h ? ib : ia;
                if (g == 0 && i < m) {
                    s_key[i] = key_of(p[3 * h]);
                    ahead[(int64_t)t * n + sg.off + i] = make_double2(p[3 * h + 1], p[3 * h + 2]);
                }
            }
        }
    } else {
        for (int j = tid; j < d; j += blockDim.x) s_r[j] = Rn[(int64_t)ch * d + j];
        __syncthreads();
        const int g = tid & 7, pt = tid >> 3;
        for (int base = 0; base < m; base += 32) {
            int i = base + pt;
            int ii = i < m ? i : 0;
            double p;
            if constexpr (Q8) p = group8_dot64_q8<VEC>(Xq + (int64_t)s_perm[ii] * dq, s_r, d, g);
            else p = group8_dot64<VEC>(X + (int64_t)s_perm[ii] * d, s_r, d, g);
            if (g == 0 && i < m) s_key[i] = key_of(p);
        }
    }
    __syncthreads();

    // ---- select rank floor(m/2) in (key, index) order: 8-bit radix passes over the 96-bit key
    uint64_t phi = 0;
    uint32_t plo = 0;
    int nbits = 0;
    uint32_t rank = (uint32_t)(m / 2), cnt = (uint32_t)m;
    while (cnt > 1 && nbits < 96) {
        const int lo_bit = 88 - nbits;
        const unsigned __int128 P = key96(phi, plo);
        s_hist[tid] = 0;
        __syncthreads();
        for (int i = tid; i < m; i += blockDim.x) {
            unsigned __int128 K = key96(s_key[i], (uint32_t)s_perm[i]);
            if (nbits == 0 || (K >> (96 - nbits)) == (P >> (96 - nbits)))
                atomicAdd(&s_hist[(uint32_t)(K >> lo_bit) & 255u], 1u);
        }
        __syncthreads();
        uint32_t v = s_hist[tid], excl, total;
        block_excl_scan256(v, s_misc, excl, total);
        if (excl <= rank && rank < excl + v) {
            s_misc[8] = tid;
            s_misc[9] = excl;
            s_misc[10] = v;
        }
        __syncthreads();
        const uint32_t b = s_misc[8];
        rank -= s_misc[9];
        cnt = s_misc[10];
        unsigned __int128 NP = P | ((unsigned __int128)b << lo_bit);
        phi = (uint64_t)(NP >> 32);
        plo = (uint32_t)NP;
        nbits += 8;
        __syncthreads();
    }
    if (nbits < 96) {  // exactly one key matches the prefix: it is the median
        const unsigned __int128 P = key96(phi, plo);
        for (int i = tid; i < m; i += blockDim.x) {
            unsigned __int128 K = key96(s_key[i], (uint32_t)s_perm[i]);
            if ((K >> (96 - nbits)) == (P >> (96 - nbits))) {
                s_misc[12] = (uint32_t)s_key[i];
                s_misc[13] = (uint32_t)(s_key[i] >> 32);
                s_misc[14] = (uint32_t)s_perm[i];
            }
        }
        __syncthreads();
        phi = ((uint64_t)s_misc[13] << 32) | s_misc[12];
        plo = s_misc[14];
    }

    // ---- stable partition: left = keys below (c, c_idx), in position (= index) order
    const int half = m / 2;
    int32_t *pout = perm_out + (int64_t)t * n + sg.off;
    uint32_t lefts = 0;
    for (int base = 0; base < m; base += 256) {
        const int i = base + tid;
        const bool valid = i < m;
        const bool left = valid && key_less(s_key[i], (uint32_t)s_perm[i], phi, plo);
        uint32_t excl, total;
        block_excl_scan256(left ? 1u : 0u, s_misc, excl, total);
        if (valid) {
            uint32_t lb = lefts + excl;
            int pos = left ? (int)lb : half + (i - (int)lb);
            if (pos >= 0 && pos < m) {  // always true when the select is consistent
                pout[pos] = s_perm[i];
                if (LEAD) {  // the row's key at the next level: its projection onto its child
                    const double2 a = ahead[(int64_t)t * n + sg.off + i];
                    keys_next[(int64_t)t * n + sg.off + pos] = key_of(left ? a.x : a.y);
                }
            }
        }
        lefts += total;
    }
    if (tid == 0) {
        const int64_t hs = (int64_t)t * H + (sg.heap - 1);
        split[hs] = val_of(phi);
        split_idx[hs] = (int32_t)plo;
        chosen[hs] = ch;
        if (lefts != (uint32_t)half) atomicOr(err, 1);
    }
}


// Fed levels of small segments (at most 64 E members, one direction per node): one wave per
// (segment, tree), four segments per workgroup.  The wave holds the keys the lead level's
// partition made and the member ids in registers, E per lane (position i = lane + 64 e),
// selects the member of rank floor(m/2) in (key, index) order with 8-bit
// radix passes over a per-wave LDS histogram, and writes the stable partition: the same
// operations and result as k_level_small on a fed level, without workgroup barriers.
constexpr int kWaveSeg = 1024;  // largest segment of the wave-per-segment fed level

template <int E>
__global__ __launch_bounds__(256) void k_level_fed_wave(const SegDesc *__restrict__ segs, int nseg,
                                                        const int32_t *__restrict__ perm_in,
                                                        int32_t *__restrict__ perm_out, int64_t n, int64_t H,
                                                        double *__restrict__ split, int32_t *__restrict__ split_idx,
                                                        int32_t *__restrict__ chosen, int32_t *__restrict__ err,
                                                        const uint64_t *__restrict__ keys_in) {
    __shared__ uint32_t s_hist[4][256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int k = blockIdx.x * 4 + w, t = blockIdx.y;
    if (k >= nseg) return;  // a whole wave; nothing below waits on the workgroup
    const SegDesc sg = segs[k];
    const int m = sg.size;
    const int32_t *pin = perm_in + (int64_t)t * n + sg.off;
    const uint64_t *kin = keys_in + (int64_t)t * n + sg.off;
    uint64_t kk[E];
    uint32_t id[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int i = lane + 64 * e;
        kk[e] = i < m ? kin[i] : 0;
        id[e] = i < m ? (uint32_t)pin[i] : 0u;
    }
    uint32_t *h = s_hist[w];
    uint64_t phi = 0;
    uint32_t plo = 0;
    int nbits = 0;
    uint32_t rank = (uint32_t)(m / 2), cnt = (uint32_t)m;
    while (cnt > 1 && nbits < 96) {
        const int lo_bit = 88 - nbits;
        const unsigned __int128 P = key96(phi, plo);
#pragma unroll
        for (int j = 0; j < 4; j++) h[lane + 64 * j] = 0;
        wave_sync();
#pragma unroll
        for (int e = 0; e < E; e++) {
            const int i = lane + 64 * e;
            const unsigned __int128 K = key96(kk[e], id[e]);
            if (i < m && (nbits == 0 || (K >> (96 - nbits)) == (P >> (96 - nbits))))
                atomicAdd(&h[(uint32_t)(K >> lo_bit) & 255u], 1u);
        }
        wave_sync();
        // lane l holds bins 4l .. 4l + 3; an inclusive scan of their sums over the lanes
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            v[j] = h[4 * lane + j];
            sum += v[j];
        }
        uint32_t incl = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        uint32_t run = incl - sum;  // members in the bins below this lane's
        int bsel = -1;
        uint32_t ex = 0, vc = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (bsel < 0 && run <= rank && rank < run + v[j]) {
                bsel = 4 * lane + j;
                ex = run;
                vc = v[j];
            }
            run += v[j];
        }
        const uint64_t own = __ballot(bsel >= 0);  // exactly one lane holds the rank
        const int src = own ? __builtin_ctzll(own) : 0;
        const uint32_t b = (uint32_t)__shfl(bsel, src, 64);
        rank -= (uint32_t)__shfl((int)ex, src, 64);
        cnt = (uint32_t)__shfl((int)vc, src, 64);
        const unsigned __int128 NP = P | ((unsigned __int128)b << lo_bit);
        phi = (uint64_t)(NP >> 32);
        plo = (uint32_t)NP;
        nbits += 8;
        wave_sync();  // every read of the histogram is done before the next pass clears it
    }
    if (nbits < 96) {  // exactly one key matches the prefix: it is the median
        const unsigned __int128 P = key96(phi, plo);
        uint64_t mh = 0;
        uint32_t ml = 0;
        bool found = false;
#pragma unroll
        for (int e = 0; e < E; e++) {
            const int i = lane + 64 * e;
            const unsigned __int128 K = key96(kk[e], id[e]);
            if (i < m && (K >> (96 - nbits)) == (P >> (96 - nbits))) {
                mh = kk[e];
                ml = id[e];
                found = true;
            }
        }
        const uint64_t own = __ballot(found);
        const int src = own ? __builtin_ctzll(own) : 0;
        phi = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(mh >> 32), src, 64) << 32) |
              (uint32_t)__shfl((int)(uint32_t)mh, src, 64);
        plo = (uint32_t)__shfl((int)ml, src, 64);
    }
    // stable partition: left = keys below (c, c_idx), in position (= index) order
    const int half = m / 2;
    int32_t *pout = perm_out + (int64_t)t * n + sg.off;
    uint32_t lefts = 0;
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int i = lane + 64 * e;
        const bool valid = i < m;
        const bool left = valid && key_less(kk[e], id[e], phi, plo);
        const uint64_t mk = __ballot(left);
        if (valid) {
            const int lb = (int)lefts + mask_rank(mk);
            const int pos = left ? lb : half + (i - lb);
            if (pos >= 0 && pos < m) pout[pos] = (int32_t)id[e];
        }
        lefts += (uint32_t)__popcll(mk);
    }
    if (lane == 0) {
        const int64_t hs = (int64_t)t * H + (sg.heap - 1);
        split[hs] = val_of(phi);
        split_idx[hs] = (int32_t)plo;
        chosen[hs] = 0;
        if (lefts != (uint32_t)half) atomicOr(err, 1);
    }
}

// ================================================================ small subtrees: one persistent launch

// One internal node of a subtree, by the whole block (256 threads), nTry = 1: project the
// members s_perm[0 .. m) onto the node's direction r (binary64, canonical order), select the
// member of rank floor(m/2) in (p, index) order, and write the stable partition to s_out.
// The same operations, in the same order, as k_level_small on a one-direction level.
template <bool VEC>
__device__ inline void subtree_node(const float *__restrict__ X, int d, const float *__restrict__ r,
                                    const int32_t *s_perm, int32_t *s_out, int m, uint64_t *s_key, float *s_r,
                                    uint32_t *s_hist, uint32_t *s_misc, double *split_out, int32_t *split_idx_out,
                                    int32_t *chosen_out, int32_t *err) {
    const int tid = threadIdx.x;
    for (int j = tid; j < d; j += blockDim.x) s_r[j] = r[j];
    __syncthreads();
    {
        const int g = tid & 7, pt = tid >> 3;
        for (int base = 0; base < m; base += 32) {
            const int i = base + pt;
            const double p = group8_dot64<VEC>(X + (int64_t)s_perm[i < m ? i : 0] * d, s_r, d, g);
            if (g == 0 && i < m) s_key[i] = key_of(p);
        }
    }
    __syncthreads();
    uint64_t phi = 0;
    uint32_t plo = 0;
    int nbits = 0;
    uint32_t rank = (uint32_t)(m / 2), cnt = (uint32_t)m;
    while (cnt > 1 && nbits < 96) {
        const int lo_bit = 88 - nbits;
        const unsigned __int128 P = key96(phi, plo);
        s_hist[tid] = 0;
        __syncthreads();
        for (int i = tid; i < m; i += blockDim.x) {
            const unsigned __int128 K = key96(s_key[i], (uint32_t)s_perm[i]);
            if (nbits == 0 || (K >> (96 - nbits)) == (P >> (96 - nbits)))
                atomicAdd(&s_hist[(uint32_t)(K >> lo_bit) & 255u], 1u);
        }
        __syncthreads();
        const uint32_t v = s_hist[tid];
        uint32_t excl, total;
        block_excl_scan256(v, s_misc, excl, total);
        if (excl <= rank && rank < excl + v) {
            s_misc[8] = tid;
            s_misc[9] = excl;
            s_misc[10] = v;
        }
        __syncthreads();
        const uint32_t b = s_misc[8];
        rank -= s_misc[9];
        cnt = s_misc[10];
        const unsigned __int128 NP = P | ((unsigned __int128)b << lo_bit);
        phi = (uint64_t)(NP >> 32);
        plo = (uint32_t)NP;
        nbits += 8;
        __syncthreads();
    }
    if (nbits < 96) {  // exactly one key matches the prefix: it is the median
        const unsigned __int128 P = key96(phi, plo);
        for (int i = tid; i < m; i += blockDim.x) {
            const unsigned __int128 K = key96(s_key[i], (uint32_t)s_perm[i]);
            if ((K >> (96 - nbits)) == (P >> (96 - nbits))) {
                s_misc[12] = (uint32_t)s_key[i];
                s_misc[13] = (uint32_t)(s_key[i] >> 32);
                s_misc[14] = (uint32_t)s_perm[i];
            }
        }
        __syncthreads();
        phi = ((uint64_t)s_misc[13] << 32) | s_misc[12];
        plo = s_misc[14];
    }
    const int half = m / 2;
    uint32_t lefts = 0;
    for (int base = 0; base < m; base += 256) {
        const int i = base + tid;
        const bool valid = i < m;
        const bool left = valid && key_less(s_key[i], (uint32_t)s_perm[i], phi, plo);
        uint32_t excl, total;
        block_excl_scan256(left ? 1u : 0u, s_misc, excl, total);
        if (valid) {
            const uint32_t lb = lefts + excl;
            const int pos = left ? (int)lb : half + (i - (int)lb);
            if (pos >= 0 && pos < m) s_out[pos] = s_perm[i];  // always in range when the select is consistent
        }
        lefts += total;
    }
    if (tid == 0) {
        *split_out = val_of(phi);
        *split_idx_out = (int32_t)plo;
        *chosen_out = 0;
        if (lefts != (uint32_t)half) atomicOr(err, 1);
    }
    __syncthreads();
}

// Persistent launch over the small levels: a fixed grid of resident blocks takes items (tree,
// internal node of the first small level) from a device counter until none is left, and
// grows each item's whole subtree inside the block, level by level (a node's children only
// after its partition: the level dependencies stay inside the block).  The item's permutation
// segment stays in LDS (two buffers, one per level parity) and is written once, in leaf order,
// to perm_out.  Every block leaves the loop when the counter passes the item count.
template <bool VEC>
__global__ __launch_bounds__(256) void k_subtree(const float *__restrict__ X, int d, const float *__restrict__ R,
                                                 int64_t H, const SubItem *__restrict__ items, int nitems, int T,
                                                 int n0, const int32_t *__restrict__ perm_in,
                                                 int32_t *__restrict__ perm_out, int64_t n,
                                                 double *__restrict__ split, int32_t *__restrict__ split_idx,
                                                 int32_t *__restrict__ chosen, int32_t *__restrict__ err,
                                                 uint32_t *__restrict__ next, int max_m) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int mp = (max_m + 3) & ~3;
    int32_t *s_pa = reinterpret_cast<int32_t *>(smem);
    int32_t *s_pb = s_pa + mp;
    uint64_t *s_key = reinterpret_cast<uint64_t *>(s_pb + mp);
    float *s_r = reinterpret_cast<float *>(s_key + mp);
    uint32_t *s_hist = reinterpret_cast<uint32_t *>(s_r + ((d + 3) & ~3));
    uint32_t *s_misc = s_hist + 256;  // 16 words; [15] = the block's current item
    const int tid = threadIdx.x;
    const uint32_t total = (uint32_t)nitems * (uint32_t)T;
    while (true) {
        if (tid == 0) s_misc[15] = atomicAdd(next, 1u);
        __syncthreads();
        const uint32_t w = s_misc[15];
        __syncthreads();
        if (w >= total) break;
        const int t = (int)(w / (uint32_t)nitems);
        const SubItem it = items[w % (uint32_t)nitems];
        const int m0 = it.size;
        int32_t *pa = s_pa, *pb = s_pb;
        const int32_t *pin = perm_in + (int64_t)t * n + it.off;
        for (int i = tid; i < m0; i += blockDim.x) pa[i] = pin[i];
        for (int k = 0; k < 31; k++) {  // relative depth k: nodes j = 0 .. 2^k - 1 of the subtree
            for (int i = tid; i < m0; i += blockDim.x) pb[i] = pa[i];  // leaves stay in place
            __syncthreads();
            bool any = false;
            for (int j = 0; j < (1 << k); j++) {
                int lo = 0, sz = m0;
                int64_t hl = it.heap - it.hbase;  // heap id within the data set
                bool present = true;
                for (int b = k - 1; b >= 0; b--) {  // walk down from the item: left = floor(m/2)
                    if (sz <= n0) {
                        present = false;
                        break;
                    }
                    const int left = sz / 2;
                    if ((j >> b) & 1) {
                        lo += left;
                        sz -= left;
                        hl = 2 * hl + 1;
                    } else {
                        sz = left;
                        hl = 2 * hl;
                    }
                }
                if (!present || sz <= n0) continue;
                any = true;
                const int64_t hs = (int64_t)t * H + (it.hbase + hl - 1);
                subtree_node<VEC>(X, d, R + hs * d, pa + lo, pb + lo, sz, s_key, s_r, s_hist, s_misc, split + hs,
                                  split_idx + hs, chosen + hs, err);
            }
            if (!any) break;
            int32_t *tmp = pa;
            pa = pb;
            pb = tmp;
        }
        __syncthreads();
        int32_t *pout = perm_out + (int64_t)t * n + it.off;
        for (int i = tid; i < m0; i += blockDim.x) pout[i] = pa[i];
        __syncthreads();
    }
}

size_t subtree_lds(int max_m, int d) {
    const size_t mp = (size_t)((max_m + 3) & ~3);
    return mp * 4 * 2 + mp * 8 + (size_t)((d + 3) & ~3) * 4 + 4 * (256 + 16);
}

void launch_subtree(hipStream_t s, bool vec, const float *X, int d, const float *R, int64_t H, const SubItem *items,
                    int nitems, int T, int n0, const int32_t *pin, int32_t *pout, int64_t n, double *split,
                    int32_t *split_idx, int32_t *chosen, int32_t *err, uint32_t *next, int max_m, int lds_limit) {
    if (nitems <= 0) return;
    const size_t lds = subtree_lds(max_m, d);
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int per_cu = std::max(1, std::min(8, (int)((size_t)lds_limit / std::max<size_t>(lds, 1))));
    const int64_t total = (int64_t)nitems * T;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(total, (int64_t)std::max(cus, 1) * per_cu));
    fill_u32(next, 1, 0, s);
    auto go = [&](auto kern) {
        hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), lds, s, X, d, R, H, items, nitems, T, n0, pin, pout, n, split,
                           split_idx, chosen, err, next, max_m);
    };
    if (vec) go(k_subtree<true>);
    else go(k_subtree<false>);
    launch_check(s, "k_subtree");
}

// ================================================================ large segments

// Q8: rows read from the int8 grid copy Xq (stride dq) instead of X; the same values
template <bool VEC, bool LEAD, bool Q8 = false>
__global__ __launch_bounds__(256) void k_proj_chunks(
    const float *__restrict__ X, int d, const float *__restrict__ R, int64_t H, int n_try,
    const SegDesc *__restrict__ segs, const ChunkDesc *__restrict__ chunks,
    const int32_t *__restrict__ perm, int64_t n, SelState *__restrict__ state, int nseg,
    int mode,  // 0: final projection -> keys + digit-0 histogram; 1: raw projection of try `tr`
    int tr, uint64_t *__restrict__ keys, double *__restrict__ praw, uint32_t *__restrict__ hist,
    const LookDesc *__restrict__ look, double2 *__restrict__ ahead, const int8_t *__restrict__ Xq, int dq) {
    // the node's direction (binary32); on a lead level it and its children's, as binary64
    extern __shared__ __align__(16) uint8_t s_dir[];
    float *s_r = reinterpret_cast<float *>(s_dir);
    __shared__ uint32_t s_hist[kDigitBins];
    const int t = blockIdx.y;
    const ChunkDesc c = chunks[blockIdx.x];
    const SegDesc sg = segs[c.seg];
    const int tid = threadIdx.x;
    const SelState *st = state + (int64_t)t * nseg + c.seg;
    const int ch = mode == 0 ? st->chosen : tr;
    const float *Rn = R + (((int64_t)t * H + (sg.heap - 1)) * n_try + ch) * (int64_t)d;
    const int32_t *pp = perm + (int64_t)t * n;
    if (mode == 0)
        for (int b = tid; b < kDigitBins; b += 256) s_hist[b] = 0;
    const int g = tid & 7, pt = tid >> 3;
    if (LEAD && d <= 1024) {  // lead level: the children's projections from the same read of X
        const LookDesc lk = look[c.seg];
        const int ds = (d + 3) & ~3;
        double *s_rd = reinterpret_cast<double *>(s_dir);
        for (int j = tid; j < d; j += 256) {
            s_rd[j] = Rn[j];
#pragma unroll
            for (int b = 0; b < 2; b++)  // a leaf child has no direction: project onto zero
                s_rd[ds * (b + 1) + j] =
                    lk.child_heap[b] > 0 ? R[((int64_t)t * H + (lk.child_heap[b] - 1)) * (int64_t)d + j] : 0.f;
        }
        __syncthreads();
        for (int base = 0; base < c.len; base += 64) {  // rows base + pt and base + 32 + pt
            const int ia = base + pt, ib = ia + 32;
            const int64_t sa = c.start + (ia < c.len ? ia : 0), sb = c.start + (ib < c.len ? ib : 0);
            double p[6];
            if constexpr (Q8) group8_dot64x3r2_q8<VEC>(Xq + (int64_t)pp[sa] * dq, Xq + (int64_t)pp[sb] * dq, s_rd, ds, d, g, p);
            else group8_dot64x3r2<VEC>(X + (int64_t)pp[sa] * d, X + (int64_t)pp[sb] * d, s_rd, ds, d, g, p);
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int i = h ? ib : ia;
                const int64_t s = h ? sb : sa;
                if (g == 0 && i < c.len) {
                    uint64_t u = key_of(p[3 * h]);
                    keys[(int64_t)t * n + s] = u;
                    ahead[(int64_t)t * n + s] = make_double2(p[3 * h + 1], p[3 * h + 2]);
                    atomicAdd(&s_hist[(uint32_t)(u >> 53)], 1u);
                }
            }
        }
    } else if (d <= 1024) {  // longer directions are read from global memory by the scalar loop below
        for (int j = tid; j < d; j += 256) s_r[j] = Rn[j];
        __syncthreads();
        for (int base = 0; base < c.len; base += 32) {
            const int i = base + pt;
            const int64_t s = c.start + (i < c.len ? i : 0);
            double p;
            if constexpr (Q8) p = group8_dot64_q8<VEC>(Xq + (int64_t)pp[s] * dq, s_r, d, g);
            else p = group8_dot64<VEC>(X + (int64_t)pp[s] * d, s_r, d, g);
            if (g == 0 && i < c.len) {
                if (mode == 0) {
                    uint64_t u = key_of(p);
                    keys[(int64_t)t * n + s] = u;
                    atomicAdd(&s_hist[(uint32_t)(u >> 53)], 1u);
                } else {
                    praw[(int64_t)t * n + s] = p;
                }
            }
        }
    } else {
        for (int base = 0; base < c.len; base += 32) {
            const int i = base + pt;
            const int64_t s = c.start + (i < c.len ? i : 0);
            double p;
            if constexpr (Q8) p = group8_dot64_q8<false>(Xq + (int64_t)pp[s] * dq, Rn, d, g);
            else p = group8_dot64<false>(X + (int64_t)pp[s] * d, Rn, d, g);
            if (g == 0 && i < c.len) {
                if (mode == 0) {
                    uint64_t u = key_of(p);
                    keys[(int64_t)t * n + s] = u;
                    atomicAdd(&s_hist[(uint32_t)(u >> 53)], 1u);
                } else {
                    praw[(int64_t)t * n + s] = p;
                }
            }
        }
    }
    if (mode == 0) {
        __syncthreads();
        uint32_t *gh = hist + ((int64_t)t * nseg + c.seg) * kDigitBins;
        for (int b = tid; b < kDigitBins; b += 256)
            if (s_hist[b]) atomicAdd(&gh[b], s_hist[b]);
    }
}

__global__ void k_sel_init(const SegDesc *__restrict__ segs, int nseg, int T, SelState *state) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nseg * T) return;
    const SegDesc sg = segs[i % nseg];
    SelState s;
    s.pfx_hi = 0;
    s.pfx_lo = 0;
    s.nbits = 0;
    s.rank = sg.size / 2;
    s.cnt = sg.size;
    s.mode = SEL_HIST;
    s.chosen = 0;
    s.best_s2 = 0.0;
    s.s1 = 0.0;
    s.counted = 0;
    s.pad = 0;
    state[i] = s;
}

// digit j covers key bits [lo_bit, lo_bit + width) of the 96-bit key, from the top
__device__ inline int digit_width(int j) { return j < 8 ? 11 : 8; }

__global__ __launch_bounds__(256) void k_sel_scan(SelState *__restrict__ state, int nseg,
                                                  uint32_t *__restrict__ hist) {
    __shared__ uint32_t s_w[8];
    __shared__ uint32_t s_res[4];
    const int t = blockIdx.y, k = blockIdx.x, tid = threadIdx.x;
    SelState *stp = state + (int64_t)t * nseg + k;
    const int mode = stp->mode;
    if (mode == SEL_COMPACT) {
        if (tid == 0) stp->mode = SEL_GATHERED;
        return;
    }
    if (mode != SEL_HIST) return;
    const int j = stp->nbits / kDigitBits;
    const int w = digit_width(j);
    const int lo_bit = 96 - stp->nbits - w;
    uint32_t *h = hist + ((int64_t)t * nseg + k) * kDigitBins;
    const int nb = 1 << w;
    const int per = nb / 256;  // 8 (11-bit digit) or 1 (8-bit digit)
    uint32_t loc[8];
    uint32_t sum = 0;
    for (int q = 0; q < per; q++) {
        loc[q] = h[tid * per + q];
        sum += loc[q];
    }
    uint32_t excl;
    // block exclusive scan of per-thread sums (64-bit ranks fit in 32 bits: segments < 2^31)
    {
        const int lane = tid & 63, wv = tid >> 6;
        uint32_t x = sum;
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_w[wv] = x;
        __syncthreads();
        uint32_t wb = 0;
        for (int q = 0; q < 4; q++)
            if (q < wv) wb += s_w[q];
        excl = wb + x - sum;
    }
    const uint32_t rank = (uint32_t)stp->rank;
    if (excl <= rank && rank < excl + sum) {
        uint32_t c = excl;
        for (int q = 0; q < per; q++) {
            if (rank < c + loc[q]) {
                s_res[0] = tid * per + q;
                s_res[1] = c;
                s_res[2] = loc[q];
                break;
            }
            c += loc[q];
        }
    }
    __syncthreads();
    for (int q = 0; q < per; q++) h[tid * per + q] = 0;  // ready for the next digit
    if (tid == 0) {
        const uint32_t b = s_res[0];
        unsigned __int128 P = key96(stp->pfx_hi, stp->pfx_lo) | ((unsigned __int128)b << lo_bit);
        stp->pfx_hi = (uint64_t)(P >> 32);
        stp->pfx_lo = (uint32_t)P;
        stp->nbits += w;
        stp->rank = rank - s_res[1];
        stp->cnt = s_res[2];
        if (stp->nbits == 96) stp->mode = SEL_DONE;
        else if (stp->cnt <= kCandCap) stp->mode = SEL_COMPACT;
    }
}

__global__ __launch_bounds__(256) void k_sel_pass(const ChunkDesc *__restrict__ chunks,
                                                  const uint64_t *__restrict__ keys,
                                                  const int32_t *__restrict__ perm, int64_t n,
                                                  SelState *__restrict__ state, int nseg,
                                                  uint32_t *__restrict__ hist,
                                                  Cand *__restrict__ cand,
                                                  uint32_t *__restrict__ cand_cnt,
                                                  uint32_t *__restrict__ lcount, int nchunk) {
    __shared__ uint32_t s_hist[kDigitBins];
    __shared__ uint32_t s_w[8];
    const int t = blockIdx.y, tid = threadIdx.x;
    const ChunkDesc c = chunks[blockIdx.x];
    const SelState st = state[(int64_t)t * nseg + c.seg];
    if (st.mode != SEL_HIST && st.mode != SEL_COMPACT) return;
    const unsigned __int128 P = key96(st.pfx_hi, st.pfx_lo);
    const int sh = 96 - st.nbits;
    const uint64_t *kk = keys + (int64_t)t * n;
    const int32_t *pp = perm + (int64_t)t * n;
    if (st.mode == SEL_HIST) {
        const int j = st.nbits / kDigitBits;
        const int w = digit_width(j);
        const int lo_bit = 96 - st.nbits - w;
        const uint32_t msk = (1u << w) - 1;
        for (int b = tid; b < kDigitBins; b += 256) s_hist[b] = 0;
        __syncthreads();
        for (int i = tid; i < c.len; i += 256) {
            const int64_t s = c.start + i;
            unsigned __int128 K = key96(kk[s], (uint32_t)pp[s]);
            if (st.nbits == 0 || (K >> sh) == (P >> sh)) atomicAdd(&s_hist[(uint32_t)(K >> lo_bit) & msk], 1u);
        }
        __syncthreads();
        uint32_t *gh = hist + ((int64_t)t * nseg + c.seg) * kDigitBins;
        for (int b = tid; b < kDigitBins; b += 256)
            if (s_hist[b]) atomicAdd(&gh[b], s_hist[b]);
    } else {
        // gather the keys matching the prefix (at most kCandCap of them in the segment), each
        // with its chunk; the chunk's keys below the prefix are counted on the way, so that
        // the median's final step can complete the chunk's left count for the partition
        uint32_t mine = 0, below = 0;
        for (int i = tid; i < c.len; i += 256) {
            const int64_t s = c.start + i;
            unsigned __int128 K = key96(kk[s], (uint32_t)pp[s]);
            mine += ((K >> sh) == (P >> sh)) ? 1u : 0u;
            below += ((K >> sh) < (P >> sh)) ? 1u : 0u;
        }
        const int lane = tid & 63, wv = tid >> 6;
        uint32_t x = mine;
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        for (int o = 32; o > 0; o >>= 1) below += __shfl_xor(below, o, 64);
        if (lane == 63) s_w[wv] = x;
        if (lane == 0) s_w[4 + wv] = below;
        __syncthreads();
        uint32_t wb = 0, total = 0;
        for (int q = 0; q < 4; q++) {
            if (q < wv) wb += s_w[q];
            total += s_w[q];
        }
        if (tid == 0) lcount[(int64_t)t * nchunk + blockIdx.x] = s_w[4] + s_w[5] + s_w[6] + s_w[7];
        if (total == 0) return;
        __syncthreads();  // s_w[4] is read above before it is reused below
        if (tid == 0) s_w[4] = atomicAdd(&cand_cnt[(int64_t)t * nseg + c.seg], total);
        __syncthreads();
        uint32_t pos = s_w[4] + wb + x - mine;
        Cand *cc = cand + ((int64_t)t * nseg + c.seg) * kCandCap;
        for (int i = tid; i < c.len; i += 256) {
            const int64_t s = c.start + i;
            unsigned __int128 K = key96(kk[s], (uint32_t)pp[s]);
            if ((K >> sh) == (P >> sh)) {
                if (pos < (uint32_t)kCandCap) cc[pos] = Cand{kk[s], (uint32_t)pp[s], (uint32_t)blockIdx.x};
                pos++;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_sel_finish(const SegDesc *__restrict__ segs,
                                                    SelState *__restrict__ state, int nseg,
                                                    const Cand *__restrict__ cand,
                                                    const uint32_t *__restrict__ cand_cnt,
                                                    int64_t H, double *__restrict__ split,
                                                    int32_t *__restrict__ split_idx,
                                                    int32_t *__restrict__ chosen,
                                                    int32_t *__restrict__ err,
                                                    uint32_t *__restrict__ lcount, int nchunk) {
    __shared__ uint64_t s_hi[kCandCap];
    __shared__ uint32_t s_lo[kCandCap];
    __shared__ uint32_t s_h[256];
    __shared__ uint32_t s_w[8];
    __shared__ uint32_t s_sel[3];
    const int t = blockIdx.y, k = blockIdx.x, tid = threadIdx.x;
    SelState *stp = state + (int64_t)t * nseg + k;
    const SelState st = *stp;
    __syncthreads();
    if (st.mode == SEL_GATHERED) {
        const uint32_t cnt = cand_cnt[(int64_t)t * nseg + k];
        if (cnt != (uint32_t)st.cnt || cnt > (uint32_t)kCandCap) {
            if (tid == 0) atomicOr(err, 2);
            return;
        }
        const Cand *cc = cand + ((int64_t)t * nseg + k) * kCandCap;
        for (uint32_t i = tid; i < cnt; i += 256) {
            s_hi[i] = cc[i].hi;
            s_lo[i] = cc[i].lo;
        }
        __syncthreads();
        // in-block radix select over the candidates, which share the top st.nbits bits:
        // 8-bit digits of the 96-bit key until one candidate matches the prefix
        unsigned __int128 P = key96(st.pfx_hi, st.pfx_lo);
        int nbits = st.nbits;
        uint32_t rank = (uint32_t)st.rank, c = cnt;
        while (c > 1 && nbits < 96) {
            const int w = 96 - nbits < 8 ? 96 - nbits : 8;
            const int lo_bit = 96 - nbits - w;
            s_h[tid] = 0;
            __syncthreads();
            for (uint32_t i = tid; i < cnt; i += 256) {
                const unsigned __int128 Kc = key96(s_hi[i], s_lo[i]);
                if ((Kc >> (96 - nbits)) == (P >> (96 - nbits)))
                    atomicAdd(&s_h[(uint32_t)(Kc >> lo_bit) & ((1u << w) - 1u)], 1u);
            }
            __syncthreads();
            const uint32_t v = s_h[tid];
            uint32_t excl, total;
            block_excl_scan256(v, s_w, excl, total);
            if (excl <= rank && rank < excl + v) {
                s_sel[0] = tid;
                s_sel[1] = excl;
                s_sel[2] = v;
            }
            __syncthreads();
            P |= (unsigned __int128)s_sel[0] << lo_bit;
            rank -= s_sel[1];
            c = s_sel[2];
            nbits += w;
            __syncthreads();
        }
        for (uint32_t i = tid; i < cnt; i += 256) {  // the one candidate with the full prefix
            const unsigned __int128 Kc = key96(s_hi[i], s_lo[i]);
            if ((Kc >> (96 - nbits)) == (P >> (96 - nbits))) {
                stp->pfx_hi = s_hi[i];
                stp->pfx_lo = s_lo[i];
                stp->nbits = 96;
                stp->mode = SEL_DONE;
            }
        }
        __syncthreads();
        // the partition's left count of every chunk: its keys below the gathered prefix
        // (counted by the gathering pass) plus its candidates below the median
        const SelState fs = *stp;
        if (fs.mode == SEL_DONE) {
            const unsigned __int128 S = key96(fs.pfx_hi, fs.pfx_lo);
            for (uint32_t i = tid; i < cnt; i += 256)
                if (key96(s_hi[i], s_lo[i]) < S) atomicAdd(&lcount[(int64_t)t * nchunk + cc[i].pad], 1u);
            if (tid == 0) stp->counted = 1;
        }
    } else if (st.mode != SEL_DONE) {
        if (tid == 0) atomicOr(err, 4);
        return;
    }
    if (tid == 0) {
        const SelState fin = *stp;
        const int64_t hs = (int64_t)t * H + (segs[k].heap - 1);
        split[hs] = val_of(fin.pfx_hi);
        split_idx[hs] = (int32_t)fin.pfx_lo;
        chosen[hs] = fin.chosen;
        if (fin.mode != SEL_DONE) atomicOr(err, 8);
    }
}

__global__ __launch_bounds__(256) void k_part_count(const ChunkDesc *__restrict__ chunks, int nchunk,
                                                    const uint64_t *__restrict__ keys,
                                                    const int32_t *__restrict__ perm, int64_t n,
                                                    const SelState *__restrict__ state, int nseg,
                                                    uint32_t *__restrict__ lcount) {
    __shared__ uint32_t s_w[4];
    const int t = blockIdx.y, tid = threadIdx.x;
    const ChunkDesc c = chunks[blockIdx.x];
    const SelState st = state[(int64_t)t * nseg + c.seg];
    if (st.counted) return;  // the median's final step counted this chunk already
    uint32_t mine = 0;
    for (int i = tid; i < c.len; i += 256) {
        const int64_t s = c.start + i;
        mine += key_less(keys[(int64_t)t * n + s], (uint32_t)perm[(int64_t)t * n + s], st.pfx_hi, st.pfx_lo) ? 1u : 0u;
    }
    for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o, 64);
    if ((tid & 63) == 0) s_w[tid >> 6] = mine;
    __syncthreads();
    if (tid == 0) lcount[(int64_t)t * nchunk + blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

__global__ void k_part_scan(const SegDesc *__restrict__ segs, const ChunkDesc *__restrict__ chunks,
                            int nchunk, int nseg, uint32_t *__restrict__ lcount,
                            int32_t *__restrict__ err) {
    // lcount[t][c] becomes the number of left members before chunk c within its segment
    const int t = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nseg) return;
    const SegDesc sg = segs[k];
    uint32_t run = 0;
    for (int q = 0; q < sg.nchunk; q++) {
        uint32_t *p = lcount + (int64_t)t * nchunk + sg.chunk0 + q;
        uint32_t v = *p;
        *p = run;
        run += v;
    }
    if (run != (uint32_t)(sg.size / 2)) atomicOr(err, 16);
}

__global__ __launch_bounds__(256) void k_part_scatter(const SegDesc *__restrict__ segs,
                                                      const ChunkDesc *__restrict__ chunks, int nchunk,
                                                      const uint64_t *__restrict__ keys,
                                                      const int32_t *__restrict__ perm_in,
                                                      int32_t *__restrict__ perm_out, int64_t n,
                                                      const SelState *__restrict__ state, int nseg,
                                                      const uint32_t *__restrict__ lbase,
                                                      const LookDesc *__restrict__ look,
                                                      const double2 *__restrict__ ahead,
                                                      uint64_t *__restrict__ keys_next,
                                                      uint32_t *__restrict__ hist_next, int nseg_next) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_hn[2][kDigitBins];  // lead level: digit-0 histograms of the two children
    const int t = blockIdx.y, tid = threadIdx.x;
    const ChunkDesc c = chunks[blockIdx.x];
    const SegDesc sg = segs[c.seg];
    const SelState st = state[(int64_t)t * nseg + c.seg];
    const int64_t half = sg.size / 2;
    uint32_t lefts = lbase[(int64_t)t * nchunk + blockIdx.x];
    const int64_t rel0 = c.start - sg.off;  // chunk position within the segment
    int32_t *pout = perm_out + (int64_t)t * n + sg.off;
    const bool lead = look != nullptr, hn = lead && hist_next != nullptr;
    LookDesc lk{{-1, -1}, {0, 0}};
    if (lead) lk = look[c.seg];
    if (hn) {
        for (int b = tid; b < 2 * kDigitBins; b += 256) (&s_hn[0][0])[b] = 0;
        __syncthreads();
    }
    for (int base = 0; base < c.len; base += 256) {
        const int i = base + tid;
        const bool valid = i < c.len;
        const int64_t s = c.start + (valid ? i : 0);
        const int32_t id = perm_in[(int64_t)t * n + s];
        const bool left = valid && key_less(keys[(int64_t)t * n + s], (uint32_t)id, st.pfx_hi, st.pfx_lo);
        uint32_t excl, total;
        block_excl_scan256(left ? 1u : 0u, s_w, excl, total);
        if (valid) {
            const int64_t lb = (int64_t)lefts + excl;
            const int64_t rel = rel0 + i;
            const int64_t pos = left ? lb : half + (rel - lb);
            if (pos >= 0 && pos < sg.size) {  // always true when the select is consistent
                pout[pos] = id;
                if (lead) {  // the row's key at the next level: its projection onto its child
                    const double2 a = ahead[(int64_t)t * n + s];
                    const uint64_t u = key_of(left ? a.x : a.y);
                    keys_next[(int64_t)t * n + sg.off + pos] = u;
                    if (hn && lk.child_seg[left ? 0 : 1] >= 0) atomicAdd(&s_hn[left ? 0 : 1][(uint32_t)(u >> 53)], 1u);
                }
            }
        }
        lefts += total;
    }
    if (hn) {
        __syncthreads();
        for (int b = 0; b < 2; b++) {
            if (lk.child_seg[b] < 0) continue;
            uint32_t *gh = hist_next + ((int64_t)t * nseg_next + lk.child_seg[b]) * kDigitBins;
            for (int q = tid; q < kDigitBins; q += 256)
                if (s_hn[b][q]) atomicAdd(&gh[q], s_hn[b][q]);
        }
    }
}

// Lead projections of the first level for every tree from one read of X.  At the roots the
// permutation is the identity in every tree, so the rows of a chunk are the same rows for
// all trees: a block keeps 64 of them in registers (eight lanes per row, two rows per group,
// d <= 128 and d % 4 == 0) and walks the trees, staging each tree's three directions (node
// and children, as binary64) in LDS, double-buffered.  Each projection is computed exactly
// as group8_dot64 computes it.  Writes the keys and the children's projections; the
// first-digit histograms come from a selection pass over the keys.
__global__ __launch_bounds__(256) void k_proj_root(const float *__restrict__ X, int d, const float *__restrict__ R,
                                                   int64_t H, int ntree, const SegDesc *__restrict__ segs,
                                                   const ChunkDesc *__restrict__ chunks,
                                                   const LookDesc *__restrict__ look, int64_t n,
                                                   uint64_t *__restrict__ keys, double2 *__restrict__ ahead) {
    constexpr int NJ = 4;                   // float4 steps per lane: d <= 128
    __shared__ __align__(16) double s_rd[2][3 * 128];
    const ChunkDesc c = chunks[blockIdx.x];
    const int sub0 = 64 * blockIdx.y;
    if (sub0 >= c.len) return;
    const SegDesc sg = segs[c.seg];
    const LookDesc lk = look[c.seg];
    const int tid = threadIdx.x, g = tid & 7, pt = tid >> 3;
    const int ia = sub0 + pt, ib = ia + 32;  // rows within the chunk
    const bool oka = ia < c.len, okb = ib < c.len;
    const float *xa = X + (c.start + (oka ? ia : 0)) * (int64_t)d;
    const float *xb = X + (c.start + (okb ? ib : 0)) * (int64_t)d;
    float4 ra[NJ], rb[NJ];
#pragma unroll
    for (int k = 0; k < NJ; k++) {
        const int j = 4 * g + 32 * k;
        ra[k] = j < d ? *reinterpret_cast<const float4 *>(xa + j) : make_float4(0.f, 0.f, 0.f, 0.f);
        rb[k] = j < d ? *reinterpret_cast<const float4 *>(xb + j) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // a tree's three directions (node, left child, right child; zero for a leaf child): thread
    // tid holds elements tid and tid + 256.  The loads for tree t + 2 are issued while tree t
    // is projected, and stored to LDS after it, so their latency is hidden.
    float nv[2];
    auto fetch = [&](int t) {
#pragma unroll
        for (int e = 0; e < 2; e++) {
            const int j = tid + 256 * e, k = j >> 7, jj = j & 127;
            float v = 0.f;
            if (j < 3 * 128 && jj < d) {
                const int heap = k == 0 ? sg.heap : k == 1 ? lk.child_heap[0] : lk.child_heap[1];
                if (heap > 0) v = R[((int64_t)t * H + (heap - 1)) * (int64_t)d + jj];
            }
            nv[e] = v;
        }
    };
    auto put = [&](double *dst) {
#pragma unroll
        for (int e = 0; e < 2; e++)
            if (tid + 256 * e < 3 * 128) dst[tid + 256 * e] = nv[e];
    };
    fetch(0);
    put(s_rd[0]);
    if (ntree > 1) fetch(1);
    for (int t = 0; t < ntree; t++) {
        __syncthreads();  // s_rd[t & 1] is staged; everyone is done with s_rd[(t + 1) & 1]
        const double *r = s_rd[t & 1];
        double s[6][4];
#pragma unroll
        for (int q = 0; q < 6; q++) s[q][0] = s[q][1] = s[q][2] = s[q][3] = 0.0;
#pragma unroll
        for (int k = 0; k < NJ; k++) {
            const int j = 4 * g + 32 * k;
            if (j < d) {
                const double a0 = ra[k].x, a1 = ra[k].y, a2 = ra[k].z, a3 = ra[k].w;
                const double b0 = rb[k].x, b1 = rb[k].y, b2 = rb[k].z, b3 = rb[k].w;
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    const double2 u = *reinterpret_cast<const double2 *>(r + 128 * q + j);
                    const double2 v = *reinterpret_cast<const double2 *>(r + 128 * q + j + 2);
                    s[q][0] = __builtin_fma(a0, u.x, s[q][0]);
                    s[q][1] = __builtin_fma(a1, u.y, s[q][1]);
                    s[q][2] = __builtin_fma(a2, v.x, s[q][2]);
                    s[q][3] = __builtin_fma(a3, v.y, s[q][3]);
                    s[q + 3][0] = __builtin_fma(b0, u.x, s[q + 3][0]);
                    s[q + 3][1] = __builtin_fma(b1, u.y, s[q + 3][1]);
                    s[q + 3][2] = __builtin_fma(b2, v.x, s[q + 3][2]);
                    s[q + 3][3] = __builtin_fma(b3, v.y, s[q + 3][3]);
                }
            }
        }
        double p[6];
#pragma unroll
        for (int q = 0; q < 6; q++) {
            double w = (s[q][0] + s[q][1]) + (s[q][2] + s[q][3]);
            w = w + shfl_xor_d(w, 1);
            w = w + shfl_xor_d(w, 2);
            w = w + shfl_xor_d(w, 4);
            p[q] = w + 0.0;
        }
        if (g == 0) {
            const int64_t base = (int64_t)t * n + c.start;
            if (oka) {
                keys[base + ia] = key_of(p[0]);
                ahead[base + ia] = make_double2(p[1], p[2]);
            }
            if (okb) {
                keys[base + ib] = key_of(p[3]);
                ahead[base + ib] = make_double2(p[4], p[5]);
            }
        }
        if (t + 1 < ntree) {  // tree t + 1's directions (loaded during this tree), then t + 2's loads
            put(s_rd[(t + 1) & 1]);
            if (t + 2 < ntree) fetch(t + 2);
        }
    }
}

// ---- Alg. 2 on large segments: canonical sums over aligned power-of-two chunks

// partial canon_sum of one chunk: of p (what = 0) or of (p - mu)^2 (what = 1)
__global__ __launch_bounds__(256) void k_chunk_sum(const ChunkDesc *__restrict__ chunks, int nchunk,
                                                   const SegDesc *__restrict__ segs,
                                                   const double *__restrict__ praw, int64_t n,
                                                   const SelState *__restrict__ state, int nseg,
                                                   int what, double *__restrict__ part) {
    __shared__ double s[kChunk];
    const int t = blockIdx.y, tid = threadIdx.x;
    const ChunkDesc c = chunks[blockIdx.x];
    const SegDesc sg = segs[c.seg];
    const double mu = what ? state[(int64_t)t * nseg + c.seg].s1 / (double)sg.size : 0.0;
    for (int i = tid; i < kChunk; i += 256) {
        double v = 0.0;
        if (i < c.len) {
            double p = praw[(int64_t)t * n + c.start + i];
            if (what) {
                double dev = p - mu;
                v = __dmul_rn(dev, dev);
            } else {
                v = p;
            }
        }
        s[i] = v;
    }
    __syncthreads();
    for (int h = 1; h < kChunk; h <<= 1) {
        for (int i = 2 * h * tid; i < kChunk; i += 2 * h * 256) s[i] = s[i] + s[i + h];
        __syncthreads();
    }
    if (tid == 0) part[(int64_t)t * nchunk + blockIdx.x] = s[0];
}

// combine chunk partials of each segment by the same tree; what = 0 stores S1, what = 1
// compares S2 with the best so far (Alg. 2: strictly larger wins)
__global__ void k_seg_sum(const SegDesc *__restrict__ segs, int nseg, int nchunk,
                          double *__restrict__ part, SelState *__restrict__ state, int what, int tr) {
    const int t = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nseg) return;
    const SegDesc sg = segs[k];
    // pairwise tree over the chunk partials in place; a missing right operand is the +0.0
    // padding, and x + 0.0 == x for the non-negative-zero-free values summed here
    double *v = part + (int64_t)t * nchunk + sg.chunk0;
    for (int h = 1; h < sg.nchunk; h <<= 1)
        for (int i = 0; i + h < sg.nchunk; i += 2 * h) v[i] = v[i] + v[i + h];
    SelState *st = state + (int64_t)t * nseg + k;
    if (what == 0) {
        st->s1 = v[0];
    } else if (v[0] > st->best_s2) {
        st->best_s2 = v[0];
        st->chosen = tr;
    }
}

__global__ void k_copy_segments(const LeafDesc *__restrict__ segs, int nseg,
                                const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                int64_t n) {
    const int t = blockIdx.y;
    const LeafDesc sg = segs[blockIdx.x];
    for (int i = threadIdx.x; i < sg.size; i += blockDim.x)
        out[(int64_t)t * n + sg.off + i] = in[(int64_t)t * n + sg.off + i];
}

__global__ void k_iota(int32_t *__restrict__ perm, int64_t n) {
    const int t = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        perm[(int64_t)t * n + i] = (int32_t)i;
}

// ================================================================ leaves (neighbourhoods)

// leaf_of, leaf centroid mu (binary32 mean of the members), and the leaf-ordered, centred
// copy Xc[t][pos][0..dp) in the tile precision, with |Xc row|^2 (binary32, of the stored
// low-precision values) and |x - mu| (binary32) per position.
template <typename T>
__device__ inline T to_tile(float v);
template <>
__device__ inline float to_tile<float>(float v) { return v; }
template <>
__device__ inline __bf16 to_tile<__bf16>(float v) { return (__bf16)v; }
template <>
__device__ inline _Float16 to_tile<_Float16>(float v) { return (_Float16)v; }

template <typename T>
__global__ __launch_bounds__(256) void k_leaf_finalize(
    const float *__restrict__ X, int d, int dp, const LeafDesc *__restrict__ leaves, int nleaf,
    const int32_t *__restrict__ perm, int64_t n, int32_t *__restrict__ leaf_of,
    float *__restrict__ centroid, T *__restrict__ Xc, float2 *__restrict__ nrm, float range_max, int ids_in_lds) {
    extern __shared__ __align__(16) float s_mu[];  // dp floats, then 4 x dp partial sums, then members
    const int t = blockIdx.y, tid = threadIdx.x;
    const LeafDesc lf = leaves[blockIdx.x];
    const int m = lf.size;
    float *s_part = s_mu + dp;
    const int32_t *pp = perm + (int64_t)t * n + lf.off;
    // member ids: staged in LDS when the launch reserved room for them, else read in place
    int32_t *s_lds_id = reinterpret_cast<int32_t *>(s_part + 4 * dp);
    const int32_t *s_id = ids_in_lds ? s_lds_id : pp;
    for (int i = tid; i < m; i += 256) {
        const int id = pp[i];
        if (ids_in_lds) s_lds_id[i] = id;
        leaf_of[(int64_t)t * n + id] = lf.heap;
    }
    __syncthreads();
    // mean: wave w sums rows w, w+4, ... in order (lane j holds columns j, j+64, ...); four
    // rows are loaded before they are added, then the four partial sums are added in wave
    // order -- a fixed order, so the centroid is reproducible
    const int lane = tid & 63, wv = tid >> 6;
    for (int j0 = 0; j0 < dp; j0 += 64 * 4) {
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        int i = wv;
        for (; i + 12 < m; i += 16) {
            float v[4][4];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const float *x = X + (int64_t)s_id[i + 4 * r] * d;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int j = j0 + 64 * q + lane;
                    v[r][q] = j < d ? x[j] : 0.f;
                }
            }
#pragma unroll
            for (int r = 0; r < 4; r++)
#pragma unroll
                for (int q = 0; q < 4; q++) acc[q] += v[r][q];
        }
        for (; i < m; i += 4) {
            const float *x = X + (int64_t)s_id[i] * d;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int j = j0 + 64 * q + lane;
                acc[q] += j < d ? x[j] : 0.f;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int j = j0 + 64 * q + lane;
            if (j < dp) s_part[wv * dp + j] = acc[q];
        }
    }
    __syncthreads();
    for (int j = tid; j < dp; j += 256) {
        const float sum = ((s_part[j] + s_part[dp + j]) + s_part[2 * dp + j]) + s_part[3 * dp + j];
        const float mu = j < d ? sum / (float)m : 0.f;
        s_mu[j] = mu;
        if (j < d) centroid[((int64_t)t * nleaf + blockIdx.x) * d + j] = mu;
    }
    __syncthreads();
    // centred copy in the tile precision and its norms, two rows per wave at a time
    for (int i0 = wv; i0 < m; i0 += 8) {
        float na[2] = {0.f, 0.f}, ra[2] = {0.f, 0.f};
        bool over[2] = {false, false};
        for (int j0 = 0; j0 < dp; j0 += 64 * 4) {
            float xv[2][4];
#pragma unroll
            for (int r = 0; r < 2; r++) {
                const int i = i0 + 4 * r;
                const float *x = X + (int64_t)s_id[i < m ? i : i0] * d;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int j = j0 + 64 * q + lane;
                    xv[r][q] = j < d ? x[j] : 0.f;
                }
            }
#pragma unroll
            for (int r = 0; r < 2; r++) {
                const int i = i0 + 4 * r;
                if (i >= m) continue;
                T *out = Xc ? Xc + ((int64_t)t * n + lf.off + i) * dp : nullptr;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int j = j0 + 64 * q + lane;
                    if (j >= dp) continue;
                    const float a = j < d ? xv[r][q] - s_mu[j] : 0.f;
                    over[r] |= fabsf(a) > range_max;
                    const T qv = to_tile<T>(a);
                    if (out) out[j] = qv;
                    const float qf = (float)qv;
                    na[r] = __builtin_fmaf(qf, qf, na[r]);
                    ra[r] = __builtin_fmaf(a, a, ra[r]);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 2; r++) {
            float x = na[r], y = ra[r];
            for (int o = 32; o > 0; o >>= 1) {
                x += __shfl_xor(x, o, 64);
                y += __shfl_xor(y, o, 64);
            }
            const uint64_t ov = __ballot(over[r]);
            const int i = i0 + 4 * r;
            if (lane == 0 && i < m) nrm[(int64_t)t * n + lf.off + i] = make_float2(x, ov ? INFINITY : sqrtf(y));
        }
    }
}

// The leaf-ordered, centred copy alone, for a forest whose leaf pass did not write it: each
// element is x - mu rounded to the tile type (zero past d), from the centroid the leaf pass
// stored, so it holds exactly the values the leaf pass would have written.  One block per
// (leaf, tree); four columns per thread.
template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_leaf_copy(const float *__restrict__ X, int d, int dp,
                                                   const LeafDesc *__restrict__ leaves, int nleaf,
                                                   const int32_t *__restrict__ perm, int64_t n,
                                                   const float *__restrict__ centroid, T *__restrict__ Xc) {
    const int t = blockIdx.y;
    const LeafDesc lf = leaves[blockIdx.x];
    const float *mu = centroid + ((int64_t)t * nleaf + blockIdx.x) * d;
    const int32_t *pp = perm + (int64_t)t * n + lf.off;
    const int q = dp >> 2;  // four-column groups per row (dp is a multiple of 8)
    for (int v = threadIdx.x; v < lf.size * q; v += 256) {
        const int i = v / q, c = 4 * (v - i * q);
        const float *x = X + (int64_t)pp[i] * d;
        float a[4];
        if (VEC && c < d) {  // d % 4 == 0: the four columns are all below d
            const float4 xv = *reinterpret_cast<const float4 *>(x + c);
            const float4 u = *reinterpret_cast<const float4 *>(mu + c);
            a[0] = xv.x - u.x;
            a[1] = xv.y - u.y;
            a[2] = xv.z - u.z;
            a[3] = xv.w - u.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; e++) a[e] = c + e < d ? x[c + e] - mu[c + e] : 0.f;
        }
        T qv[4];
#pragma unroll
        for (int e = 0; e < 4; e++) qv[e] = to_tile<T>(a[e]);
        T *out = Xc + ((int64_t)t * n + lf.off + i) * dp + c;
        if constexpr (sizeof(T) == 4) {
            *reinterpret_cast<float4 *>(out) = make_float4(qv[0], qv[1], qv[2], qv[3]);
        } else {
            uint2 w;
            __builtin_memcpy(&w, qv, sizeof(w));
            *reinterpret_cast<uint2 *>(out) = w;
        }
    }
}

// The leaf statistics without the copy, for forests whose all-points search centres the rows
// itself as it stages them (leaves of at most 256 points): leaf_of, the centroid mu (binary32
// mean, a fixed order: each of 32 row groups sums its rows in order, then the groups in
// order) and per position |tile(x - mu)|^2 of the tile-type values and |x - mu| (+inf past
// the tile type's range).  A copy made later from this centroid holds exactly the values
// these norms describe.  One block of 1024 threads per (leaf, tree): 32 lanes per row, four
// columns each per step of 128 columns, and the block's 32 row groups hold all of the leaf's
// rows of a step in registers, so X is read once.
// NT threads hold leaves of up to NT / 4 points (1024 threads for 256-point leaves, 256 for
// leaves of at most 64, where a larger block would leave most of its rows empty).
template <typename T, bool VEC, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8))) void k_leaf_stats(const float *__restrict__ X, int d, int dp,
                                                     const LeafDesc *__restrict__ leaves, int nleaf,
                                                     const int32_t *__restrict__ perm, int64_t n,
                                                     int32_t *__restrict__ leaf_of, float *__restrict__ centroid,
                                                     float2 *__restrict__ nrm, float range_max) {
    constexpr int ML = NT / 4, RG = NT / 32, RK = ML / RG;  // rows, row groups, rows per group
    __shared__ __align__(16) float s_part[RG][128];
    __shared__ __align__(16) float s_mu[128];
    __shared__ int32_t s_id[ML];
    __shared__ float s_na[ML], s_ra[ML];  // the rows' norms, summed over the steps in order
    const int t = blockIdx.y, tid = threadIdx.x, lane = tid & 63;
    const LeafDesc lf = leaves[blockIdx.x];
    const int m = lf.size;
    const int32_t *pp = perm + (int64_t)t * n + lf.off;
    for (int i = tid; i < m; i += NT) {
        const int id = pp[i];
        s_id[i] = id;
        leaf_of[(int64_t)t * n + id] = lf.heap;
        s_na[i] = 0.f;
        s_ra[i] = 0.f;
    }
    __syncthreads();
    const int l32 = lane & 31, g = tid >> 5;  // rows g, g + RG, ...
    for (int cb = 0; cb < dp; cb += 128) {
        const int j = cb + 4 * l32;
        float4 x[RK];
#pragma unroll
        for (int k = 0; k < RK; k++) {  // every row of the step in flight at once
            const int r = g + RG * k;
            x[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < m) {
                const float *xr = X + (int64_t)s_id[r] * d;
                if (VEC) {
                    if (j < d) x[k] = *reinterpret_cast<const float4 *>(xr + j);
                } else {
                    x[k].x = j < d ? xr[j] : 0.f;
                    x[k].y = j + 1 < d ? xr[j + 1] : 0.f;
                    x[k].z = j + 2 < d ? xr[j + 2] : 0.f;
                    x[k].w = j + 3 < d ? xr[j + 3] : 0.f;
                }
            }
        }
        float4 cs = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int k = 0; k < RK; k++) {
            if (g + RG * k < m) {
                cs.x += x[k].x;
                cs.y += x[k].y;
                cs.z += x[k].z;
                cs.w += x[k].w;
            }
        }
        *reinterpret_cast<float4 *>(&s_part[g][4 * l32]) = cs;
        __syncthreads();
        if (tid < 128) {
            float v = 0.f;
            for (int q = 0; q < RG; q++) v += s_part[q][tid];
            const int jj = cb + tid;
            const float mu = jj < d ? v / (float)m : 0.f;
            s_mu[tid] = mu;
            if (jj < d) centroid[((int64_t)t * nleaf + blockIdx.x) * d + jj] = mu;
        }
        __syncthreads();
        const float4 u = *reinterpret_cast<const float4 *>(&s_mu[4 * l32]);
#pragma unroll
        for (int k = 0; k < RK; k++) {  // the step's share of each row's norms (past dp: zero)
            const float a[4] = {j < d ? x[k].x - u.x : 0.f, j + 1 < d ? x[k].y - u.y : 0.f,
                                j + 2 < d ? x[k].z - u.z : 0.f, j + 3 < d ? x[k].w - u.w : 0.f};
            float na = 0.f, ra = 0.f;
            bool over = false;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                over |= fabsf(a[e]) > range_max;
                const float qf = (float)to_tile<T>(a[e]);
                na = __builtin_fmaf(qf, qf, na);
                ra = __builtin_fmaf(a[e], a[e], ra);
            }
            for (int o = 1; o < 32; o <<= 1) {
                na += __shfl_xor(na, o, 64);
                ra += __shfl_xor(ra, o, 64);
            }
            const bool ov = ((__ballot(over) >> (lane & 32)) & 0xffffffffull) != 0;
            const int r = g + RG * k;
            if (l32 == 0 && r < m) {
                s_na[r] += na;
                s_ra[r] = ov ? INFINITY : s_ra[r] + ra;
            }
        }
        __syncthreads();  // s_part and s_mu are rewritten by the next step
    }
    for (int r = tid; r < m; r += NT) nrm[(int64_t)t * n + lf.off + r] = make_float2(s_na[r], sqrtf(s_ra[r]));
}

template <typename T>
static void leaf_stats(hipStream_t s, bool vec, const float *X, int d, int dp, const LeafDesc *leaves, int nleaf,
                       int ntree, const int32_t *perm, int64_t n, int32_t *leaf_of, float *centroid, float2 *nrm,
                       float range_max, int max_leaf) {
    const dim3 grid(nleaf, ntree);
    if (max_leaf <= 64) {
        if (vec)
            hipLaunchKernelGGL((k_leaf_stats<T, true, 256>), grid, dim3(256), 0, s, X, d, dp, leaves, nleaf, perm, n,
                               leaf_of, centroid, nrm, range_max);
        else
            hipLaunchKernelGGL((k_leaf_stats<T, false, 256>), grid, dim3(256), 0, s, X, d, dp, leaves, nleaf, perm, n,
                               leaf_of, centroid, nrm, range_max);
    } else {
        if (vec)
            hipLaunchKernelGGL((k_leaf_stats<T, true, 1024>), grid, dim3(1024), 0, s, X, d, dp, leaves, nleaf, perm, n,
                               leaf_of, centroid, nrm, range_max);
        else
            hipLaunchKernelGGL((k_leaf_stats<T, false, 1024>), grid, dim3(1024), 0, s, X, d, dp, leaves, nleaf, perm, n,
                               leaf_of, centroid, nrm, range_max);
    }
    launch_check(s, "k_leaf_stats");
}

// ================================================================ launchers

void launch_leaf_stats(hipStream_t s, int prec, const float *X, int d, int dp, const LeafDesc *leaves, int nleaf,
                       int ntree, const int32_t *perm, int64_t n, int32_t *leaf_of, float *centroid, float2 *nrm,
                       int max_leaf) {
    if (nleaf <= 0 || ntree <= 0 || max_leaf > 256) return;  // the caller runs the full leaf pass instead
    const bool vec = (d % 4) == 0;
    if (prec == RPF_DIST_BF16)
        leaf_stats<__bf16>(s, vec, X, d, dp, leaves, nleaf, ntree, perm, n, leaf_of, centroid, nrm, 3.0e38f, max_leaf);
    else if (prec == RPF_DIST_FP16)
        leaf_stats<_Float16>(s, vec, X, d, dp, leaves, nleaf, ntree, perm, n, leaf_of, centroid, nrm, 60000.f, max_leaf);
    else
        leaf_stats<float>(s, vec, X, d, dp, leaves, nleaf, ntree, perm, n, leaf_of, centroid, nrm, 3.0e38f, max_leaf);
}

template <typename T>
static void leaf_copy(hipStream_t s, bool vec, const float *X, int d, int dp, const LeafDesc *leaves, int nleaf,
                      int ntree, const int32_t *perm, int64_t n, const float *centroid, void *Xc) {
    const dim3 grid(nleaf, ntree);
    if (vec)
        hipLaunchKernelGGL((k_leaf_copy<T, true>), grid, dim3(256), 0, s, X, d, dp, leaves, nleaf, perm, n, centroid,
                           (T *)Xc);
    else
        hipLaunchKernelGGL((k_leaf_copy<T, false>), grid, dim3(256), 0, s, X, d, dp, leaves, nleaf, perm, n, centroid,
                           (T *)Xc);
    launch_check(s, "k_leaf_copy");
}

void launch_leaf_copy(hipStream_t s, int prec, const float *X, int d, int dp, const LeafDesc *leaves, int nleaf,
                      int ntree, const int32_t *perm, int64_t n, const float *centroid, void *Xc) {
    if (nleaf <= 0 || ntree <= 0) return;
    const bool vec = (d % 4) == 0;
    if (prec == RPF_DIST_BF16)
        leaf_copy<__bf16>(s, vec, X, d, dp, leaves, nleaf, ntree, perm, n, centroid, Xc);
    else if (prec == RPF_DIST_FP16)
        leaf_copy<_Float16>(s, vec, X, d, dp, leaves, nleaf, ntree, perm, n, centroid, Xc);
    else
        leaf_copy<float>(s, vec, X, d, dp, leaves, nleaf, ntree, perm, n, centroid, Xc);
}

size_t level_small_lds(int max_m, int d, int n_try) {
    size_t lds = ((((4 * (size_t)max_m + 15) & ~(size_t)15) + 8 * (size_t)max_m + 15) & ~(size_t)15) +
                 3 * 8 * (size_t)((d + 3) & ~3) + 4 * (256 + 16);
    lds = (lds + 7) & ~(size_t)7;
    if (n_try > 1) {
        int P2 = 1;
        while (P2 < max_m) P2 <<= 1;
        lds += 8 * (size_t)max_m + 8 * (size_t)P2;
    }
    return lds;
}

void launch_level_small(hipStream_t s, bool vec, const float *X, int d, const float *R, int64_t H,
                        int n_try, const SegDesc *segs, int nseg, int max_m, int T,
                        const int32_t *pin, int32_t *pout, int64_t n, double *split,
                        int32_t *split_idx, int32_t *chosen, int32_t *err, const LevelLink &lk) {
    if (!lk.look && lk.keys_in && n_try == 1 && max_m <= kWaveSeg) {  // fed level of small segments
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3((nseg + 3) / 4, T), dim3(256), 0, s, segs, nseg, pin, pout, n, H, split,
                               split_idx, chosen, err, lk.keys_in);
        };
        if (max_m <= 512) go(k_level_fed_wave<8>);
        else go(k_level_fed_wave<16>);
        launch_check(s, "k_level_fed_wave");
        return;
    }
    const size_t lds = level_small_lds(max_m, d, n_try);
    dim3 grid(nseg, T);
    auto go = [&](auto kern) {
        hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, X, d, R, H, n_try, segs, pin, pout, n, split, split_idx,
                           chosen, err, lk.look, lk.ahead, lk.keys_next, lk.keys_in, lk.xq, lk.dq);
    };
    const bool q8 = lk.xq && n_try == 1;  // (several tries project through the binary32 rows)
    if (lk.look) {
        if (q8 && vec) go(k_level_small<true, true, true>);
        else if (q8) go(k_level_small<false, true, true>);
        else if (vec) go(k_level_small<true, true>);
        else go(k_level_small<false, true>);
    } else {
        if (q8 && vec) go(k_level_small<true, false, true>);
        else if (q8) go(k_level_small<false, false, true>);
        else if (vec) go(k_level_small<true, false>);
        else go(k_level_small<false, false>);
    }
    launch_check(s, "k_level_small");
}

size_t cand_bytes() { return sizeof(Cand); }

template <bool VEC>
static void proj_chunks(hipStream_t s, dim3 gc, const float *X, int d, const float *R, int64_t H, int n_try,
                        const SegDesc *segs, const ChunkDesc *chunks, const int32_t *pin, int64_t n,
                        const LargeBufs &b, int nseg, int mode, int tr, const LevelLink &lk) {
    const size_t ds = (size_t)((d + 3) & ~3);
    const size_t lds = d > 1024 ? 0 : lk.look ? 3 * ds * sizeof(double) : ds * sizeof(float);
    const bool q8 = lk.xq != nullptr;
    if (lk.look && q8)
        hipLaunchKernelGGL((k_proj_chunks<VEC, true, true>), gc, dim3(256), lds, s, X, d, R, H, n_try, segs, chunks,
                           pin, n, b.state, nseg, mode, tr, b.keys, b.praw, b.hist, lk.look, lk.ahead, lk.xq, lk.dq);
    else if (lk.look)
        hipLaunchKernelGGL((k_proj_chunks<VEC, true>), gc, dim3(256), lds, s, X, d, R, H, n_try, segs, chunks, pin, n,
                           b.state, nseg, mode, tr, b.keys, b.praw, b.hist, lk.look, lk.ahead, lk.xq, lk.dq);
    else if (q8)
        hipLaunchKernelGGL((k_proj_chunks<VEC, false, true>), gc, dim3(256), lds, s, X, d, R, H, n_try, segs, chunks,
                           pin, n, b.state, nseg, mode, tr, b.keys, b.praw, b.hist, lk.look, lk.ahead, lk.xq, lk.dq);
    else
        hipLaunchKernelGGL((k_proj_chunks<VEC, false>), gc, dim3(256), lds, s, X, d, R, H, n_try, segs, chunks, pin, n,
                           b.state, nseg, mode, tr, b.keys, b.praw, b.hist, lk.look, lk.ahead, lk.xq, lk.dq);
    launch_check(s, "k_proj_chunks");
}

void launch_level_large(hipStream_t s, bool vec, const float *X, int d, const float *R, int64_t H,
                        int n_try, const SegDesc *segs, int nseg, const ChunkDesc *chunks, int nchunk,
                        int T, const int32_t *pin, int32_t *pout, int64_t n, double *split,
                        int32_t *split_idx, int32_t *chosen, int32_t *err, const LargeBufs &b0,
                        double proj_bytes, const LevelLink &lk) {
    dim3 gs(nseg, T), gc(nchunk, T);
    LargeBufs b = b0;
    if (lk.keys_in) {  // fed level: keys and digit-0 histograms come from the level above
        b.keys = const_cast<uint64_t *>(lk.keys_in);
        b.hist = lk.hist_in;
    }
    hipLaunchKernelGGL(k_sel_init, dim3((nseg * T + 255) / 256), dim3(256), 0, s, segs, nseg, T, b.state);
    launch_check(s, "k_sel_init");
    // fill kernels, not memsets: the level may be recorded in a graph
    if (!lk.keys_in) fill_u32(b.hist, (int64_t)kDigitBins * nseg * T, 0, s);
    if (lk.hist_next) fill_u32(lk.hist_next, (int64_t)kDigitBins * lk.nseg_next * T, 0, s);
    fill_u32(b.cand_cnt, (int64_t)nseg * T, 0, s);
    launch_check(s, "select memsets");
    if (n_try > 1) {
        for (int tr = 0; tr < n_try; tr++) {
            {
                ProfScope ps(s, "proj_try", proj_bytes, 0);
                if (vec) proj_chunks<true>(s, gc, X, d, R, H, n_try, segs, chunks, pin, n, b, nseg, 1, tr, LevelLink{});
                else proj_chunks<false>(s, gc, X, d, R, H, n_try, segs, chunks, pin, n, b, nseg, 1, tr, LevelLink{});
            }
            for (int what = 0; what < 2; what++) {
                hipLaunchKernelGGL(k_chunk_sum, gc, dim3(256), 0, s, chunks, nchunk, segs, b.praw, n, b.state,
                                   nseg, what, b.part);
                launch_check(s, "k_chunk_sum");
                hipLaunchKernelGGL(k_seg_sum, dim3((nseg + 63) / 64, T), dim3(64), 0, s, segs, nseg, nchunk, b.part,
                                   b.state, what, tr);
                launch_check(s, "k_seg_sum");
            }
        }
    }
    if (lk.roots) {  // every tree's root projections from one read of X, then the first digit
        ProfScope ps(s, "proj_roots", proj_bytes, 0);
        hipLaunchKernelGGL(k_proj_root, dim3(nchunk, kChunk / 64), dim3(256), 0, s, X, d, R, H, T, segs, chunks,
                           lk.look, n, b.keys, lk.ahead);
        launch_check(s, "k_proj_root");
        hipLaunchKernelGGL(k_sel_pass, gc, dim3(256), 0, s, chunks, b.keys, pin, n, b.state, nseg, b.hist, b.cand,
                           b.cand_cnt, b.lcount, nchunk);
        launch_check(s, "k_sel_pass");
    } else if (!lk.keys_in) {
        ProfScope ps(s, lk.look ? "proj_chunks_x3" : "proj_chunks", proj_bytes, 0);
        if (vec) proj_chunks<true>(s, gc, X, d, R, H, n_try, segs, chunks, pin, n, b, nseg, 0, 0, lk);
        else proj_chunks<false>(s, gc, X, d, R, H, n_try, segs, chunks, pin, n, b, nseg, 0, 0, lk);
    }
    {
        ProfScope ps(s, "select_passes", 0, 0);
        for (int j = 0; j < kNumDigits; j++) {
            hipLaunchKernelGGL(k_sel_scan, gs, dim3(256), 0, s, b.state, nseg, b.hist);
            launch_check(s, "k_sel_scan");
            if (j + 1 < kNumDigits) {
                hipLaunchKernelGGL(k_sel_pass, gc, dim3(256), 0, s, chunks, b.keys, pin, n, b.state, nseg, b.hist,
                                   b.cand, b.cand_cnt, b.lcount, nchunk);
                launch_check(s, "k_sel_pass");
            }
        }
        hipLaunchKernelGGL(k_sel_finish, gs, dim3(256), 0, s, segs, b.state, nseg, b.cand, b.cand_cnt, H, split,
                           split_idx, chosen, err, b.lcount, nchunk);
        launch_check(s, "k_sel_finish");
    }
    {
        ProfScope ps(s, "partition", 0, 0);
        hipLaunchKernelGGL(k_part_count, gc, dim3(256), 0, s, chunks, nchunk, b.keys, pin, n, b.state, nseg,
                           b.lcount);
        launch_check(s, "k_part_count");
        hipLaunchKernelGGL(k_part_scan, dim3((nseg + 63) / 64, T), dim3(64), 0, s, segs, chunks, nchunk, nseg,
                           b.lcount, err);
        launch_check(s, "k_part_scan");
        hipLaunchKernelGGL(k_part_scatter, gc, dim3(256), 0, s, segs, chunks, nchunk, b.keys, pin, pout, n, b.state,
                           nseg, b.lcount, lk.look, lk.ahead, lk.keys_next, lk.hist_next, lk.nseg_next);
        launch_check(s, "k_part_scatter");
    }
}

void launch_copy_segments(hipStream_t s, const LeafDesc *segs, int nseg, int T, const int32_t *in,
                          int32_t *out, int64_t n) {
    if (nseg == 0) return;
    hipLaunchKernelGGL(k_copy_segments, dim3(nseg, T), dim3(256), 0, s, segs, nseg, in, out, n);
    launch_check(s, "k_copy_segments");
}

void launch_iota(hipStream_t s, int32_t *perm, int64_t n, int T) {
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_iota, dim3(blocks, T), dim3(256), 0, s, perm, n);
    launch_check(s, "k_iota");
}

// Row stride of a leaf staged in LDS: an odd number of 16-byte chunks, so that the eight rows
// a wave centres at once (one per group of eight lanes) fall in different bank groups.
__host__ __device__ inline int leaf_row_stride(int d) {
    const int s = (d + 3) & ~3;
    return ((s >> 2) & 1) ? s : s + 4;
}

// Mean and centred copy of one leaf whose m rows (stride ds floats) are in LDS, by a block of
// 512 threads: the centroid is a fixed-order sum (R row classes per column, then the classes
// in order), so it is reproducible; then eight lanes per row write the centred row, four
// consecutive columns at a time, and its two norms.
template <typename T>
__device__ __attribute__((always_inline)) inline void leaf_centre_staged(const float *s_rows, float *s_mu, float *s_part, int m, int d, int ds,
                                          int dp, int t, int leaf, int nleaf, const LeafDesc &lf, int64_t n,
                                          float *__restrict__ centroid, T *__restrict__ Xc,
                                          float2 *__restrict__ nrm, float range_max) {
    constexpr int NT = 512, NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (ds <= NT) {  // R row classes per column: class g sums rows g, g+R, ... (two chains)
        const int R = NT / ds, g = tid / ds, j = tid - g * ds;
        if (g < R) {
            float a0 = 0.f, a1 = 0.f;
            if (j < d) {
                int i = g;
                for (; i + R < m; i += 2 * R) {
                    a0 += s_rows[(size_t)i * ds + j];
                    a1 += s_rows[(size_t)(i + R) * ds + j];
                }
                if (i < m) a0 += s_rows[(size_t)i * ds + j];
            }
            s_part[tid] = a0 + a1;
        }
        __syncthreads();
        if (tid < ds) {
            float sum = 0.f;
            for (int c = 0; c < R; c++) sum += s_part[c * ds + tid];
            const float mu = tid < d ? sum / (float)m : 0.f;
            s_mu[tid] = mu;
            if (tid < d) centroid[((int64_t)t * nleaf + leaf) * d + tid] = mu;
        }
    } else {
        for (int j = tid; j < ds; j += NT) {
            float acc = 0.f;
            if (j < d)
                for (int i = 0; i < m; i++) acc += s_rows[(size_t)i * ds + j];
            const float mu = j < d ? acc / (float)m : 0.f;
            s_mu[j] = mu;
            if (j < d) centroid[((int64_t)t * nleaf + leaf) * d + j] = mu;
        }
    }
    __syncthreads();
    // centred copy and norms: eight lanes per row, each lane four consecutive columns at a
    // time, so a wave has eight rows in flight and reduces each over three shuffle steps
    const int sub = lane & 7, grp = lane >> 3;
    for (int i0 = wv * 8; i0 < m; i0 += NW * 8) {
        const int i = i0 + grp;
        const bool live = i < m;
        const int ir = live ? i : m - 1;
        T *out = Xc ? Xc + ((int64_t)t * n + lf.off + ir) * dp : nullptr;
        float na = 0.f, ra = 0.f;
        bool over = false;
        for (int c = 4 * sub; c < dp; c += 32) {
            float a[4];
            if (c < ds) {
                const float4 x = *reinterpret_cast<const float4 *>(s_rows + (size_t)ir * ds + c);
                const float4 u = *reinterpret_cast<const float4 *>(s_mu + c);
                a[0] = c + 0 < d ? x.x - u.x : 0.f;
                a[1] = c + 1 < d ? x.y - u.y : 0.f;
                a[2] = c + 2 < d ? x.z - u.z : 0.f;
                a[3] = c + 3 < d ? x.w - u.w : 0.f;
            } else {
                a[0] = a[1] = a[2] = a[3] = 0.f;
            }
            T qv[4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                over |= fabsf(a[e]) > range_max;
                qv[e] = to_tile<T>(a[e]);
                const float qf = (float)qv[e];
                na = __builtin_fmaf(qf, qf, na);
                ra = __builtin_fmaf(a[e], a[e], ra);
            }
            if (live && out) {
                if constexpr (sizeof(T) == 4) {
                    *reinterpret_cast<float4 *>(out + c) = make_float4(qv[0], qv[1], qv[2], qv[3]);
                } else {
                    uint2 w;
                    __builtin_memcpy(&w, qv, sizeof(w));
                    *reinterpret_cast<uint2 *>(out + c) = w;
                }
            }
        }
        for (int o = 4; o > 0; o >>= 1) {
            na += __shfl_xor(na, o, 64);
            ra += __shfl_xor(ra, o, 64);
        }
        const uint64_t ov = (__ballot(over) >> (8 * grp)) & 0xffu;
        if (live && sub == 0) nrm[(int64_t)t * n + lf.off + i] = make_float2(na, ov ? INFINITY : sqrtf(ra));
    }
}

// The same leaf pass with the leaf's rows staged in LDS: X is read once (the two-pass
// kernel reads it once for the mean and again to centre).  One block per (leaf, tree); the
// leaf (up to ~130 KB) is loaded with every load of a thread in flight at once, since one
// block holds the CU's LDS.  The centroid is a fixed-order sum (R row classes per column,
// then the classes in order), so it is reproducible.
template <typename T, bool VEC>
__global__ __launch_bounds__(512) void k_leaf_staged(
    const float *__restrict__ X, int d, int dp, const LeafDesc *__restrict__ leaves, int nleaf,
    const int32_t *__restrict__ perm, int64_t n, int32_t *__restrict__ leaf_of,
    float *__restrict__ centroid, T *__restrict__ Xc, float2 *__restrict__ nrm, float range_max) {
    extern __shared__ __align__(16) float s_rows[];  // m rows of ds floats, centroid (ds), member ids (m)
    __shared__ float s_part[512];
    const int t = blockIdx.y, tid = threadIdx.x;
    constexpr int NT = 512, KV = 16;
    const LeafDesc lf = leaves[blockIdx.x];
    const int m = lf.size;
    const int ds = leaf_row_stride(d);
    float *s_mu = s_rows + (size_t)m * ds;
    int32_t *s_id = reinterpret_cast<int32_t *>(s_mu + ds);
    const int32_t *pp = perm + (int64_t)t * n + lf.off;
    for (int i = tid; i < m; i += NT) {
        const int id = pp[i];
        s_id[i] = id;
        leaf_of[(int64_t)t * n + id] = lf.heap;
    }
    __syncthreads();
    if constexpr (VEC) {  // 16-byte loads, KV of them in flight per thread
        const int q = d >> 2, tot = m * q;
        for (int v0 = 0; v0 < tot; v0 += NT * KV) {
            float4 r[KV];
#pragma unroll
            for (int k = 0; k < KV; k++) {  // past the end: reload the last element, not stored
                const int v = min(v0 + k * NT + tid, tot - 1);
                const int i = v / q, c = v - i * q;
                r[k] = reinterpret_cast<const float4 *>(X + (int64_t)s_id[i] * d)[c];
            }
#pragma unroll
            for (int k = 0; k < KV; k++) {
                const int v = v0 + k * NT + tid;
                const int i = v / q, c = v - i * q;
                if (v < tot) reinterpret_cast<float4 *>(s_rows + (size_t)i * ds)[c] = r[k];
            }
        }
    } else {
        const int tot = m * d;
        for (int v0 = 0; v0 < tot; v0 += NT * KV) {
            float r[KV];
#pragma unroll
            for (int k = 0; k < KV; k++) {
                const int v = min(v0 + k * NT + tid, tot - 1);
                const int i = v / d, j = v - i * d;
                r[k] = X[(int64_t)s_id[i] * d + j];
            }
#pragma unroll
            for (int k = 0; k < KV; k++) {
                const int v = v0 + k * NT + tid;
                const int i = v / d, j = v - i * d;
                if (v < tot) s_rows[(size_t)i * ds + j] = r[k];
            }
        }
    }
    __syncthreads();
    leaf_centre_staged<T>(s_rows, s_mu, s_part, m, d, ds, dp, t, blockIdx.x, nleaf, lf, n, centroid, Xc, nrm,
                          range_max);
}

// The staged leaf pass as a software pipeline: each block (one per CU: a leaf fills its LDS)
// walks the (tree, leaf) items w = blockIdx.x, + gridDim.x, ...; while it centres and writes
// item w from LDS, the rows of the next item are in flight into registers and the member ids
// of the one after are in flight too.  Needs d % 4 == 0, every leaf at most 512 members and
// at most 512 * 16 row quarters.
template <typename T>
__global__ __launch_bounds__(512) void k_leaf_pipe(
    const float *__restrict__ X, int d, int dp, const LeafDesc *__restrict__ leaves, int nleaf, int ntree,
    const int32_t *__restrict__ perm, int64_t n, int32_t *__restrict__ leaf_of,
    float *__restrict__ centroid, T *__restrict__ Xc, float2 *__restrict__ nrm, float range_max, int max_leaf) {
    extern __shared__ __align__(16) float s_rows[];  // max_leaf rows of S floats, centroid (S), ids (max_leaf)
    __shared__ float s_part[512];
    constexpr int NT = 512, KV = 16;
    const int tid = threadIdx.x, q = d >> 2, G = gridDim.x;
    const int items = nleaf * ntree;
    const int S = leaf_row_stride(d);
    float *s_mu = s_rows + (size_t)max_leaf * S;
    int32_t *s_id = reinterpret_cast<int32_t *>(s_mu + S);
    float r0[KV], r1[KV], r2[KV], r3[KV];  // the next item's row quarters (scalars stay in registers)
    // item w -> tree w / nleaf, leaf w % nleaf: neighbouring blocks take neighbouring leaves
    auto id_of = [&](int w) -> int32_t {  // member tid of item w (0 past its end)
        if (w >= items) return 0;
        const int t = w / nleaf;
        const LeafDesc lf = leaves[w - t * nleaf];
        return tid < lf.size ? perm[(int64_t)t * n + lf.off + tid] : 0;
    };
    auto stage_ids = [&](int w, int32_t id) {  // ids of item w into LDS, and its leaf_of entries
        if (w >= items) return;
        const int t = w / nleaf;
        const LeafDesc lf = leaves[w - t * nleaf];
        if (tid < lf.size) {
            s_id[tid] = id;
            leaf_of[(int64_t)t * n + id] = lf.heap;
        }
    };
    // rows of item w into registers (its ids in LDS); past the end of the leaf the last element
    // is loaded again and not stored
#define RPF_ISSUE_ROWS(W)                                                                       \
    {                                                                                           \
        const bool ok_ = (W) < items;  /* past the last item: row 0, never stored */            \
        const int tw_ = ok_ ? (W) / nleaf : 0;                                                  \
        const int tot_ = ok_ ? leaves[(W) - tw_ * nleaf].size * q : 1;                          \
        _Pragma("unroll") for (int k = 0; k < KV; k++) {                                        \
            const int v = min(k * NT + tid, tot_ - 1);                                          \
            const int i = v / q, c = v - i * q;                                                 \
            const int64_t row = ok_ ? s_id[i] : 0;                                              \
            const float4 x_ = reinterpret_cast<const float4 *>(X + row * d)[c];                 \
            r0[k] = x_.x; r1[k] = x_.y; r2[k] = x_.z; r3[k] = x_.w;                             \
        }                                                                                       \
    }
    int w = blockIdx.x;
    stage_ids(w, id_of(w));
    __syncthreads();
    RPF_ISSUE_ROWS(w)
    int32_t idn = id_of(w + G);
    for (; w < items; w += G) {
        const int t = w / nleaf, leaf = w - t * nleaf;
        const LeafDesc lf = leaves[leaf];
        const int m = lf.size, tot = m * q;
        __syncthreads();  // the previous item is done with s_rows and s_id
#pragma unroll
        for (int k = 0; k < KV; k++) {
            const int v = k * NT + tid;
            const int i = v / q, c = v - i * q;
            if (v < tot) reinterpret_cast<float4 *>(s_rows + (size_t)i * S)[c] = make_float4(r0[k], r1[k], r2[k], r3[k]);
        }
        stage_ids(w + G, idn);
        __syncthreads();
        RPF_ISSUE_ROWS(w + G)  // in flight while item w is centred
        idn = id_of(w + 2 * G);
        leaf_centre_staged<T>(s_rows, s_mu, s_part, m, d, S, dp, t, leaf, nleaf, lf, n, centroid, Xc, nrm,
                              range_max);
    }
#undef RPF_ISSUE_ROWS
}

size_t leaf_staged_lds(int d, int max_leaf) {  // dynamic part; 2 KB of static LDS come on top
    return sizeof(float) * (size_t)leaf_row_stride(d) * ((size_t)max_leaf + 1) + sizeof(int32_t) * (size_t)max_leaf;
}

template <typename T>
static void leaf_staged(hipStream_t s, dim3 grid, size_t lds, bool vec, const float *X, int d, int dp,
                        const LeafDesc *leaves, int nleaf, const int32_t *perm, int64_t n, int32_t *leaf_of,
                        float *centroid, void *Xc, float2 *nrm, float range_max) {
    if (vec) {
        hipFuncSetAttribute((const void *)k_leaf_staged<T, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_leaf_staged<T, true>), grid, dim3(512), lds, s, X, d, dp, leaves, nleaf, perm, n, leaf_of,
                           centroid, (T *)Xc, nrm, range_max);
    } else {
        hipFuncSetAttribute((const void *)k_leaf_staged<T, false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_leaf_staged<T, false>), grid, dim3(512), lds, s, X, d, dp, leaves, nleaf, perm, n,
                           leaf_of, centroid, (T *)Xc, nrm, range_max);
    }
    launch_check(s, "k_leaf_staged");
}

template <typename T>
static void leaf_pipe(hipStream_t s, size_t lds, const float *X, int d, int dp, const LeafDesc *leaves, int nleaf,
                      int ntree, const int32_t *perm, int64_t n, int32_t *leaf_of, float *centroid, void *Xc,
                      float2 *nrm, float range_max, int max_leaf) {
    hipFuncSetAttribute((const void *)k_leaf_pipe<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int dev = 0, cus = 0, per = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_leaf_pipe<T>, 512, lds);
    const int64_t items = (int64_t)nleaf * ntree;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(items, (int64_t)std::max(cus, 1) * std::max(per, 1)));
    hipLaunchKernelGGL(k_leaf_pipe<T>, dim3(grid), dim3(512), lds, s, X, d, dp, leaves, nleaf, ntree, perm, n, leaf_of,
                       centroid, (T *)Xc, nrm, range_max, max_leaf);
    launch_check(s, "k_leaf_pipe");
}

template <typename T>
static void leaf_finalize(hipStream_t s, dim3 grid, size_t lds, const float *X, int d, int dp,
                          const LeafDesc *leaves, int nleaf, const int32_t *perm, int64_t n, int32_t *leaf_of,
                          float *centroid, void *Xc, float2 *nrm, float range_max, int ids_in_lds) {
    hipFuncSetAttribute((const void *)k_leaf_finalize<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_leaf_finalize<T>, grid, dim3(256), lds, s, X, d, dp, leaves, nleaf, perm, n, leaf_of,
                       centroid, (T *)Xc, nrm, range_max, ids_in_lds);
    launch_check(s, "k_leaf_finalize");
}

size_t leaf_finalize_lds(int dp, int max_leaf, bool ids) {
    return sizeof(float) * 5 * (size_t)dp + (ids ? sizeof(int32_t) * (size_t)max_leaf : 0);
}

void launch_leaf_finalize(hipStream_t s, int prec, const float *X, int d, int dp, const LeafDesc *leaves,
                          int nleaf, int T, const int32_t *perm, int64_t n, int32_t *leaf_of, float *centroid,
                          void *Xc, float2 *nrm, int max_leaf, int lds_limit) {
    dim3 grid(nleaf, T);
    const size_t piped = sizeof(float) * (size_t)leaf_row_stride(d) * ((size_t)max_leaf + 1) +
                         sizeof(int32_t) * (size_t)max_leaf;
    if (d % 4 == 0 && max_leaf <= 512 && max_leaf * (d / 4) <= 512 * 16 && piped + 2048 <= (size_t)lds_limit &&
        (int64_t)nleaf * T < (1ll << 31)) {  // a leaf fits a block's registers and LDS: pipelined
        if (prec == RPF_DIST_BF16)
            leaf_pipe<__bf16>(s, piped, X, d, dp, leaves, nleaf, T, perm, n, leaf_of, centroid, Xc, nrm, 3.0e38f,
                              max_leaf);
        else if (prec == RPF_DIST_FP16)
            leaf_pipe<_Float16>(s, piped, X, d, dp, leaves, nleaf, T, perm, n, leaf_of, centroid, Xc, nrm, 60000.f,
                                max_leaf);
        else
            leaf_pipe<float>(s, piped, X, d, dp, leaves, nleaf, T, perm, n, leaf_of, centroid, Xc, nrm, 3.0e38f,
                             max_leaf);
        return;
    }
    const size_t staged = leaf_staged_lds(d, max_leaf);
    if (staged + 2048 <= (size_t)lds_limit) {  // the leaf's rows fit in LDS: read X once
        const bool vec = (d % 4) == 0;
        if (prec == RPF_DIST_BF16)
            leaf_staged<__bf16>(s, grid, staged, vec, X, d, dp, leaves, nleaf, perm, n, leaf_of, centroid, Xc, nrm, 3.0e38f);
        else if (prec == RPF_DIST_FP16)
            leaf_staged<_Float16>(s, grid, staged, vec, X, d, dp, leaves, nleaf, perm, n, leaf_of, centroid, Xc, nrm,
                                  60000.f);
        else
            leaf_staged<float>(s, grid, staged, vec, X, d, dp, leaves, nleaf, perm, n, leaf_of, centroid, Xc, nrm, 3.0e38f);
        return;
    }
    const int ids = leaf_finalize_lds(dp, max_leaf, true) <= (size_t)lds_limit ? 1 : 0;
    const size_t lds = leaf_finalize_lds(dp, max_leaf, ids != 0);
    if (prec == RPF_DIST_BF16)
        leaf_finalize<__bf16>(s, grid, lds, X, d, dp, leaves, nleaf, perm, n, leaf_of, centroid, Xc, nrm, 3.0e38f, ids);
    else if (prec == RPF_DIST_FP16)
        leaf_finalize<_Float16>(s, grid, lds, X, d, dp, leaves, nleaf, perm, n, leaf_of, centroid, Xc, nrm, 60000.f,
                                ids);
    else
        leaf_finalize<float>(s, grid, lds, X, d, dp, leaves, nleaf, perm, n, leaf_of, centroid, Xc, nrm, 3.0e38f, ids);
}

}  // namespace rpf
