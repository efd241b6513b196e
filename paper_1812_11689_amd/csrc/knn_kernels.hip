// Candidate stage of Alg. 3: N_q = union of q's leaves over the T trees, exact distances,
// K closest.  Exactness is kept while the bulk arithmetic runs in low precision:
//
//  1. Tiles (k_tile): for every tree and leaf, the Gram matrix of the leaf's rows (or of
//     the queries routed to the leaf against the leaf's rows) runs on MFMA over leaf-centred
//     copies in binary32 / bfloat16 / float16 with binary32 accumulation.  Each pair gets a
//     rigorous interval [lb, ub] for its squared distance:
//        Dt = |a|^2 + |b|^2 - 2 a.b (tile values),  e = E (|a|^2 + |b|^2),
//        delta = C (|a'| + |b'|) with a' = a - mu in binary32,
//        lb = (max(0, sqrt(max(0, Dt - e)) - delta))^2,  ub = (sqrt(Dt + e) + delta)^2,
//     E covering the accumulation (2 gamma_{d+2}, doubled for the unknown MFMA order) and
//     C the rounding of the centred copy.  A pair is kept iff lb <= tau(row).
//  2. Phase I (the first tree, tau = +inf) keeps every pair; k_merge_init sets
//     tau(row) = K-th smallest ub and keeps the pairs with lb <= tau.
//  3. Phase II (the other trees) keeps pairs with lb <= tau(row) only.  Every true
//     neighbour passes in every tree that holds it, since lb <= D <= K-th D <= tau.
//  4. k_final: dedup by index, tau' = K-th smallest ub, rerank {lb <= tau'} with the
//     canonical binary32 distance; the window D32 <= D32_(K) (1 + w) (w covers the
//     binary32 error) is ordered by the canonical binary64 distance and the index.
//  5. Rows whose buffers overflowed take k_fallback: the exhaustive union in binary64.
#include <math.h>
#include <stdlib.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "rpf_internal.h"

namespace rpf {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <int PREC>
struct TileCfg;
template <>
struct TileCfg<RPF_DIST_FP32> {
    using T = float;
    static constexpr int KC = 32, LDW = 33, KSTEP = 2;
};
template <>
struct TileCfg<RPF_DIST_BF16> {
    using T = __bf16;
    static constexpr int KC = 64, LDW = 72, KSTEP = 16;
};
template <>
struct TileCfg<RPF_DIST_FP16> {
    using T = _Float16;
    static constexpr int KC = 64, LDW = 72, KSTEP = 16;
};
// split bfloat16: every staged binary32 value a is held as hi = bf16(a) and lo = bf16(a - hi)
// in two LDS tiles of this shape (hi tile, then lo tile)
template <>
struct TileCfg<RPF_DIST_BF16X3> {
    using T = __bf16;
    static constexpr int KC = 32, LDW = 40, KSTEP = 16;
};

// k-chunk of the all-points symmetric tiles.  binary32: 32 columns, whose rows arrive in LDS
// as gathered (the raw tile, written by direct global-to-LDS loads while the previous chunk
// is on MFMA) and are then centred into the operand tile.  16-bit tiles: twice the chunk of
// the other tiles, staged from X directly; their operand tile is the only large LDS array and
// the Phase II queues and Phase I transposes reuse its space, and fewer chunks mean fewer
// exposed row gathers.  (The 16-bit kernels hold their registers at the occupancy cap, where
// spill reloads in the k loop would make the MFMAs wait for the raw tile's loads.)
// ALT, the tuner's alternative chunk: binary32 64 columns staged from X directly; 16-bit
// tiles the chunk of the other tiles.
template <int PREC, bool ALT = false>
struct SymCfg {
    using T = typename TileCfg<PREC>::T;
    static constexpr bool DMA = PREC == RPF_DIST_FP32 && !ALT;
    static constexpr int KC = PREC == RPF_DIST_FP32 ? (ALT ? 64 : 32) : (ALT ? 1 : 2) * TileCfg<PREC>::KC;
    static constexpr int LDW = PREC == RPF_DIST_FP32 ? KC + 1 : KC + 8;
    static constexpr int KSTEP = TileCfg<PREC>::KSTEP;
};

template <int PREC>
__device__ inline f32x16 mfma_step(const typename TileCfg<PREC>::T *sa, const typename TileCfg<PREC>::T *sb,
                                   f32x16 acc) {
    if constexpr (PREC == RPF_DIST_FP32) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(*sa, *sb, acc, 0, 0, 0);
    } else if constexpr (PREC == RPF_DIST_BF16) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8 *>(sa),
                                                       *reinterpret_cast<const bf16x8 *>(sb), acc, 0, 0, 0);
    } else {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(*reinterpret_cast<const f16x8 *>(sa),
                                                      *reinterpret_cast<const f16x8 *>(sb), acc, 0, 0, 0);
    }
}

// MFMA operand of one lane: one binary32, or eight 16-bit values
template <int PREC>
struct MfmaOperand {
    using type = float;
};
template <>
struct MfmaOperand<RPF_DIST_BF16> {
    using type = bf16x8;
};
template <>
struct MfmaOperand<RPF_DIST_FP16> {
    using type = f16x8;
};
template <>
struct MfmaOperand<RPF_DIST_BF16X3> {
    using type = bf16x8;
};

template <int PREC>
__device__ inline f32x16 mfma_op(typename MfmaOperand<PREC>::type a, typename MfmaOperand<PREC>::type b, f32x16 acc) {
    if constexpr (PREC == RPF_DIST_FP32)
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    else if constexpr (PREC == RPF_DIST_BF16 || PREC == RPF_DIST_BF16X3)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc, 0, 0, 0);
}

template <int PREC>
__device__ inline void stage_rows(typename TileCfg<PREC>::T *s, const typename TileCfg<PREC>::T *g, int rows,
                                  int rows_pad, int dp, int k0, int nthreads) {
    using C = TileCfg<PREC>;
    using T = typename C::T;
    if constexpr (PREC == RPF_DIST_FP32) {
        constexpr int VPR = C::KC / 4;  // float4 per row chunk
        for (int v = threadIdx.x; v < rows_pad * VPR; v += nthreads) {
            const int r = v / VPR, c = (v % VPR) * 4;
            float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < rows && k0 + c < dp) val = *reinterpret_cast<const float4 *>(g + (int64_t)r * dp + k0 + c);
            T *dst = s + r * C::LDW + c;
            dst[0] = val.x;
            dst[1] = val.y;
            dst[2] = val.z;
            dst[3] = val.w;
        }
    } else {
        constexpr int VPR = C::KC / 8;  // 16-byte vectors of 8 elements
        for (int v = threadIdx.x; v < rows_pad * VPR; v += nthreads) {
            const int r = v / VPR, c = (v % VPR) * 8;
            uint4 val = make_uint4(0, 0, 0, 0);
            if (r < rows && k0 + c < dp) val = *reinterpret_cast<const uint4 *>(g + (int64_t)r * dp + k0 + c);
            *reinterpret_cast<uint4 *>(s + r * C::LDW + c) = val;
        }
    }
}

// Rows 0 .. rows-1 of a leaf staged straight from X: row r is point pt[r], centred on the
// leaf's centroid mu and rounded to the tile type (zero past d), columns [k0, k0 + KC), rows
// up to rows_pad zero-filled.  These are exactly the values of the leaf-ordered centred copy
// (x - mu in binary32, then one rounding to the tile type), so a tile staged this way equals
// one staged from that copy.  VEC: d % 4 == 0 (four-column groups never straddle d).
template <int PREC, bool VEC, bool ALT = false>
__device__ inline void stage_rows_x(typename TileCfg<PREC>::T *s, const float *__restrict__ X, int d,
                                    const int32_t *s_pt, const float *__restrict__ mu, int rows, int rows_pad,
                                    int k0, int nthreads, typename TileCfg<PREC>::T *s_lo = nullptr) {
    using C = SymCfg<PREC, ALT>;
    using T = typename C::T;
    constexpr int EV = PREC == RPF_DIST_FP32 ? 4 : 8;  // elements per LDS vector
    constexpr int VPR = C::KC / EV;
    for (int v = threadIdx.x; v < rows_pad * VPR; v += nthreads) {
        const int r = v / VPR, c = (v % VPR) * EV, j = k0 + c;
        float a[EV];
#pragma unroll
        for (int e = 0; e < EV; e++) a[e] = 0.f;
        if (VEC) {
            // every load of the vector is issued before the first is used (one wait per
            // vector): addresses past the leaf or past d are clamped to the first four values
            // of X and of the centroid (present whenever d >= 4), and those lanes keep zero
            const bool rok = r < rows;
            const float *x = X + (rok ? (int64_t)s_pt[r] * d : 0);
            float4 xv[EV / 4], uv[EV / 4];
#pragma unroll
            for (int h = 0; h < EV / 4; h++) {
                const int o = rok && j + 4 * h < d ? j + 4 * h : 0;
                xv[h] = *reinterpret_cast<const float4 *>(x + o);
                uv[h] = *reinterpret_cast<const float4 *>(mu + (j + 4 * h < d ? j + 4 * h : 0));
            }
#pragma unroll
            for (int h = 0; h < EV / 4; h++) {
                if (rok && j + 4 * h < d) {
                    a[4 * h] = xv[h].x - uv[h].x;
                    a[4 * h + 1] = xv[h].y - uv[h].y;
                    a[4 * h + 2] = xv[h].z - uv[h].z;
                    a[4 * h + 3] = xv[h].w - uv[h].w;
                }
            }
        } else if (r < rows) {
            const float *x = X + (int64_t)s_pt[r] * d;
#pragma unroll
            for (int e = 0; e < EV; e++)
                if (j + e < d) a[e] = x[j + e] - mu[j + e];
        }
        T *dst = s + r * C::LDW + c;
        if constexpr (PREC == RPF_DIST_BF16X3) {
            // hi = RN_bf16(a); a - hi is exact in binary32; lo = RN_bf16(a - hi)
            T hq[EV], lq[EV];
#pragma unroll
            for (int e = 0; e < EV; e++) {
                hq[e] = (T)a[e];
                lq[e] = (T)(a[e] - (float)hq[e]);
            }
            uint4 wh, wl;
            __builtin_memcpy(&wh, hq, sizeof(wh));
            __builtin_memcpy(&wl, lq, sizeof(wl));
            *reinterpret_cast<uint4 *>(dst) = wh;
            *reinterpret_cast<uint4 *>(s_lo + r * C::LDW + c) = wl;
        } else if constexpr (PREC == RPF_DIST_FP32) {
#pragma unroll
            for (int e = 0; e < EV; e++) dst[e] = a[e];
        } else {
            T q[EV];
#pragma unroll
            for (int e = 0; e < EV; e++) q[e] = (T)a[e];
            uint4 w;
            __builtin_memcpy(&w, q, sizeof(w));
            *reinterpret_cast<uint4 *>(dst) = w;
        }
    }
}

// Rows 0 .. rows-1 of a leaf, columns [k0, k0 + KC), from the raw tile (binary32 rows as
// gathered, KC floats each) to the operand tile(s): centred on mu and rounded to the tile
// type, exactly as stage_rows_x does from X (zero past d and past the leaf's rows).  d % 4 == 0.
template <int PREC>
__device__ inline void convert_rows(typename TileCfg<PREC>::T *s, const float *raw, int d,
                                    const float *__restrict__ mu, int rows, int rows_pad, int k0, int nthreads,
                                    typename TileCfg<PREC>::T *s_lo = nullptr) {
    using C = SymCfg<PREC>;
    using T = typename C::T;
    constexpr int EV = PREC == RPF_DIST_FP32 ? 4 : 8;
    constexpr int VPR = C::KC / EV;
    for (int v = threadIdx.x; v < rows_pad * VPR; v += nthreads) {
        const int r = v / VPR, c = (v % VPR) * EV, j = k0 + c;
        float a[EV];
#pragma unroll
        for (int e = 0; e < EV; e++) a[e] = 0.f;
        if (r < rows) {
#pragma unroll
            for (int h = 0; h < EV; h += 4) {
                if (j + h < d) {
                    const float4 xv = *reinterpret_cast<const float4 *>(raw + r * C::KC + c + h);
                    const float4 u = *reinterpret_cast<const float4 *>(mu + j + h);
                    a[h] = xv.x - u.x;
                    a[h + 1] = xv.y - u.y;
                    a[h + 2] = xv.z - u.z;
                    a[h + 3] = xv.w - u.w;
                }
            }
        }
        T *dst = s + r * C::LDW + c;
        if constexpr (PREC == RPF_DIST_BF16X3) {
            T hq[EV], lq[EV];
#pragma unroll
            for (int e = 0; e < EV; e++) {
                hq[e] = (T)a[e];
                lq[e] = (T)(a[e] - (float)hq[e]);
            }
            uint4 wh, wl;
            __builtin_memcpy(&wh, hq, sizeof(wh));
            __builtin_memcpy(&wl, lq, sizeof(wl));
            *reinterpret_cast<uint4 *>(dst) = wh;
            *reinterpret_cast<uint4 *>(s_lo + r * C::LDW + c) = wl;
        } else if constexpr (PREC == RPF_DIST_FP32) {
#pragma unroll
            for (int e = 0; e < EV; e++) dst[e] = a[e];
        } else {
            T q[EV];
#pragma unroll
            for (int e = 0; e < EV; e++) q[e] = (T)a[e];
            uint4 w;
            __builtin_memcpy(&w, q, sizeof(w));
            *reinterpret_cast<uint4 *>(dst) = w;
        }
    }
}

// Issue the direct global-to-LDS loads of a chunk's rows: each wave instruction moves eight
// rows of 32 binary32 columns (16 bytes per lane, lane i to raw + 16 i bytes of its group), a
// wave takes the groups wu, wu + nw, ...  Lanes past the leaf's rows or past d load nothing
// (their raw values are never read).  d % 4 == 0 and X 16-byte aligned.
__device__ inline void issue_rows_dma(float *raw, const float *__restrict__ X, int d, const int32_t *s_pt, int rows,
                                      int k0, int wu, int nw) {
    const int lane = lane_id();  // recomputed here rather than kept live across the k loop
    for (int g = wu; 8 * g < rows; g += nw) {
        const int r = 8 * g + (lane >> 3), j = k0 + 4 * (lane & 7);
        if (r < rows && j < d)
            __builtin_amdgcn_global_load_lds(X + (int64_t)s_pt[r] * d + j,
                                             (__attribute__((address_space(3))) void *)(raw + 8 * g * 32), 16, 0, 0);
    }
}

struct BoundCoef {
    float e;      // E: accumulation error per unit of |a|^2 + |b|^2
    float c;      // C: centred-copy rounding per unit of |a'| + |b'|
    float eta;    // absolute rounding floor of the copy (float16 subnormals), times sqrt(d)
};

__device__ inline void pair_bounds(float na, float nb, float ra, float rb, float g, BoundCoef bc, float &lb,
                                   float &ub) {
    const float Dt = na + nb - 2.f * g;
    const float e = bc.e * (na + nb);
    const float delta = bc.c * (ra + rb) + bc.eta;
    const float lo = fmaxf(Dt - e, 0.f);
    const float ls = fmaxf(sqrtf(lo) - delta, 0.f);
    const float hs = sqrtf(fmaxf(Dt + e, 0.f)) + delta;
    lb = ls * ls * (1.f - 1e-6f);
    ub = hs * hs * (1.f + 1e-6f);
    if (!(ra < INFINITY) || !(rb < INFINITY) || !(lb == lb) || !(ub == ub)) {  // out of the copy's range
        lb = 0.f;
        ub = INFINITY;
    }
    lb = fminf(lb, 3.40282347e38f);  // +inf marks a Phase I slot that no pair fills, never a pair
}

// Where a tile's pairs go.
//  mode 0 (Phase I, the first trees): every pair of the leaf, as (lb, ub) at the fixed slot
//          row * cap + (tree - t0) * ML + (position of the column in its leaf); the slot
//          names the column (the leaf's permutation segment holds its index) and lb = +inf
//          marks a slot that no pair fills;
//  mode 1 (Phase II): pairs with lb <= tau(row), appended at row * cap + atomic count; or,
//          when bcnt is set (all-points symmetric tiles, where one block holds every pair of
//          a row in its tree), in the row's bucket of S records for its tree, counted in LDS:
//          row * cap + (tree - t1) * S + rank, the bucket's count stored in bcnt[row][tree - t1]
//          at the end, and records past S appended to the row's overflow list at
//          row * cap + nT2 * S + atomic count.
struct TileOut {
    int mode;
    int t0;
    int ML;
    int cap;
    Ent *ent;          // mode 1 records
    int32_t *cnt;      // mode 1 counters (bucket mode: of the overflow list)
    const float *tau;  // mode 1 thresholds
    uint32_t *plub;    // mode 0: packed bounds per slot (pack_bounds), (+inf, +inf) where empty
    int32_t *roff;     // mode 0: [tree - t0][nrows] start of the row's leaf in the permutation
    int64_t nrows;
    uint8_t *bcnt;     // mode 1 bucket counts [nrows][nT2], or nullptr (counted lists)
    int t1;            // bucket mode: first Phase II tree
    int S;             // bucket mode: records per bucket
    int nT2;           // bucket mode: Phase II trees
    int capO;          // bucket mode: overflow records per row
    int shape;         // Phase II symmetric tile shape (k_tile_sym SHAPE)
};

constexpr int kQueue = 512;  // per-wave queue of Phase II pairs that pass the cheap test

__device__ inline Ent make_ent(int idx, float lb, float ub) {
    Ent e;
    e.idx = idx;
    e.lb = lb;
    e.ub = ub;
    e.pad = 0;
    return e;
}

__device__ inline Ent invalid_rec() { return make_ent(-1, INFINITY, INFINITY); }

// A Phase I slot: the pair's bounds in four bytes, each kept to the top 16 bits of its
// binary32 pattern (the bfloat16 range) rounded outward -- lb toward zero (truncation of a
// non-negative value), ub away from it -- so they stay bounds on the squared distance.  The
// low half holds lb, the high half ub; +inf in both marks an empty slot.
__device__ inline uint32_t pack_bounds(float lb, float ub) {
    const uint32_t l = __float_as_uint(lb) >> 16;
    const uint32_t u = (__float_as_uint(ub) + 0xffffu) >> 16;  // +inf stays +inf
    return (u << 16) | l;
}

__device__ inline void put_first(const TileOut &o, int64_t slot, float lb, float ub) {
    o.plub[slot] = pack_bounds(lb, ub);
}

__device__ inline void put_first_empty(const TileOut &o, int64_t slot) { put_first(o, slot, INFINITY, INFINITY); }

__device__ inline void emit_filtered(const TileOut &o, int a_pt, int b_pt, float lb, float ub) {
    const int slot = atomicAdd(&o.cnt[a_pt], 1);
    if (slot < o.cap) o.ent[(int64_t)a_pt * o.cap + slot] = make_ent(b_pt, lb, ub);
}

// bucket mode: the record's rank among its row's records of this tree comes from the block's
// LDS counter of that row; only a record past the bucket takes a device-scope atomic
__device__ inline void emit_bucket(const TileOut &o, int32_t *s_cnt, int r, int tb2, int a_pt, int b_pt, float lb,
                                   float ub) {
    const int slot = atomicAdd(&s_cnt[r], 1);
    const int64_t base = (int64_t)a_pt * o.cap;
    if (slot < o.S) {
        o.ent[base + (int64_t)tb2 * o.S + slot] = make_ent(b_pt, lb, ub);
    } else {
        const int q = atomicAdd(&o.cnt[a_pt], 1);
        if (q < o.capO) o.ent[base + (int64_t)o.nT2 * o.S + q] = make_ent(b_pt, lb, ub);
    }
}

// per-row threshold of the cheap test  |b|^2 - 2 a.b <= phi(row),  a necessary condition for
// lb <= tau(row) with the per-pair error terms replaced by their largest value over the tile
__device__ inline float cheap_phi(float tv, float na, float ra, float nmax, float rmax, BoundCoef bc) {
    if (!(tv < INFINITY)) return INFINITY;
    if (tv < 0.f) return -INFINITY;
    if (!(ra < INFINITY) || !(rmax < INFINITY)) return INFINITY;
    const float dmax = bc.c * (ra + rmax) + bc.eta;
    const float emax = bc.e * (na + nmax);
    const float st = sqrtf(tv / (1.f - 1e-6f)) + dmax;
    const float th = st * st + emax;
    return (th - na) + 1e-5f * (th + na + nmax) + 1e-30f;
}

// Workgroups are dealt to the eight XCDs in turn, so block b runs on XCD b % 8.  Block b takes
// job (b % 8) * per + b / 8: each XCD walks one contiguous range of the job list front to back,
// so the tiles of one leaf, which read the same rows, meet in that XCD's L2.  The grid is
// 8 * per blocks with per = ceil(njobs / 8); blocks past the list return.
__device__ inline int64_t xcd_job() {
    const int64_t per = (int64_t)gridDim.x >> 3;
    return (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// One tile job per block: A rows x B rows of one leaf (or query group x leaf), MB waves,
// wave w owns A rows [32w, 32w + 32) against all B rows.  Jobs are taken in XCD order (xcd_job).
template <int MB, int PREC>
__global__ __launch_bounds__(64 * MB) void k_tile(
    const TileJob *__restrict__ jobs, int64_t njobs, const void *__restrict__ A_, const void *__restrict__ B_, int dp,
    int64_t a_stride_tree, int64_t b_stride_tree, const float2 *__restrict__ a_nrm, const float2 *__restrict__ b_nrm,
    const int32_t *__restrict__ a_dest, const int32_t *__restrict__ b_pt, BoundCoef bc, int exclude_self,
    TileOut out) {
    using C = TileCfg<PREC>;
    using T = typename C::T;
    constexpr int M = 32 * MB;
    constexpr int NT = 64 * MB;
    __shared__ __align__(16) T s_a[M * C::LDW];
    __shared__ __align__(16) T s_b[M * C::LDW];
    __shared__ float s_na[M], s_ra[M], s_nb[M], s_rb[M], s_tau[M];
    __shared__ __align__(16) float s_phi[M];
    __shared__ int32_t s_dst[M], s_bpt[M];
    __shared__ float s_bmax[2];
    __shared__ uint2 s_que[MB][kQueue];

    const int64_t ji = xcd_job();
    if (ji >= njobs) return;
    const TileJob job = jobs[ji];
    const int t = job.tree;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wu = __builtin_amdgcn_readfirstlane(w);
    const bool same = job.same != 0;
    const T *A = reinterpret_cast<const T *>(A_) + (t * a_stride_tree + job.a_off) * dp;
    const T *B = reinterpret_cast<const T *>(B_) + (t * b_stride_tree + job.b_off) * dp;
    const float2 *an = a_nrm + t * a_stride_tree + job.a_off;
    const float2 *bn = b_nrm + t * b_stride_tree + job.b_off;
    const int32_t *ad = a_dest + t * a_stride_tree + job.a_off;
    const int32_t *bp = b_pt + t * b_stride_tree + job.b_off;
    const int tb = t - out.t0;
    if (out.mode == 0 && job.leaf_m > out.ML) {
        // a leaf above the first-phase slot stride (a uniform-rule leaf kept whole at the
        // depth cap): its rows take the exhaustive path, which a negative leaf start tells
        // the merge; no slot is written
        for (int r = tid; r < job.a_rows; r += NT) out.roff[(int64_t)tb * out.nrows + ad[r]] = -1;
        return;
    }

    for (int r = tid; r < M; r += NT) {
        if (r < job.a_rows) {
            const float2 q = an[r];
            s_na[r] = q.x;
            s_ra[r] = q.y;
            const int dst = ad[r];
            s_dst[r] = dst;
            s_tau[r] = out.mode == 1 ? out.tau[dst] : INFINITY;
        } else {
            s_na[r] = 0.f;
            s_ra[r] = 0.f;
            s_dst[r] = -1;
            s_tau[r] = -1.f;
        }
        if (r < job.b_rows) {
            const float2 q = bn[r];
            s_nb[r] = q.x;
            s_rb[r] = q.y;
            s_bpt[r] = bp[r];
        } else {
            s_nb[r] = 0.f;
            s_rb[r] = 0.f;
            s_bpt[r] = -1;
        }
    }
    __syncthreads();
    if (tid < 64) {
        float mn = 0.f, mr = 0.f;
        for (int r = lane; r < job.b_rows; r += 64) {
            mn = fmaxf(mn, s_nb[r]);
            mr = fmaxf(mr, s_rb[r]);
        }
        for (int o = 32; o > 0; o >>= 1) {
            mn = fmaxf(mn, __shfl_xor(mn, o, 64));
            mr = fmaxf(mr, __shfl_xor(mr, o, 64));
        }
        if (lane == 0) {
            s_bmax[0] = mn;
            s_bmax[1] = mr;
        }
    }
    __syncthreads();
    for (int r = tid; r < M; r += NT) s_phi[r] = cheap_phi(s_tau[r], s_na[r], s_ra[r], s_bmax[0], s_bmax[1], bc);
    if (out.mode == 0) {  // Phase I: the slots no pair of this tile fills (past the leaf, self)
        const bool last = job.b_pos + job.b_rows == job.leaf_m;
        for (int r = tid; r < job.a_rows; r += NT) {
            const int64_t er = (int64_t)s_dst[r] * out.cap + (int64_t)tb * out.ML;
            if (last) {
                for (int c = job.leaf_m; c < out.ML; c++) put_first_empty(out, er + c);
                out.roff[(int64_t)tb * out.nrows + s_dst[r]] = (int32_t)(job.b_off - job.b_pos);
            }
            if (same && exclude_self) put_first_empty(out, er + job.b_pos + r);
        }
    }

    f32x16 acc[MB];
#pragma unroll
    for (int cb = 0; cb < MB; cb++)
#pragma unroll
        for (int v = 0; v < 16; v++) acc[cb][v] = 0.f;
    const int nbb = (job.b_rows + 31) >> 5;
    const bool active = 32 * wu < job.a_rows;
    const int fr = lane & 31;
    const int fk = PREC == RPF_DIST_FP32 ? (lane >> 5) : 8 * (lane >> 5);
    const int a_pad = ((job.a_rows + 31) >> 5) << 5;
    const int b_pad = nbb << 5;
    for (int k0 = 0; k0 < dp; k0 += C::KC) {
        __syncthreads();
        stage_rows<PREC>(s_a, A, job.a_rows, a_pad, dp, k0, NT);
        if (!same) stage_rows<PREC>(s_b, B, job.b_rows, b_pad, dp, k0, NT);
        __syncthreads();
        const T *sb_base = same ? s_a : s_b;
        int kmax = dp - k0 < C::KC ? dp - k0 : C::KC;
        kmax = (kmax + C::KSTEP - 1) / C::KSTEP * C::KSTEP;
        if (active) {
            for (int kk = 0; kk < kmax; kk += C::KSTEP) {
                const T *pa = s_a + (32 * wu + fr) * C::LDW + kk + fk;
#pragma unroll
                for (int cb = 0; cb < MB; cb++) {
                    if (cb < nbb) {
                        const T *pb = sb_base + (32 * cb + fr) * C::LDW + kk + fk;
                        acc[cb] = mfma_step<PREC>(pa, pb, acc[cb]);
                    }
                }
            }
        }
    }
    if (!active) return;

    if (out.mode == 0) {
#pragma unroll
        for (int cb = 0; cb < MB; cb++) {
            if (cb >= nbb) continue;
            const int col = 32 * cb + (lane & 31);
            if (col >= job.b_rows) continue;
            const float nb = s_nb[col], rb = s_rb[col];
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int row = 32 * wu + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                if (row >= job.a_rows || (same && exclude_self && row == col)) continue;
                float lb, ub;
                pair_bounds(s_na[row], nb, s_ra[row], rb, acc[cb][v], bc, lb, ub);
                put_first(out, (int64_t)s_dst[row] * out.cap + (int64_t)tb * out.ML + job.b_pos + col, lb, ub);
            }
        }
        return;
    }
    // Phase II: a cheap test over every pair; the pairs that pass are compacted by ballot
    // into a per-wave LDS queue, whose exact bounds and emissions run when it would overflow
    // and at the end (wave-uniform decisions throughout)
    uint2 *que = s_que[wu];
    uint32_t qc = 0;
    auto flush = [&](uint32_t nq) {
        wave_sync();
        for (uint32_t i = lane; i < nq; i += 64) {
            const uint2 e = que[i];
            const int row = e.x & 255, col = (e.x >> 8) & 255;
            float lb, ub;
            pair_bounds(s_na[row], s_nb[col], s_ra[row], s_rb[col], __uint_as_float(e.y), bc, lb, ub);
            if (lb <= s_tau[row]) emit_filtered(out, s_dst[row], s_bpt[col], lb, ub);
        }
        wave_sync();
    };
    // the lane's 16 rows come in four runs of four: their thresholds are read up front
    // (rows past the block hold -inf), so the tests below are branch-free register work
    float pr[16];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const float4 p4 = *reinterpret_cast<const float4 *>(s_phi + 32 * wu + 8 * j + 4 * (lane >> 5));
        pr[4 * j] = p4.x; pr[4 * j + 1] = p4.y; pr[4 * j + 2] = p4.z; pr[4 * j + 3] = p4.w;
    }
#pragma unroll
    for (int cb = 0; cb < MB; cb++) {
        if (cb >= nbb) continue;
        const int col = 32 * cb + (lane & 31);  // < M: columns past the block hold n = 0
        const bool colok = col < job.b_rows;
        const float nb = s_nb[col];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            uint32_t bits = 0;
            uint64_t mk[8];
            uint32_t tot = 0;
#pragma unroll
            for (int v8 = 0; v8 < 8; v8++) {
                const int v = 8 * h + v8;
                const int row = 32 * wu + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const bool p = colok & (__builtin_fmaf(-2.f, acc[cb][v], nb) <= pr[v]) &
                               !(same & (exclude_self != 0) & (row == col));
                bits |= (p ? 1u : 0u) << v8;
                mk[v8] = __ballot(p);
                tot += (uint32_t)__popcll(mk[v8]);
            }
            if (qc + tot > (uint32_t)kQueue) {
                flush(qc);
                qc = 0;
            }
#pragma unroll
            for (int v8 = 0; v8 < 8; v8++) {
                const int v = 8 * h + v8;
                if ((bits >> v8) & 1u) {
                    const int row = 32 * wu + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    que[qc + mask_rank(mk[v8])] = make_uint2((uint32_t)row | ((uint32_t)col << 8), __float_as_uint(acc[cb][v]));
                }
                qc += (uint32_t)__popcll(mk[v8]);
            }
        }
    }
    flush(qc);
}

// ---------------------------------------------------------------- tiles on the 1/255 grid

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
constexpr int kQ8KC = 64;   // int8 columns staged per chunk
constexpr int kQ8LDW = 80;  // LDS row stride in bytes (16-byte aligned, padded against bank conflicts)

// Bounds on the binary64 squared distance of two grid points from their exact grid distance
// dint = sum (k_a - k_b)^2.  With q = k / 255 and each coordinate x = q (1 + e), |e| <= 2^-24
// (one correctly rounded division), the real distance of the binary32 points is within
// 2^-24 (|q_a| + |q_b|) of sqrt(dint) / 255; dint / 255^2 in binary32 is off by at most 3
// roundings (2^-24 each); the 1e-6 widening covers the square roots (the hardware
// instruction, within 1 ulp: 2^-22 relative once squared; its argument is 0 or at least
// 1/65025, never subnormal) and the binary64 canonical sum.
__device__ inline void lattice_bounds(int32_t dint, float ra, float rb, float &lb, float &ub) {
    constexpr float u = 5.9604645e-8f;  // 2^-24
    const float dt = (float)dint * (1.f / 65025.f);
    const float delta = u * 1.01f * (ra + rb);
    const float lo = fmaxf(__builtin_amdgcn_sqrtf(dt * (1.f - 4.f * u)) - delta, 0.f);
    const float hi = __builtin_amdgcn_sqrtf(dt * (1.f + 4.f * u)) + delta;
    lb = fminf(lo * lo * (1.f - 1e-6f), 3.40282347e38f);
    ub = hi * hi * (1.f + 1e-6f);
}

// Integer threshold of the cheap test of a row: lb <= tau(row) implies
// dint <= phi_d = (sqrt(tau / (1 - 1e-6)) + delta_max)^2 * 255^2 / ((1 - 4u)(1 - 3u)), taken with
// slack upward; returned as phi_d - |k_row - 128|^2 so that the test reads |k_col - 128|^2 - 2G <= phi.
__device__ inline int32_t lattice_phi(float tv, int32_t na, float ra, float rbmax) {
    if (!(tv < INFINITY)) return INT32_MAX;
    if (tv < 0.f) return INT32_MIN;
    constexpr float u = 5.9604645e-8f;
    const float st = sqrtf(tv / (1.f - 1e-6f)) + u * 1.01f * (ra + rbmax);
    const double pd = (double)st * (double)st * 65025.0 * (1.0 + 1e-5) + 2.0;
    const double ph = pd - (double)na;
    return ph >= 2.0e9 ? INT32_MAX : (int32_t)ph;
}

// All-points tile of grid points (one job: A rows x B rows of one leaf, MB waves; wave w owns
// A rows [32w, 32w + 32)): rows are gathered from the int8 copy through the permutation, the
// integer Gram product runs on v_mfma_i32_32x32x32_i8, and the grid distance
// |k_a - 128|^2 + |k_b - 128|^2 - 2G is exact.  Outputs as the other tiles (Phase I slots,
// Phase II records below the row's threshold).  Jobs are taken in XCD order (xcd_job).
template <int MB>
__global__ __launch_bounds__(64 * MB) void k_tile_q8(const TileJob *__restrict__ jobs, int64_t njobs,
                                                    const int8_t *__restrict__ Xq,
                                                    int dq, const LatNorm *__restrict__ qn,
                                                    const int32_t *__restrict__ perm, int64_t n, int exclude_self,
                                                    TileOut out) {
    constexpr int M = 32 * MB;
    constexpr int NT = 64 * MB;
    __shared__ __align__(16) int8_t s_a[2][M * kQ8LDW];
    __shared__ __align__(16) int8_t s_b[2][M * kQ8LDW];
    __shared__ int32_t s_na[M], s_nb[M], s_phi[M];
    __shared__ float s_ra[M], s_rb[M], s_tau[M];
    __shared__ int32_t s_dst[M], s_bpt[M];
    __shared__ float s_rbmax;
    __shared__ uint2 s_que[MB][kQueue];

    const int64_t ji = xcd_job();
    if (ji >= njobs) return;
    const TileJob job = jobs[ji];
    const int t = job.tree;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wu = __builtin_amdgcn_readfirstlane(w);
    const bool same = job.same != 0;
    const int32_t *ap = perm + (int64_t)t * n + job.a_off;
    const int32_t *bp = perm + (int64_t)t * n + job.b_off;
    const int tb = t - out.t0;
    if (out.mode == 0 && job.leaf_m > out.ML) {  // as in k_tile: the rows take the exhaustive path
        for (int r = tid; r < job.a_rows; r += NT) out.roff[(int64_t)tb * out.nrows + ap[r]] = -1;
        return;
    }
    for (int r = tid; r < M; r += NT) {
        if (r < job.a_rows) {
            const int p = ap[r];
            const LatNorm q = qn[p];
            s_dst[r] = p;
            s_na[r] = q.na;
            s_ra[r] = q.ra;
            s_tau[r] = out.mode == 1 ? out.tau[p] : INFINITY;
        } else {
            s_dst[r] = -1;
            s_na[r] = 0;
            s_ra[r] = 0.f;
            s_tau[r] = -1.f;
        }
        if (r < job.b_rows) {
            const int p = bp[r];
            const LatNorm q = qn[p];
            s_bpt[r] = p;
            s_nb[r] = q.na;
            s_rb[r] = q.ra;
        } else {
            s_bpt[r] = -1;
            s_nb[r] = 0;
            s_rb[r] = 0.f;
        }
    }
    __syncthreads();
    if (tid < 64) {
        float mr = 0.f;
        for (int r = lane; r < job.b_rows; r += 64) mr = fmaxf(mr, s_rb[r]);
        for (int o = 32; o > 0; o >>= 1) mr = fmaxf(mr, __shfl_xor(mr, o, 64));
        if (lane == 0) s_rbmax = mr;
    }
    __syncthreads();
    for (int r = tid; r < M; r += NT) s_phi[r] = lattice_phi(s_tau[r], s_na[r], s_ra[r], s_rbmax);
    if (out.mode == 0) {  // Phase I: the slots no pair of this tile fills (past the leaf, self)
        const bool last = job.b_pos + job.b_rows == job.leaf_m;
        for (int r = tid; r < job.a_rows; r += NT) {
            const int64_t er = (int64_t)s_dst[r] * out.cap + (int64_t)tb * out.ML;
            if (last) {
                for (int c = job.leaf_m; c < out.ML; c++) put_first_empty(out, er + c);
                out.roff[(int64_t)tb * out.nrows + s_dst[r]] = (int32_t)(job.b_off - job.b_pos);
            }
            if (same && exclude_self) put_first_empty(out, er + job.b_pos + r);
        }
    }

    i32x16 acc[MB];
#pragma unroll
    for (int cb = 0; cb < MB; cb++)
#pragma unroll
        for (int v = 0; v < 16; v++) acc[cb][v] = 0;
    const int nbb = (job.b_rows + 31) >> 5;
    const bool active = 32 * wu < job.a_rows;
    const int fr = lane & 31;
    const int fk = 16 * (lane >> 5);  // the lane's 16 consecutive int8 of the 32-column step
    const int a_pad = ((job.a_rows + 31) >> 5) << 5;
    const int b_pad = nbb << 5;
    // Staging: thread tid owns the 16-byte piece (tid % VPR) of rows tid / VPR + SR * i (i < 2)
    // of each side.  Chunks are double-buffered in LDS and the gathers of chunk c + 1 are issued
    // before the MFMAs of chunk c, so their latency hides behind the products.  Rows past the
    // tile load a valid row (the tile's first) and stage zeros.
    constexpr int VPR = kQ8KC / 16;  // 16-byte vectors per staged row chunk
    constexpr int SR = NT / VPR;     // rows staged per pass (M = 2 SR)
    static_assert(M == 2 * SR, "two staged rows per thread and side");
    const int sc = (tid % VPR) * 16;
    const int sr0 = tid / VPR, sr1 = sr0 + SR;
    const bool oka0 = sr0 < job.a_rows, oka1 = sr1 < job.a_rows;
    const bool okb0 = sr0 < job.b_rows, okb1 = sr1 < job.b_rows;
    const bool sta0 = sr0 < a_pad, sta1 = sr1 < a_pad;
    const bool stb0 = !same && sr0 < b_pad, stb1 = !same && sr1 < b_pad;
    const int8_t *ga0 = Xq + (int64_t)s_dst[oka0 ? sr0 : 0] * dq + sc;
    const int8_t *ga1 = Xq + (int64_t)s_dst[oka1 ? sr1 : 0] * dq + sc;
    const int8_t *gb0 = Xq + (int64_t)s_bpt[okb0 ? sr0 : 0] * dq + sc;
    const int8_t *gb1 = Xq + (int64_t)s_bpt[okb1 ? sr1 : 0] * dq + sc;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 z4 = {0u, 0u, 0u, 0u};
    u32x4 va0, va1, vb0 = z4, vb1 = z4;
    auto gather = [&](int k0) {
        va0 = *reinterpret_cast<const u32x4 *>(ga0 + k0);
        va1 = *reinterpret_cast<const u32x4 *>(ga1 + k0);
        if (!same) {
            vb0 = *reinterpret_cast<const u32x4 *>(gb0 + k0);
            vb1 = *reinterpret_cast<const u32x4 *>(gb1 + k0);
        }
    };
    auto put = [&](int buf) {
        int8_t *pa = s_a[buf], *pb = s_b[buf];
        if (sta0) *reinterpret_cast<u32x4 *>(pa + sr0 * kQ8LDW + sc) = oka0 ? va0 : z4;
        if (sta1) *reinterpret_cast<u32x4 *>(pa + sr1 * kQ8LDW + sc) = oka1 ? va1 : z4;
        if (stb0) *reinterpret_cast<u32x4 *>(pb + sr0 * kQ8LDW + sc) = okb0 ? vb0 : z4;
        if (stb1) *reinterpret_cast<u32x4 *>(pb + sr1 * kQ8LDW + sc) = okb1 ? vb1 : z4;
    };
    gather(0);
    put(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < dq; k0 += kQ8KC) {
        const bool more = k0 + kQ8KC < dq;
        if (more) gather(k0 + kQ8KC);
        const int8_t *sa = s_a[buf];
        const int8_t *sb = same ? s_a[buf] : s_b[buf];
        if (active) {
#pragma unroll
            for (int kk = 0; kk < kQ8KC; kk += 32) {
                const i32x4 fa = *reinterpret_cast<const i32x4 *>(sa + (32 * wu + fr) * kQ8LDW + kk + fk);
                i32x4 fb[MB];
#pragma unroll
                for (int cb = 0; cb < MB; cb++)
                    fb[cb] = *reinterpret_cast<const i32x4 *>(sb + (32 * (cb < nbb ? cb : 0) + fr) * kQ8LDW + kk + fk);
#pragma unroll
                for (int cb = 0; cb < MB; cb++)
                    if (cb < nbb) acc[cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa, fb[cb], acc[cb], 0, 0, 0);
            }
        }
        if (more) put(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    if (!active) return;

    if (out.mode == 0) {
#pragma unroll
        for (int cb = 0; cb < MB; cb++) {
            if (cb >= nbb) continue;
            const int col = 32 * cb + (lane & 31);
            if (col >= job.b_rows) continue;
            const int32_t nb = s_nb[col];
            const float rb = s_rb[col];
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int row = 32 * wu + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                if (row >= job.a_rows || (same && exclude_self && row == col)) continue;
                float lb, ub;
                lattice_bounds(s_na[row] + nb - 2 * acc[cb][v], s_ra[row], rb, lb, ub);
                put_first(out, (int64_t)s_dst[row] * out.cap + (int64_t)tb * out.ML + job.b_pos + col, lb, ub);
            }
        }
        return;
    }
    // Phase II: the integer cheap test over every pair; passing pairs are compacted into a
    // per-wave LDS queue and get their exact bounds when it would overflow and at the end
    uint2 *que = s_que[wu];
    uint32_t qc = 0;
    auto flush = [&](uint32_t nq) {
        wave_sync();
        for (uint32_t i = lane; i < nq; i += 64) {
            const uint2 e = que[i];
            const int row = e.x & 255, col = (e.x >> 8) & 255;
            float lb, ub;
            lattice_bounds(s_na[row] + s_nb[col] - 2 * (int32_t)e.y, s_ra[row], s_rb[col], lb, ub);
            if (lb <= s_tau[row]) emit_filtered(out, s_dst[row], s_bpt[col], lb, ub);
        }
        wave_sync();
    };
    int32_t pr[16];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int4 p4 = *reinterpret_cast<const int4 *>(s_phi + 32 * wu + 8 * j + 4 * (lane >> 5));
        pr[4 * j] = p4.x; pr[4 * j + 1] = p4.y; pr[4 * j + 2] = p4.z; pr[4 * j + 3] = p4.w;
    }
#pragma unroll
    for (int cb = 0; cb < MB; cb++) {
        if (cb >= nbb) continue;
        const int col = 32 * cb + (lane & 31);
        const bool colok = col < job.b_rows;
        const int32_t nb = s_nb[col];
        // wave-uniform: only the block on the diagonal holds self pairs, and only the tile's
        // last block columns past the leaf; the others take the test alone
        const bool full = (same && exclude_self != 0 && cb == wu) || 32 * cb + 32 > job.b_rows;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            uint32_t bits = 0;
            uint64_t mk[8];
            uint32_t tot = 0;
            auto test = [&](auto FULL) {
#pragma unroll
                for (int v8 = 0; v8 < 8; v8++) {
                    const int v = 8 * h + v8;
                    bool p = nb - 2 * acc[cb][v] <= pr[v];
                    if constexpr (decltype(FULL)::value) {
                        const int row = 32 * wu + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                        p = p & colok & !(same & (exclude_self != 0) & (row == col));
                    }
                    bits |= (p ? 1u : 0u) << v8;
                    mk[v8] = __ballot(p);
                    tot += (uint32_t)__popcll(mk[v8]);
                }
            };
            if (full) test(std::true_type{});
            else test(std::false_type{});
            if (qc + tot > (uint32_t)kQueue) {
                flush(qc);
                qc = 0;
            }
#pragma unroll
            for (int v8 = 0; v8 < 8; v8++) {
                const int v = 8 * h + v8;
                if ((bits >> v8) & 1u) {
                    const int row = 32 * wu + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    que[qc + mask_rank(mk[v8])] = make_uint2((uint32_t)row | ((uint32_t)col << 8), (uint32_t)acc[cb][v]);
                }
                qc += (uint32_t)__popcll(mk[v8]);
            }
        }
    }
    flush(qc);
}

// All-points tile of one leaf whose rows all fit (m <= 32 NB): the Gram matrix is symmetric,
// so only blocks (i, j) with i <= j run on MFMA and an off-diagonal block serves both
// (row -> col) and (col -> row).  Block rows p and NB-1-p form a pair of NB + 1 blocks,
// split between two waves (ceil and floor of half), so NB waves share the triangle evenly;
// both operands come from the same LDS tile.  Blocks wholly past the leaf are skipped.
//
// Phase II at NB = 8 runs 12 waves: three per pair of block rows, three blocks each, so the
// accumulators take 48 registers rather than 80 and six waves share a SIMD instead of four.
//
// SHAPE (Phase II tile shapes the tuner chooses among; 0 is the default): bit 0 the
// alternative k-chunk (SymCfg ALT), bit 1 queues of 256 entries per wave, bit 2 (NB = 8) eight
// waves per block (five blocks each) instead of twelve.
constexpr int sym_waves(int NB, int MODE, int SHAPE = 0) {
    return NB >= 2 ? (MODE >= 1 && NB == 8 && !(SHAPE & 4) ? 12 : NB) : 1;
}

template <int NB, int PREC, int MODE, int SHAPE = 0>
__global__ __launch_bounds__(64 * sym_waves(NB, MODE, SHAPE)) __attribute__((amdgpu_waves_per_eu(sym_waves(NB, MODE, SHAPE) > 8 ? 6 : NB == 8 ? 4 : 1)))
void k_tile_sym(
    const TileJob *__restrict__ jobs, const float *__restrict__ X, int d, int dp, const float *__restrict__ centroid,
    int nleaf, int64_t stride_tree, const float2 *__restrict__ nrm, const int32_t *__restrict__ pt, BoundCoef bc,
    int exclude_self, TileOut out) {
    constexpr bool ALT = (SHAPE & 1) != 0;
    using C = SymCfg<PREC, ALT>;
    using T = typename C::T;
    constexpr int M = 32 * NB;
    constexpr int NW = sym_waves(NB, MODE, SHAPE);
    constexpr int NT = 64 * NW;
    constexpr int PAIR = NB + 1;
    constexpr int WPP = NB >= 2 ? NW / (NB / 2) : 1;  // waves per pair of block rows
    constexpr int SLOTS = NB >= 2 ? (PAIR + WPP - 1) / WPP : 1;
    constexpr bool SPLIT = PREC == RPF_DIST_BF16X3;   // hi and lo tiles, three products per step
    // queue entries per wave (LDS for two blocks)
    constexpr int QL = (SHAPE & 2) ? 256 : NW > 8 ? (SPLIT ? 352 : 384) : kQueue;
    // one LDS area: the operand tile(s) during the k loop, then the Phase II queues or the
    // Phase I transposes
    // LDS: the operand tile(s) during the k loop, whose space then holds the Phase II queues
    // or the Phase I transposes; and the raw tile, a separate array so that the operand
    // tile's reads need not wait for the next chunk's loads into it
    static_assert(!C::DMA || C::KC == 32, "the raw tile's row groups are 32 binary32 columns");
    constexpr size_t kTileBytes = (size_t)(SPLIT ? 2 : 1) * M * C::LDW * sizeof(T);
    constexpr size_t kQueBytes = MODE >= 1 ? (size_t)NW * QL * sizeof(uint2) : 0;
    constexpr size_t kTrBytes = MODE == 0 ? (size_t)NW * 32 * 33 * sizeof(float) : 0;
    constexpr size_t kBuf = kTileBytes > kQueBytes ? (kTileBytes > kTrBytes ? kTileBytes : kTrBytes)
                                                   : (kQueBytes > kTrBytes ? kQueBytes : kTrBytes);
    __shared__ __align__(16) uint8_t s_buf[kBuf];
    __shared__ __align__(16) float s_raw[C::DMA ? M * C::KC : 1];
    T *s_a = reinterpret_cast<T *>(s_buf);
    __shared__ __align__(16) float s_n[M];
    __shared__ __align__(16) float s_r[M];
    __shared__ __align__(16) float s_phi[M];
    __shared__ float s_tau[M];
    __shared__ int32_t s_pt[M];
    __shared__ float s_max[2];
    __shared__ int32_t s_cnt[MODE == 2 ? M : 1];  // bucket mode: records of each row so far

    const TileJob job = jobs[blockIdx.x];
    const int t = job.tree;
    const int m = job.a_rows;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wu = __builtin_amdgcn_readfirstlane(w);  // wave-uniform (scalar) wave index
    const float *mu = centroid + ((int64_t)t * nleaf + job.leaf) * d;
    const float2 *an = nrm + t * stride_tree + job.a_off;
    const int32_t *ap = pt + t * stride_tree + job.a_off;
    const int tb = t - out.t0;
    if (MODE == 0 && m > out.ML) {  // as in k_tile: the rows take the exhaustive path
        for (int r = tid; r < m; r += NT) out.roff[(int64_t)tb * out.nrows + ap[r]] = -1;
        return;
    }
    for (int r = tid; r < M; r += NT) {
        if (r < m) {
            const float2 q = an[r];
            s_n[r] = q.x;
            s_r[r] = q.y;
            const int p = ap[r];
            s_pt[r] = p;
            s_tau[r] = MODE >= 1 ? out.tau[p] : INFINITY;
        } else {
            s_n[r] = 0.f;
            s_r[r] = 0.f;
            s_pt[r] = -1;
            s_tau[r] = -1.f;
        }
        if constexpr (MODE == 2) s_cnt[r] = 0;
    }
    __syncthreads();
    // rows of 16-byte multiples: the first chunk's rows go straight to LDS while the rest of
    // the set-up runs
    const bool dma = C::DMA && (d % 4) == 0;
    if (dma) issue_rows_dma(s_raw, X, d, s_pt, m, 0, wu, NW);
    if (tid < 64) {
        float mn = 0.f, mr = 0.f;
        for (int r = lane; r < m; r += 64) {
            mn = fmaxf(mn, s_n[r]);
            mr = fmaxf(mr, s_r[r]);
        }
        for (int o = 32; o > 0; o >>= 1) {
            mn = fmaxf(mn, __shfl_xor(mn, o, 64));
            mr = fmaxf(mr, __shfl_xor(mr, o, 64));
        }
        if (lane == 0) {
            s_max[0] = mn;
            s_max[1] = mr;
        }
    }
    __syncthreads();
    for (int r = tid; r < M; r += NT) s_phi[r] = cheap_phi(s_tau[r], s_n[r], s_r[r], s_max[0], s_max[1], bc);
    if constexpr (MODE == 0) {  // Phase I: the slots no pair fills (past the leaf, and self)
        for (int r = tid; r < m; r += NT) {
            const int64_t er = (int64_t)s_pt[r] * out.cap + (int64_t)tb * out.ML;
            for (int c = m; c < out.ML; c++) put_first_empty(out, er + c);
            if (exclude_self) put_first_empty(out, er + r);
            out.roff[(int64_t)tb * out.nrows + s_pt[r]] = (int32_t)job.a_off;
        }
    }

    // scalar block coordinates of every slot of this wave; act = the block holds leaf rows
    int sbi[SLOTS], sbj[SLOTS];
    bool act[SLOTS];
#pragma unroll
    for (int sl = 0; sl < SLOTS; sl++) {
        int bi = -1, bj = -1;
        if (NB == 1) {
            bi = bj = 0;
        } else {
            const int p = wu / WPP, q = (wu % WPP) * SLOTS + sl;
            const int r1 = p, r2 = NB - 1 - p, len1 = NB - r1;
            if (q < len1) {
                bi = r1;
                bj = r1 + q;
            } else if (q < PAIR) {
                bi = r2;
                bj = r2 + (q - len1);
            }
        }
        act[sl] = bj >= 0 && 32 * bj < m;
        // a slot past the pair repeats the block row before it, so that a wave's slots name
        // at most two block rows, in order (the K loop loads one A fragment per row)
        sbi[sl] = bi >= 0 ? bi : sl > 0 ? sbi[sl - 1] : 0;
        sbj[sl] = bj < 0 ? 0 : bj;
    }
    f32x16 acc[SLOTS];
#pragma unroll
    for (int sl = 0; sl < SLOTS; sl++)
#pragma unroll
        for (int v = 0; v < 16; v++) acc[sl][v] = 0.f;
    const int fr = lane & 31;
    const int fk = PREC == RPF_DIST_FP32 ? (lane >> 5) : 8 * (lane >> 5);
    for (int k0 = 0; k0 < dp; k0 += C::KC) {
        if (dma) {
            __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of the chunk are in LDS
            __syncthreads();                 // and every wave's; the last chunk's MFMA reads are done
            convert_rows<PREC>(s_a, s_raw, d, mu, m, M, k0, NT, s_a + (SPLIT ? M * C::LDW : 0));
            __syncthreads();  // operand tile complete, raw tile free: the next chunk's loads fly
            if (k0 + C::KC < dp) issue_rows_dma(s_raw, X, d, s_pt, m, k0 + C::KC, wu, NW);
        } else {
            __syncthreads();
            if (d % 4 == 0) stage_rows_x<PREC, true, ALT>(s_a, X, d, s_pt, mu, m, M, k0, NT, s_a + (SPLIT ? M * C::LDW : 0));
            else stage_rows_x<PREC, false, ALT>(s_a, X, d, s_pt, mu, m, M, k0, NT, s_a + (SPLIT ? M * C::LDW : 0));
            __syncthreads();
        }
        int kmax = dp - k0 < C::KC ? dp - k0 : C::KC;
        kmax = (kmax + C::KSTEP - 1) / C::KSTEP * C::KSTEP;
        const T *base = s_a + fr * C::LDW + fk;
        using Frag = typename MfmaOperand<PREC>::type;
        for (int kk = 0; kk < kmax; kk += C::KSTEP) {
            // all fragment loads of the step first, then the MFMAs; a wave's slots lie in at
            // most two block rows (bi0 for the first ones, bi1 after), so two A fragments
            Frag fa0, fa1, fb[SLOTS];
            fa0 = *reinterpret_cast<const Frag *>(base + 32 * sbi[0] * C::LDW + kk);
            fa1 = *reinterpret_cast<const Frag *>(base + 32 * sbi[SLOTS - 1] * C::LDW + kk);
#pragma unroll
            for (int sl = 0; sl < SLOTS; sl++) fb[sl] = *reinterpret_cast<const Frag *>(base + 32 * sbj[sl] * C::LDW + kk);
            // (split: every slot's MFMA runs -- an inactive slot's accumulator is never read --
            // so that the three passes stay one basic block and the accumulators in registers)
#pragma unroll
            for (int sl = 0; sl < SLOTS; sl++)
                if (SPLIT || act[sl]) acc[sl] = mfma_op<PREC>(sbi[sl] == sbi[0] ? fa0 : fa1, fb[sl], acc[sl]);
            if constexpr (SPLIT) {
                // hi_a . lo_b, then lo_a . hi_b: at most five fragments live at a time (the
                // scheduling barriers keep the next pass's loads behind this pass's MFMAs)
                const T *lo = base + M * C::LDW;
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int sl = 0; sl < SLOTS; sl++) fb[sl] = *reinterpret_cast<const Frag *>(lo + 32 * sbj[sl] * C::LDW + kk);
#pragma unroll
                for (int sl = 0; sl < SLOTS; sl++)
                    acc[sl] = mfma_op<PREC>(sbi[sl] == sbi[0] ? fa0 : fa1, fb[sl], acc[sl]);
                __builtin_amdgcn_sched_barrier(0);
                fa0 = *reinterpret_cast<const Frag *>(lo + 32 * sbi[0] * C::LDW + kk);
                fa1 = *reinterpret_cast<const Frag *>(lo + 32 * sbi[SLOTS - 1] * C::LDW + kk);
#pragma unroll
                for (int sl = 0; sl < SLOTS; sl++) fb[sl] = *reinterpret_cast<const Frag *>(base + 32 * sbj[sl] * C::LDW + kk);
#pragma unroll
                for (int sl = 0; sl < SLOTS; sl++)
                    acc[sl] = mfma_op<PREC>(sbi[sl] == sbi[0] ? fa0 : fa1, fb[sl], acc[sl]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }

    if constexpr (MODE == 0) {
        // (row -> col) slots: lanes hold consecutive columns, so each store covers 128-byte
        // runs of a row.  (col -> row) slots go through a per-wave 32 x 33 LDS transpose in
        // the operand tile, which every wave has finished reading: then each store covers a
        // 128-byte run of a column's row as well.
        __syncthreads();  // every wave is done with the operand tile: its space holds the transposes
        float *tr = reinterpret_cast<float *>(s_buf) + wu * (32 * 33);
#pragma unroll
        for (int sl = 0; sl < SLOTS; sl++) {
            if (!act[sl]) continue;
            const int bi = sbi[sl], bj = sbj[sl];
            const bool diag = bi == bj;
            const int cl = lane & 31, col = 32 * bj + cl;
            const bool colok = col < m;
            const float ncol = s_n[colok ? col : 0], rcol = s_r[colok ? col : 0];
            float lbv[16], ubv[16];
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int rl = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), row = 32 * bi + rl;
                const bool rowok = row < m;
                pair_bounds(s_n[rowok ? row : 0], ncol, s_r[rowok ? row : 0], rcol, acc[sl][v], bc, lbv[v], ubv[v]);
                if (colok && rowok && !(diag && (row > col || (row == col && exclude_self))))
                    put_first(out, (int64_t)s_pt[row] * out.cap + (int64_t)tb * out.ML + col, lbv[v], ubv[v]);
            }
            // transposed: output row = column c of the block, positions 32 bi + r; the packed
            // bounds go through the transpose and are stored
            uint32_t *tru = reinterpret_cast<uint32_t *>(tr);
            wave_sync();
#pragma unroll
            for (int v = 0; v < 16; v++)
                tru[cl * 33 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)] = pack_bounds(lbv[v], ubv[v]);
            wave_sync();
#pragma unroll
            for (int c0 = 0; c0 < 32; c0 += 2) {
                const int c = c0 + (lane >> 5), r = lane & 31;
                const int cg = 32 * bj + c, rg = 32 * bi + r;
                if (cg < m && rg < m && rg != cg && !(diag && rg > cg))
                    out.plub[(int64_t)s_pt[cg] * out.cap + (int64_t)tb * out.ML + rg] = tru[c * 33 + r];
            }
        }
        return;
    }
    if constexpr (MODE >= 1) {
        // Phase II: a cheap test over every pair (both directions); the pairs that pass are
        // compacted by ballot into a per-wave LDS queue, whose exact bounds and emissions
        // run when it would overflow and at the end (wave-uniform decisions throughout)
        __syncthreads();  // every wave is done with the operand tile: its space holds the queues
        uint2 *que = reinterpret_cast<uint2 *>(s_buf) + (size_t)wu * QL;
        uint32_t qc = 0;
        constexpr bool bucket = MODE == 2;
        const int tb2 = t - out.t1;
        auto flush = [&](uint32_t nq) {
            wave_sync();
            for (uint32_t i = lane; i < nq; i += 64) {
                const uint2 e = que[i];
                const int row = e.x & 255, col = (e.x >> 8) & 255;
                float lb, ub;
                pair_bounds(s_n[row], s_n[col], s_r[row], s_r[col], __uint_as_float(e.y), bc, lb, ub);
                if constexpr (bucket) {
                    if (((e.x >> 16) & 1) && lb <= s_tau[row]) emit_bucket(out, s_cnt, row, tb2, s_pt[row], s_pt[col], lb, ub);
                    if (((e.x >> 17) & 1) && lb <= s_tau[col]) emit_bucket(out, s_cnt, col, tb2, s_pt[col], s_pt[row], lb, ub);
                } else {
                    if (((e.x >> 16) & 1) && lb <= s_tau[row]) emit_filtered(out, s_pt[row], s_pt[col], lb, ub);
                    if (((e.x >> 17) & 1) && lb <= s_tau[col]) emit_filtered(out, s_pt[col], s_pt[row], lb, ub);
                }
            }
            wave_sync();
        };
#pragma unroll
        for (int sl = 0; sl < SLOTS; sl++) {
            if (!act[sl]) continue;
            const int bi = sbi[sl], bj = sbj[sl];
            const bool diag = bi == bj;
            const int col = 32 * bj + (lane & 31);  // < M: rows past the leaf hold n = 0, phi = -inf
            const bool colok = col < m;
            const float ncol = s_n[col];
            const float phicol = s_phi[col];
            const bool inner = !diag && 32 * bi + 32 <= m && 32 * bj + 32 <= m;  // wave-uniform
#pragma unroll
            for (int h = 0; h < 2; h++) {
                // the half's 8 rows of this lane come in two runs of four: their norms and
                // thresholds are read up front, so the tests below are branch-free register work
                float nr[8], pr[8];
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    const int r0 = 32 * bi + 8 * (2 * h + j) + 4 * (lane >> 5);
                    const float4 n4 = *reinterpret_cast<const float4 *>(s_n + r0);
                    const float4 p4 = *reinterpret_cast<const float4 *>(s_phi + r0);
                    nr[4 * j] = n4.x; nr[4 * j + 1] = n4.y; nr[4 * j + 2] = n4.z; nr[4 * j + 3] = n4.w;
                    pr[4 * j] = p4.x; pr[4 * j + 1] = p4.y; pr[4 * j + 2] = p4.z; pr[4 * j + 3] = p4.w;
                }
                uint32_t bits = 0;  // (p1, p2) of the 8 values of this half, two bits each
                uint64_t mk[8];
                uint32_t tot = 0;
                if (inner) {  // off the diagonal, every row and column real: the two tests alone
#pragma unroll
                    for (int v8 = 0; v8 < 8; v8++) {
                        const float g = acc[sl][8 * h + v8];
                        const bool p1 = __builtin_fmaf(-2.f, g, ncol) <= pr[v8];
                        const bool p2 = __builtin_fmaf(-2.f, g, nr[v8]) <= phicol;
                        bits |= ((p1 ? 1u : 0u) | (p2 ? 2u : 0u)) << (2 * v8);
                        mk[v8] = __ballot(p1 || p2);
                        tot += (uint32_t)__popcll(mk[v8]);
                    }
                } else {
#pragma unroll
                    for (int v8 = 0; v8 < 8; v8++) {
                        const int v = 8 * h + v8;
                        const int row = 32 * bi + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                        const float g = acc[sl][v];
                        // row -> col needs a real column and, on the diagonal block, row <= col
                        // (row < col when the point itself is excluded); col -> row needs a real
                        // row and, on the diagonal block, row < col
                        const bool p1 = colok & (__builtin_fmaf(-2.f, g, ncol) <= pr[v8]) &
                                        !(diag & ((row > col) | ((row == col) & (exclude_self != 0))));
                        const bool p2 =
                            (!diag | (row < col)) & (row < m) & (__builtin_fmaf(-2.f, g, nr[v8]) <= phicol);
                        bits |= ((p1 ? 1u : 0u) | (p2 ? 2u : 0u)) << (2 * v8);
                        mk[v8] = __ballot(p1 || p2);
                        tot += (uint32_t)__popcll(mk[v8]);
                    }
                }
                if (qc + tot > (uint32_t)QL) {
                    flush(qc);
                    qc = 0;
                }
#pragma unroll
                for (int v8 = 0; v8 < 8; v8++) {
                    const int v = 8 * h + v8;
                    const uint32_t f = (bits >> (2 * v8)) & 3u;
                    if (f) {
                        const int row = 32 * bi + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                        que[qc + mask_rank(mk[v8])] =
                            make_uint2((uint32_t)row | ((uint32_t)col << 8) | (f << 16), __float_as_uint(acc[sl][v]));
                    }
                    qc += (uint32_t)__popcll(mk[v8]);
                }
            }
        }
        flush(qc);
        if constexpr (bucket) {  // every wave has emitted: the bucket counts of the block's rows
            __syncthreads();
            for (int r = tid; r < m; r += NT)
                out.bcnt[(int64_t)s_pt[r] * out.nT2 + tb2] = (uint8_t)min(s_cnt[r], out.S);
        }
    }
}

// Query tiles for small groups: a group of at most QS queries that reached the same leaf
// (one leaf block), against every row of the block.  One wave per job, eight lanes per
// candidate row (16-byte coalesced reads straight from HBM), each lane keeping its fixed
// share of the group's centred query copy in registers; the 8-lane partial products are
// combined by shuffles.  Same stored operands and the same rigorous bounds as the MFMA
// tiles (products of two tile-precision values accumulated in binary32, any order), and
// the same outputs: Phase I fixed slots (mode 0) or records below the row's threshold
// (mode 1).  A GEMV-shaped job moves the leaf block once per query group and does no MFMA
// work on padding rows, which at a few queries per leaf is most of a 32-row MFMA block.
template <int PREC, int QS, int NCH>
__global__ __launch_bounds__(256) void k_qtile(const TileJob *__restrict__ jobs, int64_t njobs,
                                               const void *__restrict__ A_, const void *__restrict__ B_, int dp,
                                               int64_t a_stride_tree, int64_t b_stride_tree,
                                               const float2 *__restrict__ a_nrm, const float2 *__restrict__ b_nrm,
                                               const int32_t *__restrict__ a_dest, const int32_t *__restrict__ b_pt,
                                               BoundCoef bc, TileOut out) {
    using T = typename TileCfg<PREC>::T;
    constexpr int EPC = 16 / (int)sizeof(T);  // elements per 16-byte chunk
    const int lane = threadIdx.x & 63, g = lane & 7, grp = lane >> 3;
    const int64_t jid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (jid >= njobs) return;
    const TileJob job = jobs[jid];
    const int t = job.tree;
    const int nchunk = dp / EPC;  // 16-byte chunks per row (dp is a multiple of 8 elements);
                                  // lane g takes chunks g, g + 8, ... (<= NCH of them by the launch)
    const T *A = reinterpret_cast<const T *>(A_) + (t * a_stride_tree + job.a_off) * dp;
    const T *B = reinterpret_cast<const T *>(B_) + (t * b_stride_tree + job.b_off) * dp;
    const int na_rows = job.a_rows;  // <= QS by the launch
    float qv[NCH][EPC][QS];
#pragma unroll
    for (int ch = 0; ch < NCH; ch++)
#pragma unroll
        for (int e = 0; e < EPC; e++)
#pragma unroll
            for (int qi = 0; qi < QS; qi++) qv[ch][e][qi] = 0.f;
#pragma unroll
    for (int qi = 0; qi < QS; qi++) {
        if (qi >= na_rows) continue;
#pragma unroll
        for (int ch = 0; ch < NCH; ch++) {
            if (g + 8 * ch >= nchunk) continue;
            const uint4 v = *reinterpret_cast<const uint4 *>(A + (int64_t)qi * dp + (g + 8 * ch) * EPC);
            T pv[EPC];
            __builtin_memcpy(pv, &v, sizeof(v));  // bytes -> elements (no aliasing through pointers)
#pragma unroll
            for (int e = 0; e < EPC; e++) qv[ch][e][qi] = (float)pv[e];
        }
    }
    // this lane's query (g < rows of the group) for the bounds and the outputs
    const int qme = g < na_rows ? g : 0;
    const float2 aq = a_nrm[t * a_stride_tree + job.a_off + qme];
    const int dst = a_dest[t * a_stride_tree + job.a_off + qme];
    const float tq = out.mode == 1 ? out.tau[dst] : INFINITY;
    const int tb = t - out.t0;
    if (out.mode == 0 && job.b_pos + job.b_rows == job.leaf_m) {  // slots past the leaf
        for (int qi = 0; qi < na_rows; qi++) {
            const int dq = a_dest[t * a_stride_tree + job.a_off + qi];
            const int64_t er = (int64_t)dq * out.cap + (int64_t)tb * out.ML;
            for (int c = job.leaf_m + lane; c < out.ML; c += 64) put_first_empty(out, er + c);
            if (lane == 0) out.roff[(int64_t)tb * out.nrows + dq] = (int32_t)(job.b_off - job.b_pos);
        }
    }
    // QU groups of eight rows per pass (about eight 16-byte loads per lane): every chunk load
    // of the pass is issued before the first product (chunk addresses past the row are
    // clamped to its first chunk and their products skipped), so a wave waits on memory once
    // per 8 QU rows
    constexpr int QU = NCH >= 8 ? 1 : 8 / NCH;
    for (int r0 = 0; r0 < job.b_rows; r0 += 8 * QU) {
        uint4 v[QU][NCH];
#pragma unroll
        for (int u = 0; u < QU; u++) {
            const int r = r0 + 8 * u + grp;
            const T *row = B + (int64_t)(r < job.b_rows ? r : 0) * dp;
#pragma unroll
            for (int ch = 0; ch < NCH; ch++)
                v[u][ch] = *reinterpret_cast<const uint4 *>(row + (g + 8 * ch < nchunk ? g + 8 * ch : g) * EPC);
        }
#pragma unroll
        for (int u = 0; u < QU; u++) {
            const int r = r0 + 8 * u + grp;
            const bool rok = r < job.b_rows;
            float acc[QS];
#pragma unroll
            for (int qi = 0; qi < QS; qi++) acc[qi] = 0.f;
#pragma unroll
            for (int ch = 0; ch < NCH; ch++) {
                if (g + 8 * ch >= nchunk) continue;
                T pv[EPC];
                __builtin_memcpy(pv, &v[u][ch], sizeof(v[u][ch]));
#pragma unroll
                for (int e = 0; e < EPC; e++) {
                    const float x = (float)pv[e];
#pragma unroll
                    for (int qi = 0; qi < QS; qi++) acc[qi] = __builtin_fmaf(x, qv[ch][e][qi], acc[qi]);
                }
            }
#pragma unroll
            for (int qi = 0; qi < QS; qi++) {
                acc[qi] += __shfl_xor(acc[qi], 1, 64);
                acc[qi] += __shfl_xor(acc[qi], 2, 64);
                acc[qi] += __shfl_xor(acc[qi], 4, 64);
            }
            if (rok && g < na_rows) {
                float gq = acc[0];
#pragma unroll
                for (int qi = 1; qi < QS; qi++)
                    if (g == qi) gq = acc[qi];
                const float2 nb = b_nrm[t * b_stride_tree + job.b_off + r];
                const int bpt = b_pt[t * b_stride_tree + job.b_off + r];
                float lb, ub;
                pair_bounds(aq.x, nb.x, aq.y, nb.y, gq, bc, lb, ub);
                if (out.mode == 0)
                    put_first(out, (int64_t)dst * out.cap + (int64_t)tb * out.ML + job.b_pos + r, lb, ub);
                else if (lb <= tq)
                    emit_filtered(out, dst, bpt, lb, ub);
            }
        }
    }
}

// ---------------------------------------------------------------- wave-level selection

__device__ inline uint32_t fkey(float f) {  // non-negative floats (and +inf) order as uint32
    return __float_as_uint(f);
}

__device__ inline uint32_t wave_min_u32(uint32_t x) {
    for (int o = 32; o > 0; o >>= 1) x = min(x, (uint32_t)__shfl_xor((int)x, o, 64));
    return x;
}

__device__ inline uint32_t wave_max_u32(uint32_t x) {
    for (int o = 32; o > 0; o >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, o, 64));
    return x;
}

// An upper bound of the k-th smallest (0-based) of the keys held Q per lane (the wave holds
// more than k of them), within 2^13 key units of it: 2^-10 relative for the bit patterns of
// normal non-negative floats.  An entry that does not take part holds 0xffffffff, which is
// never below a candidate (every candidate is at most the largest valid key).  The bits the
// smallest and largest key share are fixed; each lower bit down to bit 13 is then set, from
// the top, exactly when at most k keys lie below the candidate, counted by ballots (one
// compare and one population count per entry and bit): no LDS and no atomics.  Every use
// below is a threshold whose correctness only needs a value at or above the exact one.
template <int Q, int kLow = 13>
__device__ inline uint32_t wave_kth_upper(const uint32_t (&v)[Q], int k) {
    uint32_t lo = 0xffffffffu, hi = 0;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        lo = min(lo, v[q]);
        hi = max(hi, v[q] == 0xffffffffu ? 0u : v[q]);
    }
    lo = wave_min_u32(lo);
    hi = wave_max_u32(hi);
    if (lo >= hi) return lo;
    const int hb = 31 - __builtin_clz(lo ^ hi);
    if (hb < kLow) return hi;
    uint32_t ans = hb >= 31 ? 0u : (lo & ~((2u << hb) - 1u));
    for (int b = hb; b >= kLow; b--) {
        const uint32_t t = ans | (1u << b);
        int c = 0;
#pragma unroll
        for (int q = 0; q < Q; q++) c += __popcll(__ballot(v[q] < t));
        if (c <= k) ans = t;
    }
    return min(ans | ((1u << kLow) - 1u), hi);
}

// Phase I merge (one wave per row).  The row's entries come from the first B trees, where
// every index occurs at most once per tree, so the (K*B)-th smallest ub of the multiset is
// an upper bound of tau = K-th smallest ub over distinct indices (ub of an index = its
// smallest ub), and the entries with ub below it hold every index's minimal entry that
// matters.  tau is bounded from above on that small set; the list keeps every entry with
// lb <= tau (duplicates included: the final merge removes them).  Every slot of the row is
// loaded at the start (Q per lane), so a wave waits on memory once.
// (kFirstTrees, kMergeCap, kSetCap and the slot geometry live in merge_index.h)

struct SlotIndex {  // where the index of a Phase I slot comes from: the row's leaf in the tree
    const int32_t *roff;  // [B][nrows] start of the row's leaf in the permutation
    const int32_t *perm;  // [T][n] leaf-ordered permutation
    int64_t n;
};

template <int Q, int HT>
__global__ __launch_bounds__(256) void k_merge_first(int64_t nrows, int K, int B, int ML,
                                                     const uint32_t *__restrict__ plub, SlotIndex si, int cap,
                                                     float *__restrict__ tau, Ent *__restrict__ list,
                                                     int32_t *__restrict__ lcnt, int lcap,
                                                     int32_t *__restrict__ cnt) {
    // per-wave open-addressing hash of the small set: index -> smallest (ub, slot), packed as
    // one 32-bit key (the order the representatives are defined by)
    constexpr int kHBits = HT == 512 ? 9 : HT == 1024 ? 10 : 11;
    static_assert((1 << kHBits) == HT, "hash range must equal the table");
    static_assert(64 * Q <= 65536, "a slot number fits the lower half of the key");
    // the kept ub is the upper half of a binary32 pattern, so (ub bits | slot) orders entries
    // by (ub, slot) in one 32-bit key (slots < 2^11)
    __shared__ int32_t s_hid[4][HT];
    __shared__ uint32_t s_hkey[4][HT];
    __shared__ uint32_t s_sm[4][2][HT / 2];  // the compacted small set of each wave: key, index
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t a = (int64_t)blockIdx.x * 4 + w;
    if (a >= nrows) return;
    const int c = B * ML;  // fixed slots of the first B trees
    // A row that takes the exhaustive path gets a negative threshold: no later tile emits a
    // record for it (lb >= 0), since the exhaustive scan does not read them.
    if (c > 64 * Q) {      // leaves above kMergeCap points: the row takes the exhaustive path
        if (lane == 0) {
            lcnt[a] = lcap + 1;
            tau[a] = -1.f;
            cnt[a] = 0;
        }
        return;
    }
    // the row's leaf in each of the B trees: lane t holds its start in the permutation
    const int32_t loff = lane < B ? si.roff[(int64_t)lane * nrows + a] : 0;
    // ML is a multiple of 64, so the slots of wave-wide column q all lie in tree q / (ML / 64):
    // the tree, its leaf start and the column offset are the same for every lane.  The index
    // arithmetic is that of merge_index.h, which a host-only test replays.
    const int ncol = first_slot_cols(B, ML);  // wave-wide slot columns of the row
    uint32_t u[Q];  // ub bits of the finite slots, 0xffffffff for the others
    float l[Q];
    int32_t id[Q];  // -1 for a slot that no pair fills (lb = +inf)
    FirstSlotCursor cur;  // tree of column q, and its first slot's position in the leaf
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const bool in = q < ncol;  // lane + 64 q < c for every lane
        const uint32_t e = in ? plub[first_slot_addr(a, cap, lane, q)] : 0x7f807f80u;  // packed bounds
        const uint32_t ub = e & 0xffff0000u;                                             // fkey of the ub kept
        const float lb = __uint_as_float(e << 16);
        u[q] = ub < 0x7f800000u ? ub : 0xffffffffu;
        l[q] = lb;
        const int32_t off = __builtin_amdgcn_readlane(loff, in ? cur.tree : 0);
        // the permutation entry is read whatever the slot holds (clamped into the tree), so
        // that it does not wait for the slot's bounds; an empty slot drops it
        const int32_t pos = first_slot_perm_pos(off, cur.col0, lane, si.n);
        const int32_t pv = in ? si.perm[(int64_t)cur.tree * si.n + pos] : -1;
        id[q] = lb < INFINITY ? pv : -1;
        first_slot_next(cur, ML);
    }
    for (int i = lane; i < HT; i += 64) {
        s_hid[w][i] = -1;
        s_hkey[w][i] = 0xffffffffu;
    }
    int nv = 0;  // finite-ub slots (empty slots hold +inf bounds)
#pragma unroll
    for (int q = 0; q < Q; q++) nv += __popcll(__ballot(u[q] != 0xffffffffu));
    const int kb = K * B;
    // theta only bounds the small set from above: 2^-5 relative is close enough
    const uint32_t theta = nv >= kb ? wave_kth_upper<Q, 18>(u, kb - 1) : 0x7f800000u;
    // the small set S = {finite slots with ub <= theta}, each entry hashed by its index
    int ns = 0;
#pragma unroll
    for (int q = 0; q < Q; q++) ns += __popcll(__ballot(u[q] <= theta));
    // a leaf start of -1: the row's leaf in a first-phase tree was above the slot stride, its
    // slots were not written (the row takes the exhaustive path)
    const bool over = ns > HT / 2 || __ballot(lane < B && loff < 0) != 0;
    float tv = INFINITY;
    if (!over) {
        // the small set compacted to the front of per-wave staging arrays ((ub, slot) key,
        // index), so the hash inserts and the representative tests below run over at most
        // HT / 128 entries per lane rather than over all Q slots
        uint32_t *s_sk = s_sm[w][0];
        int32_t *s_si = reinterpret_cast<int32_t *>(s_sm[w][1]);
        {
            int base = 0;
#pragma unroll
            for (int q = 0; q < Q; q++) {
                const bool in = u[q] <= theta;
                const uint64_t mk = __ballot(in);
                if (in) {
                    const int p = base + mask_rank(mk);
                    s_sk[p] = u[q] | (uint32_t)(lane + 64 * q);
                    s_si[p] = id[q];
                }
                base += __popcll(mk);
            }
        }
        wave_sync();  // the staged set and the cleared table are visible
        constexpr int KS = HT / 128;  // ns <= HT / 2
        int hq[KS];
        uint32_t kq[KS];
#pragma unroll
        for (int k = 0; k < KS; k++) {
            const int i = lane + 64 * k;
            hq[k] = -1;
            kq[k] = 0xffffffffu;
            if (i < ns) {
                kq[k] = s_sk[i];
                const int32_t idk = s_si[i];
                int h = (int)(((uint32_t)idk * 2654435761u) >> (32 - kHBits));
                while (true) {  // at most half full: a free or matching entry is always found
                    const int prev = atomicCAS(&s_hid[w][h], -1, idk);
                    if (prev == -1 || prev == idk) break;
                    h = (h + 1) & (HT - 1);
                }
                atomicMin(&s_hkey[w][h], kq[k]);
                hq[k] = h;
            }
        }
        wave_sync();
        // representatives: the entry of smallest (ub, slot) among equal indices; their ub keys
        // are compacted into the (now free) id column of the table, HT / 2 at most, and read
        // back HT / 128 per lane for the selection
        bool rep[KS];
#pragma unroll
        for (int k = 0; k < KS; k++) rep[k] = hq[k] >= 0 && s_hkey[w][hq[k]] == kq[k];
        wave_sync();  // every lookup is done before the id column is overwritten
        uint32_t *s_rv = reinterpret_cast<uint32_t *>(s_hid[w]);
        int nrep = 0;
#pragma unroll
        for (int k = 0; k < KS; k++) {
            const uint64_t mk = __ballot(rep[k]);
            if (rep[k]) s_rv[nrep + mask_rank(mk)] = kq[k] & 0xffff0000u;
            nrep += __popcll(mk);
        }
        wave_sync();
        constexpr int RQ = HT / 128;
        uint32_t rv[RQ];
#pragma unroll
        for (int q = 0; q < RQ; q++) {
            const int i = lane + 64 * q;
            rv[q] = i < nrep ? s_rv[i] : 0xffffffffu;
        }
        if (nrep >= K) tv = __uint_as_float(wave_kth_upper<RQ>(rv, K - 1));
    }
    const float tp = tv * (1.f + 1e-6f);
    uint32_t kept = 0;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int i = lane + 64 * q;
        // validity of a slot comes from its index (-1 marks an empty one), never from its
        // bounds: a pair outside the copy's range carries lb = 0, ub = +inf and is kept
        const bool keep = !over && i < c && l[q] <= tp && id[q] >= 0;
        const uint64_t mk = __ballot(keep);
        const uint32_t pos = kept + mask_rank(mk);
        if (keep && pos < (uint32_t)lcap)
            list[a * lcap + pos] = make_ent(id[q], l[q], __uint_as_float(u[q] == 0xffffffffu ? 0x7f800000u : u[q]));
        kept += __popcll(mk);
    }
    if (lane == 0) {
        lcnt[a] = over ? lcap + 1 : (int32_t)kept;
        tau[a] = over ? -1.f : tp;
        cnt[a] = 0;
    }
}

// ---------------------------------------------------------------- final merge and rerank

constexpr int kListCap = 256;              // Phase I list records per row
constexpr int kFinalQ = 12;                // entries per lane of the widest k_final in common use
constexpr int kFinalCap = 64 * kFinalQ;    // list + emissions per row handled by k_final
constexpr int kBigQ = 16;                  // records per thread of the block-per-row merge
constexpr int kBigCap = 256 * kBigQ;       // list + Phase II records per row it handles

struct FinalArgs {
    const Ent *list;
    const int32_t *lcnt;
    int lcap;
    const int32_t *cnt;
    const Ent *ent;
    int cap;
    int K;
    const float *X;     // data rows [n][d]
    const float *Qr;    // query rows [nrows][d] (X itself for all-points)
    int d;
    float win;          // relative window on D32 for the binary64 re-rank
    int32_t *out_idx;
    float *out_dist;
    int32_t *fb_list;   // rows for the exhaustive fallback
    int32_t *fb_cnt;
    int32_t *big_list;  // rows past the wave merge's records for the block merge (nullptr: none)
    int32_t *big_cnt;
    int64_t npts;       // rows of X: every candidate index lies in [0, npts)
    const uint8_t *bcnt;  // bucket mode (see TileOut): bucket counts [rows][nT2]; nullptr = one counted list
    int S;              // bucket mode: records per bucket
    int nT2;            // bucket mode: buckets (Phase II trees) per row, at most 128
    int capO;           // bucket mode: overflow records per row (cnt counts them)
    unsigned long long *stats;  // [kStatSlots][8]: rows, fallback, reranked32, reranked64, bad_index,
                                //                 kept1, emitted2, block-merged (summed over slots by the host)
    unsigned long long *fault;  // the forest's sticky count of rows that met a bad index
};

// counters are spread over slots by block so that a million rows do not meet on one address
__device__ inline void stat_add(const FinalArgs &A, int i, unsigned long long v) {
    atomicAdd(&A.stats[(blockIdx.x & (kStatSlots - 1)) * 8 + i], v);
}

__device__ inline void push_fallback(const FinalArgs &A, int64_t a) {
    const int slot = atomicAdd(A.fb_cnt, 1);
    A.fb_list[slot] = (int32_t)a;
    stat_add(A, 1, 1ull);
}

// A row the wave merge cannot hold goes to the block merge when its records fit the buffers
// (ovf: the Phase II records overflowed) and the block's kBigCap, else to the exhaustive
// fallback.
__device__ inline void push_overflow(const FinalArgs &A, int64_t a, int c1, int c2, bool ovf) {
    if (A.big_list && c1 <= A.lcap && !ovf && c1 + c2 <= kBigCap) {
        const int slot = atomicAdd(A.big_cnt, 1);
        A.big_list[slot] = (int32_t)a;
        stat_add(A, 7, 1ull);
    } else {
        push_fallback(A, a);
    }
}

// Bucket mode: the Phase II records of row a are bucket b = 0 .. nT2 - 1 (bcnt[a][b] records
// at a * cap + b * S), then the overflow list.  The wave's lanes read the counts of buckets
// lane and lane + 64 and scan them: s_pre[b] = the number of bucket b's first record in the
// row's sequence; s_own[j] = the bucket of record j, for j < room.  Returns the bucket
// records' total.
__device__ inline int bucket_tables_wave(const FinalArgs &A, int64_t a, int lane, int32_t *s_pre, uint8_t *s_own,
                                         int room) {
    const uint8_t *bc = A.bcnt + a * A.nT2;
    const int n0 = lane < A.nT2 ? bc[lane] : 0;
    const int n1 = lane + 64 < A.nT2 ? bc[lane + 64] : 0;
    int x0 = n0, x1 = n1;
    for (int o = 1; o < 64; o <<= 1) {
        const int y0 = __shfl_up(x0, o, 64), y1 = __shfl_up(x1, o, 64);
        if (lane >= o) {
            x0 += y0;
            x1 += y1;
        }
    }
    const int t0 = __shfl(x0, 63, 64);
    const int P = t0 + __shfl(x1, 63, 64);
    const int e0 = x0 - n0, e1 = t0 + x1 - n1;
    if (lane < A.nT2) s_pre[lane] = e0;
    if (lane + 64 < A.nT2) s_pre[lane + 64] = e1;
    for (int k = 0; k < n0 && e0 + k < room; k++) s_own[e0 + k] = (uint8_t)lane;
    for (int k = 0; k < n1 && e1 + k < room; k++) s_own[e1 + k] = (uint8_t)(lane + 64);
    wave_sync();
    return P;
}

// Phase II record j of row a (j below the row's count; P = the bucket records' total)
__device__ inline Ent phase2_rec(const FinalArgs &A, int64_t a, int j, int P, const int32_t *s_pre,
                                 const uint8_t *s_own) {
    if (!A.bcnt) return A.ent[a * A.cap + j];
    if (j < P) {
        const int b = s_own[j];
        return A.ent[a * A.cap + (int64_t)b * A.S + (j - s_pre[b])];
    }
    return A.ent[a * A.cap + (int64_t)A.nT2 * A.S + (j - P)];
}

// The Phase II record count of row a and whether its buffers overflowed.
__device__ inline void phase2_count(const FinalArgs &A, int64_t a, int P, int &c2, bool &ovf) {
    const int c = A.cnt[a];
    if (A.bcnt) {
        ovf = c > A.capO;
        c2 = P + min(c, A.capO);
    } else {
        ovf = c > A.cap;
        c2 = c;
    }
}

// The steps of k_final for one row once its records are counted: Q records per lane in
// registers, an index hash of HT entries in LDS (s_key), the per-slot ub minima and then R in
// s_r and s_d (HT / 2 each, contiguous), the compacted selection keys in s_c (256), the query
// row in s_q.
template <bool VEC, int Q, int HT>
__device__ __attribute__((always_inline)) inline void final_row(const FinalArgs &A, int64_t a, int lane,
                                                                int32_t *s_key, int32_t *s_r, uint32_t *s_d,
                                                                const float *s_q, int c1, int c2, int P,
                                                                const int32_t *s_pre, const uint8_t *s_own,
                                                                uint32_t *s_c) {
    constexpr int kHT = HT;
    constexpr int kHBits = HT == 512 ? 9 : HT == 1024 ? 10 : 11;  // log2(kHT): the hash keeps that many top bits
    static_assert((1 << kHBits) == kHT, "hash range must equal the table");
    constexpr int kRCap = kHT / 2;
    const int K = A.K;
    int nd = 0;
    bool bad = false;  // an index outside [0, npts) is an internal error, never dereferenced
    Ent ev[Q];   // every record of the row is loaded first: the wave waits on memory once
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int i = lane + 64 * q;
        ev[q] = i < c1 + c2 ? (i < c1 ? A.list[a * A.lcap + i] : phase2_rec(A, a, i - c1, P, s_pre, s_own))
                            : invalid_rec();
    }
    // the bucket tables are read: R's area (s_r, s_d) holds the per-slot ub minima during the
    // dedup
    uint32_t *s_ubn = reinterpret_cast<uint32_t *>(s_r);
    wave_sync();
    for (int k = lane; k < kHT; k += 64) s_ubn[k] = 0xffffffffu;
    wave_sync();
    // Dedup by index: the first copy of an index claims a hash slot; the slot keeps the
    // smallest ub of the index's copies (every copy's interval holds the index's distance).
    // tau' = the K-th smallest of those, and R = the indices with a copy whose lb <= tau':
    // both are functions of the set of copies, so they do not depend on which copy of an
    // index came first.
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const Ent e = ev[q];
        bad |= e.idx < -1 || (int64_t)e.idx >= A.npts;
        bool fst = false;
        if (e.idx >= 0 && (int64_t)e.idx < A.npts) {
            uint32_t h = ((uint32_t)e.idx * 2654435761u) >> (32 - kHBits);
            while (true) {
                const int old = atomicCAS(&s_key[h], -1, e.idx);
                if (old == -1) {
                    fst = true;
                    break;
                }
                if (old == e.idx) break;
                h = (h + 1) & (kHT - 1);
            }
            atomicMin(&s_ubn[h], fkey(e.ub));
        }
        nd += __popcll(__ballot(fst));
    }
    wave_sync();
    if (__ballot(bad)) {  // counted for the host to report; the row is recomputed exhaustively
        if (lane == 0) {
            stat_add(A, 4, 1ull);
            atomicAdd(A.fault, 1ull);
            push_fallback(A, a);
        }
        return;
    }
    // The distinct indices are the occupied slots.  tau' = the K-th smallest of their ub: in
    // the usual case (at most 256 indices) over their ub keys compacted four per lane (s_c),
    // else over the NS slots per lane (an empty slot reads as the largest key).
    constexpr int NS = kHT / 64;
    float tv = INFINITY;
    if (nd >= K && nd <= 256) {
        int nf = 0;
#pragma unroll
        for (int k = 0; k < NS; k++) {
            const int slot = lane + 64 * k;
            const bool occ = s_key[slot] != -1;
            const uint64_t mk = __ballot(occ);
            if (occ) s_c[nf + mask_rank(mk)] = s_ubn[slot];
            nf += __popcll(mk);
        }
        wave_sync();
        uint32_t fu[4];
#pragma unroll
        for (int q = 0; q < 4; q++) fu[q] = lane + 64 * q < nd ? s_c[lane + 64 * q] : 0xffffffffu;
        tv = __uint_as_float(wave_kth_upper<4>(fu, K - 1));
    } else if (nd >= K) {
        uint32_t fu[NS];
#pragma unroll
        for (int k = 0; k < NS; k++) {
            const int slot = lane + 64 * k;
            fu[k] = s_key[slot] != -1 ? s_ubn[slot] : 0xffffffffu;
        }
        tv = __uint_as_float(wave_kth_upper<NS>(fu, K - 1));
    }
    const uint32_t tp = fkey(tv * (1.f + 1e-6f));
    // a copy with lb <= tau' (a few per row) marks its index for R, in the top bit of the
    // slot's ub key, which a non-negative float's key never sets
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const Ent e = ev[q];
        if (e.idx >= 0 && fkey(e.lb) <= tp) {
            uint32_t h = ((uint32_t)e.idx * 2654435761u) >> (32 - kHBits);
            while (s_key[h] != e.idx) h = (h + 1) & (kHT - 1);
            atomicOr(&s_ubn[h], 0x80000000u);
        }
    }
    wave_sync();
    int32_t sid[NS];  // the slots' indices, -1 where empty or not in R
#pragma unroll
    for (int k = 0; k < NS; k++) {
        const int slot = lane + 64 * k;
        const int32_t id = s_key[slot];
        sid[k] = (id != -1 && (s_ubn[slot] >> 31)) ? id : -1;
    }
    wave_sync();  // the ub keys are read: R takes their area
    int nr = 0;   // rerank set R
#pragma unroll
    for (int k = 0; k < NS; k++) {
        const bool in = sid[k] != -1;
        const uint64_t mk = __ballot(in);
        const int pos = nr + mask_rank(mk);
        if (in && pos < kRCap) s_r[pos] = sid[k];
        nr += __popcll(mk);
    }
    wave_sync();
    if (nr > kRCap) {
        if (lane == 0) push_fallback(A, a);
        return;
    }
    // the canonical binary64 distance of every member of R (R is small: about K rows), so
    // the K best by (D64, index) come straight from R; the hash table is dead by now and
    // holds the binary64 values
    double *s_dd = reinterpret_cast<double *>(s_key);  // kHT int32 = kRCap doubles
    const int g = lane & 7, grp = lane >> 3;
    if constexpr (VEC) {  // two candidates per group of eight lanes at a time
        for (int base = 0; base < nr; base += 16) {
            const int i0 = base + grp, i1 = i0 + 8;
            const int b0 = s_r[i0 < nr ? i0 : 0], b1 = s_r[i1 < nr ? i1 : 0];
            double D64[2];
            group8_dist64x2(s_q, A.X + (int64_t)b0 * A.d, A.X + (int64_t)b1 * A.d, A.d, g, D64);
            if (g == 0 && i0 < nr) s_dd[i0] = D64[0];
            if (g == 0 && i1 < nr) s_dd[i1] = D64[1];
        }
    } else {
        for (int base = 0; base < nr; base += 8) {
            const int i = base + grp;
            const int b = s_r[i < nr ? i : 0];
            float D32;
            double D64;
            group8_dist32_64<VEC>(s_q, A.X + (int64_t)b * A.d, A.d, g, D32, D64);
            if (g == 0 && i < nr) s_dd[i] = D64;
        }
    }
    wave_sync();
    // R is sorted whole by (D64, index): it holds the true top K (every candidate with
    // lb <= tau'), so its first K are the answer
    int32_t *s_wi = s_r;
    double *s_wd = s_dd;
    const int nw = nr;
    if (nw <= 64) {  // the usual case: a bitonic network across the wave's lanes, in registers
        double dk = lane < nw ? s_wd[lane] : INFINITY;
        int ik = lane < nw ? s_wi[lane] : 0x7fffffff;
        for (int size = 2; size <= 64; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                const double dp = __shfl_xor(dk, stride, 64);
                const int ip = __shfl_xor(ik, stride, 64);
                const bool mine_first = dk < dp || (dk == dp && ik <= ip);  // in (D64, index) order
                const bool want_first = ((lane & stride) == 0) == ((lane & size) == 0);
                if (mine_first != want_first) {
                    dk = dp;
                    ik = ip;
                }
            }
        }
        if (lane < K) {
            const bool ok = lane < nw;
            A.out_idx[a * K + lane] = ok ? ik : -1;
            A.out_dist[a * K + lane] = ok ? (float)sqrt(dk) : INFINITY;
        }
        for (int k = 64 + lane; k < K; k += 64) {  // K above 64: nothing past the window
            A.out_idx[a * K + k] = -1;
            A.out_dist[a * K + k] = INFINITY;
        }
        if (lane == 0) {
            stat_add(A, 0, 1ull);
            stat_add(A, 2, (unsigned long long)nr);
            stat_add(A, 3, (unsigned long long)nw);
        }
        return;
    }
    int P2 = 1;
    while (P2 < nw) P2 <<= 1;
    for (int i = nw + lane; i < P2; i += 64) {
        s_wd[i] = INFINITY;
        s_wi[i] = 0x7fffffff;
    }
    wave_sync();
    for (int size = 2; size <= P2; size <<= 1) {  // bitonic sort by (D64, index)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = lane; i < P2 / 2; i += 64) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const double dl = s_wd[lo], dh = s_wd[hi];
                const int il = s_wi[lo], ih = s_wi[hi];
                const bool gt = dl > dh || (dl == dh && il > ih);
                if (gt == up) {
                    s_wd[lo] = dh;
                    s_wd[hi] = dl;
                    s_wi[lo] = ih;
                    s_wi[hi] = il;
                }
            }
            wave_sync();
        }
    }
    for (int k = lane; k < K; k += 64) {
        const bool ok = k < nw;
        A.out_idx[a * K + k] = ok ? s_wi[k] : -1;
        A.out_dist[a * K + k] = ok ? (float)sqrt(s_wd[k]) : INFINITY;
    }
    if (lane == 0) {
        stat_add(A, 0, 1ull);
        stat_add(A, 2, (unsigned long long)nr);
        stat_add(A, 3, (unsigned long long)nw);
    }
}

// One wave per result row, four rows per block.  Entries stay in registers; an LDS hash
// of indices marks the first copy of every index (any copy's interval is valid for it).
template <bool VEC, int Q>
__global__ __launch_bounds__(256) void k_final(FinalArgs A, int64_t nrows) {
    // hash table twice the records a row can hold (at most 64 Q), re-rank set half of it
    constexpr int kHT = Q <= 4 ? 512 : Q <= 12 ? 1024 : 2048;
    constexpr int kHBits = Q <= 4 ? 9 : Q <= 12 ? 10 : 11;  // log2(kHT): the hash keeps that many top bits
    static_assert((1 << kHBits) == kHT, "hash range must equal the table");
    constexpr int kRCap = kHT / 2;
    __shared__ __align__(16) int32_t s_key[4][kHT];  // index hash; read as doubles once the dedup is done
    // the rerank set R (first half; then, compacted in place, the window) and the selection
    // keys (second half); before the records are loaded, the bucket tables
    __shared__ int32_t s_rd[4][kHT];
    __shared__ uint32_t s_c[4][256];  // the distinct indices' ub keys, compacted
    extern __shared__ __align__(16) float s_qall[];  // 4 rows x dq floats
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t a = (int64_t)blockIdx.x * 4 + w;
    if (a >= nrows) return;
    const int dq = (A.d + 3) & ~3;
    float *s_q = s_qall + w * dq;
    int32_t *s_r = s_rd[w];
    uint32_t *s_d = reinterpret_cast<uint32_t *>(s_rd[w] + kRCap);
    int32_t *s_pre = s_rd[w];  // 128 buckets at most
    uint8_t *s_own = reinterpret_cast<uint8_t *>(s_rd[w] + 128);
    static_assert((kHT - 128) * 4 >= 64 * Q, "bucket owner table");
    const int c1 = A.lcnt[a];
    const int P = A.bcnt ? bucket_tables_wave(A, a, lane, s_pre, s_own, 64 * Q) : 0;
    int c2;
    bool ovf;
    phase2_count(A, a, P, c2, ovf);
    if (lane == 0) {
        stat_add(A, 5, (unsigned long long)max(c1, 0));
        stat_add(A, 6, (unsigned long long)max(c2, 0));
    }
    if (c1 > A.lcap || ovf || c1 + c2 > 64 * Q) {
        if (lane == 0) push_overflow(A, a, c1, c2, ovf);
        return;
    }
    for (int i = lane; i < kHT; i += 64) s_key[w][i] = -1;
    for (int j = lane; j < A.d; j += 64) s_q[j] = A.Qr[a * A.d + j];
    wave_sync();
    // most rows fill a few records per lane: they take the four-per-lane steps
    if (Q > 4 && c1 + c2 <= 256)
        final_row<VEC, 4, kHT>(A, a, lane, s_key[w], s_r, s_d, s_q, c1, c2, P, s_pre, s_own, s_c[w]);
    else if (Q > 8 && c1 + c2 <= 512)
        final_row<VEC, 8, kHT>(A, a, lane, s_key[w], s_r, s_d, s_q, c1, c2, P, s_pre, s_own, s_c[w]);
    else if (Q > 12 && c1 + c2 <= 768)
        final_row<VEC, 12, kHT>(A, a, lane, s_key[w], s_r, s_d, s_q, c1, c2, P, s_pre, s_own, s_c[w]);
    else
        final_row<VEC, Q, kHT>(A, a, lane, s_key[w], s_r, s_d, s_q, c1, c2, P, s_pre, s_own, s_c[w]);
}

// ---------------------------------------------------------------- final merge, one block per row

// For rows whose list plus Phase II records exceed one wave's 64 Q (large K against many
// trees): the same steps as k_final with the 256 threads of a block on one row, up to 4096
// records (16 per thread).  Selections are the same ballot bisection, with each bit's count
// summed over the four waves.
constexpr int kBigHT = 2 * kBigCap;    // index hash (twice the records); later R's binary64 distances
constexpr int kBigHBits = 13;          // log2(kBigHT)
constexpr int kBigRCap = 1024;         // rerank set R
constexpr int kBigWCap = 512;          // binary64 window
static_assert((1 << kBigHBits) == kBigHT, "hash range must equal the table");
static_assert(kBigHT / 2 >= kBigRCap, "the dead hash table holds R's binary64 distances");

// block-wide (256 threads) reductions through 4 LDS words; every thread gets the result
__device__ inline uint32_t block_sum4(uint32_t v, uint32_t *s4) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = v;
    __syncthreads();
    return (s4[0] + s4[1]) + (s4[2] + s4[3]);
}

__device__ inline uint32_t block_min4(uint32_t v, uint32_t *s4) {
    v = wave_min_u32(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = v;
    __syncthreads();
    return min(min(s4[0], s4[1]), min(s4[2], s4[3]));
}

__device__ inline uint32_t block_max4(uint32_t v, uint32_t *s4) {
    v = wave_max_u32(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = v;
    __syncthreads();
    return max(max(s4[0], s4[1]), max(s4[2], s4[3]));
}

// wave_kth_upper over the keys a block holds Q per thread (0xffffffff: not taking part)
template <int Q>
__device__ inline uint32_t block_kth_upper(const uint32_t (&v)[Q], int k, uint32_t *s4) {
    constexpr int kLow = 13;
    uint32_t lo = 0xffffffffu, hi = 0;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        lo = min(lo, v[q]);
        hi = max(hi, v[q] == 0xffffffffu ? 0u : v[q]);
    }
    lo = block_min4(lo, s4);
    hi = block_max4(hi, s4);
    if (lo >= hi) return lo;
    const int hb = 31 - __builtin_clz(lo ^ hi);
    if (hb < kLow) return hi;
    uint32_t ans = hb >= 31 ? 0u : (lo & ~((2u << hb) - 1u));
    for (int b = hb; b >= kLow; b--) {
        const uint32_t t = ans | (1u << b);
        uint32_t c = 0;
#pragma unroll
        for (int q = 0; q < Q; q++) c += (uint32_t)__popcll(__ballot(v[q] < t));
        __syncthreads();
        if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = c;
        __syncthreads();
        if ((s4[0] + s4[1]) + (s4[2] + s4[3]) <= (uint32_t)k) ans = t;
    }
    return min(ans | ((1u << kLow) - 1u), hi);
}

// One row of the block merge.  `counted`: the row's record counts are not yet in the stats
// (a row handed over by the wave merge was counted there).
template <bool VEC>
__device__ __attribute__((always_inline)) inline void final_blk_row(const FinalArgs &A, int64_t a, bool counted,
                                                                    int32_t *s_key, uint32_t *s_ubn, int32_t *s_r,
                                                                    uint32_t *s_d, uint32_t *s4, uint32_t *s_sc,
                                                                    float *s_q) {
    const int tid = threadIdx.x, lane = tid & 63, g = lane & 7, grp = tid >> 3;
    const int K = A.K;
    const int c1 = A.lcnt[a];
    // bucket mode: the first wave builds the row's bucket tables in s_r (first records) and
    // s_d (owner of each record), both dead until R is formed
    int32_t *s_pre = s_r;
    uint8_t *s_own = reinterpret_cast<uint8_t *>(s_d);
    static_assert(kBigRCap * 4 >= kBigCap && kBigRCap >= 128, "bucket tables");
    if (A.bcnt && tid < 64) {
        const int P = bucket_tables_wave(A, a, lane, s_pre, s_own, kBigCap);
        if (lane == 0) s4[0] = (uint32_t)P;
    }
    __syncthreads();
    const int P = A.bcnt ? (int)s4[0] : 0;
    int c2;
    bool ovf;
    phase2_count(A, a, P, c2, ovf);
    if (tid == 0 && !counted) {
        stat_add(A, 5, (unsigned long long)max(c1, 0));
        stat_add(A, 6, (unsigned long long)max(c2, 0));
    }
    if (c1 > A.lcap || ovf || c1 + c2 > kBigCap) {
        if (tid == 0) push_fallback(A, a);
        return;
    }
    for (int i = tid; i < kBigHT; i += 256) {
        s_key[i] = -1;
        s_ubn[i] = 0xffffffffu;
    }
    for (int j = tid; j < A.d; j += 256) s_q[j] = A.Qr[a * A.d + j];
    __syncthreads();
    Ent ev[kBigQ];  // every record of the row is loaded first
#pragma unroll
    for (int q = 0; q < kBigQ; q++) {
        const int i = tid + 256 * q;
        ev[q] = i < c1 + c2 ? (i < c1 ? A.list[a * A.lcap + i] : phase2_rec(A, a, i - c1, P, s_pre, s_own))
                            : invalid_rec();
    }
    // Dedup by index, as in final_row: the first copy of an index claims a hash slot, the slot
    // keeps the smallest ub of the copies (s_ubn), and a copy with lb <= tau' marks its index
    // for R.
    bool bad = false;
    uint32_t nd_mine = 0;
#pragma unroll
    for (int q = 0; q < kBigQ; q++) {
        const Ent e = ev[q];
        bad |= e.idx < -1 || (int64_t)e.idx >= A.npts;
        if (e.idx >= 0 && (int64_t)e.idx < A.npts) {
            uint32_t h = ((uint32_t)e.idx * 2654435761u) >> (32 - kBigHBits);
            while (true) {  // at most half full: a free or matching entry is always found
                const int old = atomicCAS(&s_key[h], -1, e.idx);
                if (old == -1) {
                    nd_mine++;
                    break;
                }
                if (old == e.idx) break;
                h = (h + 1) & (kBigHT - 1);
            }
            atomicMin(&s_ubn[h], fkey(e.ub));
        }
    }
    if (__syncthreads_or(bad)) {  // counted for the host to report; the row is recomputed exhaustively
        if (tid == 0) {
            stat_add(A, 4, 1ull);
            atomicAdd(A.fault, 1ull);
            push_fallback(A, a);
        }
        return;
    }
    constexpr int NS = kBigHT / 256;  // hash slots per thread
    const uint32_t nd = block_sum4(nd_mine, s4);
    float tv = INFINITY;
    if (nd >= (uint32_t)K) {
        uint32_t fu[NS];  // ub minima of the occupied slots, empty slots as the largest key
#pragma unroll
        for (int k = 0; k < NS; k++) {
            const int slot = tid + 256 * k;
            fu[k] = s_key[slot] != -1 ? s_ubn[slot] : 0xffffffffu;
        }
        tv = __uint_as_float(block_kth_upper<NS>(fu, K - 1, s4));
    }
    const uint32_t tp = fkey(tv * (1.f + 1e-6f));
#pragma unroll
    for (int q = 0; q < kBigQ; q++) {
        const Ent e = ev[q];
        if (e.idx >= 0 && fkey(e.lb) <= tp) {
            uint32_t h = ((uint32_t)e.idx * 2654435761u) >> (32 - kBigHBits);
            while (s_key[h] != e.idx) h = (h + 1) & (kBigHT - 1);
            atomicOr(&s_ubn[h], 0x80000000u);
        }
    }
    __syncthreads();
    // R = the marked indices: per-thread counts, one block scan, then the writes
    uint32_t rc = 0;
#pragma unroll
    for (int k = 0; k < NS; k++) {
        const int slot = tid + 256 * k;
        rc += (s_key[slot] != -1 && (s_ubn[slot] >> 31)) ? 1u : 0u;
    }
    uint32_t rbase, nr;
    block_excl_scan256(rc, s_sc, rbase, nr);
    if (nr > (uint32_t)kBigRCap) {
        if (tid == 0) push_fallback(A, a);
        return;
    }
#pragma unroll
    for (int k = 0; k < NS; k++) {
        const int slot = tid + 256 * k;
        const int32_t id = s_key[slot];
        if (id != -1 && (s_ubn[slot] >> 31)) s_r[rbase++] = id;
    }
    __syncthreads();  // R is complete and the hash is dead: it holds the binary64 distances now
    double *s_dd = reinterpret_cast<double *>(s_key);
    if constexpr (VEC) {  // 32 groups of eight lanes, two candidates each at a time
        for (int base = 0; base < (int)nr; base += 64) {
            const int i0 = base + grp, i1 = i0 + 32;
            const int b0 = s_r[i0 < (int)nr ? i0 : 0], b1 = s_r[i1 < (int)nr ? i1 : 0];
            float D32[2];
            double D64[2];
            group8_dist32_64x2(s_q, A.X + (int64_t)b0 * A.d, A.X + (int64_t)b1 * A.d, A.d, g, D32, D64);
            if (g == 0 && i0 < (int)nr) {
                s_d[i0] = fkey(D32[0]);
                s_dd[i0] = D64[0];
            }
            if (g == 0 && i1 < (int)nr) {
                s_d[i1] = fkey(D32[1]);
                s_dd[i1] = D64[1];
            }
        }
    } else {
        for (int base = 0; base < (int)nr; base += 32) {
            const int i = base + grp;
            const int b = s_r[i < (int)nr ? i : 0];
            float D32;
            double D64;
            group8_dist32_64<VEC>(s_q, A.X + (int64_t)b * A.d, A.d, g, D32, D64);
            if (g == 0 && i < (int)nr) {
                s_d[i] = fkey(D32);
                s_dd[i] = D64;
            }
        }
    }
    __syncthreads();
    constexpr int RQ = kBigRCap / 256;
    float d32k = INFINITY;
    if (nr >= (uint32_t)K) {
        uint32_t dv[RQ];
#pragma unroll
        for (int q = 0; q < RQ; q++) {
            const int i = tid + 256 * q;
            dv[q] = i < (int)nr ? s_d[i] : 0xffffffffu;
        }
        d32k = __uint_as_float(block_kth_upper<RQ>(dv, K - 1, s4));
    }
    const float wcut = d32k * (1.f + A.win);
    // the window, compacted in place over R: everything is read before anything is written
    int32_t wi[RQ];
    double wd[RQ];
    uint32_t wc = 0;
#pragma unroll
    for (int q = 0; q < RQ; q++) {
        const int i = tid + 256 * q;
        const bool in = i < (int)nr && __uint_as_float(s_d[i]) <= wcut;
        wi[q] = in ? s_r[i] : -1;
        wd[q] = in ? s_dd[i] : 0.0;
        wc += in ? 1u : 0u;
    }
    uint32_t wbase, nw;
    block_excl_scan256(wc, s_sc, wbase, nw);  // its barriers also order the reads above before the writes
    if (nw > (uint32_t)kBigWCap) {  // pathological window (massive distance ties): exhaustive path
        if (tid == 0) push_fallback(A, a);
        return;
    }
#pragma unroll
    for (int q = 0; q < RQ; q++)
        if (wi[q] >= 0) {
            s_r[wbase] = wi[q];
            s_dd[wbase] = wd[q];
            wbase++;
        }
    int P2 = 1;
    while (P2 < (int)nw) P2 <<= 1;
    for (int i = (int)nw + tid; i < P2; i += 256) {
        s_dd[i] = INFINITY;
        s_r[i] = 0x7fffffff;
    }
    __syncthreads();
    for (int size = 2; size <= P2; size <<= 1) {  // bitonic sort by (D64, index)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < P2 / 2; i += 256) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const double dl = s_dd[lo], dh = s_dd[hi];
                const int il = s_r[lo], ih = s_r[hi];
                const bool gt = dl > dh || (dl == dh && il > ih);
                if (gt == up) {
                    s_dd[lo] = dh;
                    s_dd[hi] = dl;
                    s_r[lo] = ih;
                    s_r[hi] = il;
                }
            }
            __syncthreads();
        }
    }
    for (int k = tid; k < K; k += 256) {
        const bool ok = k < (int)nw;
        A.out_idx[a * K + k] = ok ? s_r[k] : -1;
        A.out_dist[a * K + k] = ok ? (float)sqrt(s_dd[k]) : INFINITY;
    }
    if (tid == 0) {
        stat_add(A, 0, 1ull);
        stat_add(A, 2, (unsigned long long)nr);
        stat_add(A, 3, (unsigned long long)nw);
    }
}

// LIST = false: one block per row.  LIST = true: the blocks walk the rows the wave merge
// handed over (their count is final: the wave merge ran before on the same stream).
template <bool VEC, bool LIST>
__global__ __launch_bounds__(256) void k_final_blk(FinalArgs A) {
    __shared__ __align__(16) int32_t s_key[kBigHT];  // index hash; then R's binary64 distances
    __shared__ uint32_t s_ubn[kBigHT];                // per hash slot: smallest ub, top bit = out of R
    __shared__ int32_t s_r[kBigRCap];                // R; then, compacted, the window
    __shared__ uint32_t s_d[kBigRCap];
    __shared__ uint32_t s4[4];    // reductions and selection counts
    __shared__ uint32_t s_sc[4];  // block scans
    extern __shared__ __align__(16) float s_q[];      // the query row (d floats)
    if constexpr (LIST) {
        const int nb = *A.big_cnt;
        for (int i = blockIdx.x; i < nb; i += gridDim.x) {
            __syncthreads();  // the previous row's LDS reads are done
            final_blk_row<VEC>(A, A.big_list[i], true, s_key, s_ubn, s_r, s_d, s4, s_sc, s_q);
        }
    } else {
        final_blk_row<VEC>(A, blockIdx.x, false, s_key, s_ubn, s_r, s_d, s4, s_sc, s_q);
    }
}

// ---------------------------------------------------------------- exhaustive fallback

constexpr int kFallbackThreads = 512;  // threads per row of the exhaustive path

struct FallbackArgs {
    const int32_t *fb_list;
    const int32_t *fb_cnt;
    const float *X;
    const float *Qr;
    int d;
    int K;
    int T;
    int64_t n;
    const int32_t *perm;        // [T][n]
    const int32_t *row_leaf;    // [T][nrows] heap id of each row's leaf
    int64_t nrows;
    const int32_t *heap_leaf;   // heap id -> leaf index
    const LeafDesc *leaves;
    int64_t leaf_stride;        // leaves of tree t start at t * leaf_stride (0: one shared table)
    int32_t exclude_self;       // all-points: row a is point a
    int32_t *out_idx;
    float *out_dist;
};

// The exhaustive path, one row per block of NTH threads: the union of the row's leaves over
// all trees in binary64.  The members of up to 64 trees' leaves are taken as one list, NTH at
// a time (a piece spans trees); the ids of the next piece are read while the current one is
// measured, and every group of eight lanes measures four members at once.  Only members
// before the running list's last entry in (D, index) order can enter a full list; they are
// compacted to the front, the list is appended behind them, and the K smallest distinct
// indices are kept (a repeated index repeats its distance, so its copies sort together).
template <bool VEC, int NTH>
__global__ __launch_bounds__(NTH) void k_fallback(FallbackArgs F) {
    constexpr int NW = NTH / 64, NG = NTH / 8;
    constexpr int CAP = 2 * NTH;  // a piece's candidates and the list (K <= 256 <= NTH)
    static_assert(NTH >= 256 && (NTH & (NTH - 1)) == 0, "a power of two of at least 256 threads");
    __shared__ double s_cd[CAP];
    __shared__ int32_t s_ci[CAP];
    __shared__ double s_td[256];
    __shared__ int32_t s_ti[256];
    __shared__ int s_tn;
    __shared__ uint32_t s_scan[NW];
    __shared__ int32_t s_mid[NTH];
    __shared__ LeafDesc s_lf[64];
    __shared__ int32_t s_lo[65];  // first member of each tree's leaf in the list
    extern __shared__ __align__(16) float s_q[];
    const int tid = threadIdx.x, g = tid & 7, grp = tid >> 3;
    const int nfb = *F.fb_cnt;
    const int K = F.K;  // <= 256 on this path
    for (int q = blockIdx.x; q < nfb; q += gridDim.x) {
        const int64_t a = F.fb_list[q];
        __syncthreads();
        for (int j = tid; j < F.d; j += NTH) s_q[j] = F.Qr[a * F.d + j];
        if (tid == 0) s_tn = 0;
        __syncthreads();
        for (int t0 = 0; t0 < F.T; t0 += 64) {  // the row's leaves, 64 trees at a time
            const int nt = min(64, F.T - t0);
            __syncthreads();
            if (tid < nt)
                s_lf[tid] = F.leaves[(t0 + tid) * F.leaf_stride + F.heap_leaf[F.row_leaf[(int64_t)(t0 + tid) * F.nrows + a]]];
            __syncthreads();
            if (tid == 0) {
                int run = 0;
                for (int tt = 0; tt < nt; tt++) {
                    s_lo[tt] = run;
                    run += s_lf[tt].size;
                }
                s_lo[nt] = run;
            }
            __syncthreads();
            const int M = s_lo[nt];
            auto id_of = [&](int m) -> int32_t {  // member m of the list: its point index
                if (m >= M) return -1;
                int lo = 0, hi = nt - 1;  // the last tree whose first member is at most m
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_lo[mid] <= m) lo = mid;
                    else hi = mid - 1;
                }
                return F.perm[(int64_t)(t0 + lo) * F.n + s_lf[lo].off + (m - s_lo[lo])];
            };
            int32_t nid = id_of(tid);
            for (int base = 0; base < M; base += NTH) {
                __syncthreads();
                s_mid[tid] = nid;
                __syncthreads();
                nid = id_of(base + NTH + tid);
                if constexpr (VEC) {  // four members per group of eight lanes at a time
                    for (int sub = 0; sub < NTH; sub += 4 * NG) {
                        int bm[4];
                        const float *rows[4];
#pragma unroll
                        for (int h = 0; h < 4; h++) {
                            bm[h] = s_mid[sub + grp + NG * h];
                            rows[h] = F.X + (int64_t)(bm[h] < 0 ? 0 : bm[h]) * F.d;
                        }
                        double D64[4];
                        group8_dist64x4(s_q, rows, F.d, g, D64);
                        if (g == 0) {
#pragma unroll
                            for (int h = 0; h < 4; h++) {
                                const int l = sub + grp + NG * h, b = bm[h];
                                const bool ok = b >= 0 && !(F.exclude_self && b == a);
                                s_cd[l] = ok ? D64[h] : INFINITY;
                                s_ci[l] = ok ? b : 0x7fffffff;
                            }
                        }
                    }
                } else {
                    for (int sub = 0; sub < NTH; sub += NG) {
                        const int l = sub + grp, b = s_mid[l];
                        const double D = group8_dist64<VEC>(s_q, F.X + (int64_t)(b < 0 ? 0 : b) * F.d, F.d, g);
                        if (g == 0) {
                            const bool ok = b >= 0 && !(F.exclude_self && b == a);
                            s_cd[l] = ok ? D : INFINITY;
                            s_ci[l] = ok ? b : 0x7fffffff;
                        }
                    }
                }
                for (int i = NTH + tid; i < CAP; i += NTH) {
                    s_cd[i] = INFINITY;
                    s_ci[i] = 0x7fffffff;
                }
                __syncthreads();
                const int tn = s_tn;
                const double dc = s_cd[tid];
                const int ic = s_ci[tid];
                bool take = ic != 0x7fffffff;
                if (tn == K) {
                    const double lastd = s_td[K - 1];
                    const int lasti = s_ti[K - 1];
                    take = take && (dc < lastd || (dc == lastd && ic < lasti));
                }
                uint32_t pos, ncand;
                block_excl_scan_w<NW>(take ? 1u : 0u, s_scan, pos, ncand);  // every read above is done
                if (ncand == 0) continue;
                if (take) {
                    s_cd[pos] = dc;
                    s_ci[pos] = ic;
                }
                for (int i = tid; i < tn; i += NTH) {
                    s_cd[ncand + i] = s_td[i];
                    s_ci[ncand + i] = s_ti[i];
                }
                const int tot = (int)ncand + tn;
                __syncthreads();
                if (tot <= 64) {  // the usual case: one wave sorts in registers and keeps K distinct
                    if (tid < 64) {
                        double dk = tid < tot ? s_cd[tid] : INFINITY;
                        int ik = tid < tot ? s_ci[tid] : 0x7fffffff;
                        for (int size = 2; size <= 64; size <<= 1) {
                            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                                const double dp = __shfl_xor(dk, stride, 64);
                                const int ip = __shfl_xor(ik, stride, 64);
                                const bool mine_first = dk < dp || (dk == dp && ik <= ip);
                                const bool want_first = ((tid & stride) == 0) == ((tid & size) == 0);
                                if (mine_first != want_first) {
                                    dk = dp;
                                    ik = ip;
                                }
                            }
                        }
                        const int iprev = __shfl_up(ik, 1, 64);
                        const bool keep = ik != 0x7fffffff && (tid == 0 || ik != iprev);
                        const uint64_t mk = __ballot(keep);
                        const int r = mask_rank(mk);
                        if (keep && r < K) {
                            s_td[r] = dk;
                            s_ti[r] = ik;
                        }
                        if (tid == 0) s_tn = min(__popcll(mk), K);
                    }
                    __syncthreads();
                    continue;
                }
                int P2 = 128;  // bitonic sort of the first P2 >= tot entries (block-uniform)
                while (P2 < tot) P2 <<= 1;
                for (int i = tot + tid; i < P2; i += NTH) {
                    s_cd[i] = INFINITY;
                    s_ci[i] = 0x7fffffff;
                }
                __syncthreads();
                for (int size = 2; size <= P2; size <<= 1)
                    for (int stride = size >> 1; stride > 0; stride >>= 1) {
                        for (int i = tid; i < P2 / 2; i += NTH) {
                            const int lo = 2 * i - (i & (stride - 1));
                            const int hi = lo + stride;
                            const bool up = (lo & size) == 0;
                            const double dl = s_cd[lo], dh = s_cd[hi];
                            const int il = s_ci[lo], ih = s_ci[hi];
                            const bool gtr = dl > dh || (dl == dh && il > ih);
                            if (gtr == up) {
                                s_cd[lo] = dh;
                                s_cd[hi] = dl;
                                s_ci[lo] = ih;
                                s_ci[hi] = il;
                            }
                        }
                        __syncthreads();
                    }
                {  // K smallest distinct: thread tid holds entries E tid .. E tid + E - 1
                    constexpr int EMAX = CAP / NTH;
                    const int E = P2 > NTH ? P2 / NTH : 1;
                    bool keep[EMAX];
                    double kd[EMAX];
                    int ki[EMAX];
                    uint32_t cnt = 0;
#pragma unroll
                    for (int e = 0; e < EMAX; e++) {
                        const int i = E * tid + e;
                        const bool in = e < E && i < P2;
                        keep[e] = in && s_ci[i] != 0x7fffffff && (i == 0 || s_ci[i] != s_ci[i - 1]);
                        kd[e] = in ? s_cd[i] : INFINITY;
                        ki[e] = in ? s_ci[i] : 0x7fffffff;
                        cnt += keep[e] ? 1u : 0u;
                    }
                    uint32_t excl, total;
                    block_excl_scan_w<NW>(cnt, s_scan, excl, total);  // every read of the sorted list is done
#pragma unroll
                    for (int e = 0; e < EMAX; e++)
                        if (keep[e]) {
                            if (excl < (uint32_t)K) {
                                s_td[excl] = kd[e];
                                s_ti[excl] = ki[e];
                            }
                            excl++;
                        }
                    if (tid == 0) s_tn = (int)min(total, (uint32_t)K);
                }
                __syncthreads();
            }
        }
        for (int k = tid; k < K; k += NTH) {
            const bool ok = k < s_tn;
            F.out_idx[a * K + k] = ok ? s_ti[k] : -1;
            F.out_dist[a * K + k] = ok ? (float)sqrt(s_td[k]) : INFINITY;
        }
    }
}

// ---------------------------------------------------------------- batched forests

// neighbour indices of a forest over several data sets: global point index -> index within
// the row's own data set (candidates never leave a data set, so one offset per row)
__global__ void k_localize(int32_t *__restrict__ idx, int64_t rows, int K, const int64_t *__restrict__ off,
                           int count) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = count - 1;  // last data set whose offset is <= r
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= r) lo = mid;
            else hi = mid - 1;
        }
        const int32_t base = (int32_t)off[lo];
        int32_t *row = idx + r * K;
        for (int k = 0; k < K; k++)
            if (row[k] >= 0) row[k] -= base;
    }
}

void launch_localize(int32_t *idx, int64_t rows, int K, const int64_t *off, int count, hipStream_t s) {
    const unsigned blocks = (unsigned)std::min<int64_t>((rows + 255) / 256, 4096);
    hipLaunchKernelGGL(k_localize, dim3(blocks), dim3(256), 0, s, idx, rows, K, off, count);
    launch_check(s, "k_localize");
}

// ---------------------------------------------------------------- routing (Alg. 3, descent of a query through each tree)

template <bool VEC>
__global__ __launch_bounds__(256) void k_route(const float *__restrict__ Q, int64_t m, int d,
                                               const float *__restrict__ R, int64_t H, int n_try,
                                               const int32_t *__restrict__ chosen, const double *__restrict__ split,
                                               int64_t n, int n0, int32_t *__restrict__ out_leaf) {
    const int t = blockIdx.y;
    const int g = threadIdx.x & 7;
    const int64_t q = (int64_t)blockIdx.x * 32 + (threadIdx.x >> 3);
    const int64_t qq = q < m ? q : 0;
    const float *x = Q + qq * d;
    int64_t h = 1, size = n;
    while (size > n0) {  // the 8 lanes of a group follow the same query
        const int64_t hs = (int64_t)t * H + (h - 1);
        const float *r = R + (hs * n_try + chosen[hs]) * (int64_t)d;
        const double p = group8_dot64<VEC>(x, r, d, g);
        const bool right = p >= split[hs];
        size = right ? size - size / 2 : size / 2;
        h = 2 * h + (right ? 1 : 0);
    }
    if (g == 0 && q < m) out_leaf[(int64_t)t * m + q] = (int32_t)h;
}

// ================================================================ query preparation

// group routed queries by (tree, leaf): counts, offsets, then the grouped order
__global__ void k_group_count(const int32_t *__restrict__ qleaf, int64_t m, const int32_t *__restrict__ heap_leaf,
                              int64_t nleaf, int32_t *__restrict__ gcount) {
    const int t = blockIdx.y;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m; q += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&gcount[(int64_t)t * nleaf + heap_leaf[qleaf[(int64_t)t * m + q]]], 1);
}

__global__ __launch_bounds__(1024) void k_group_scan(const int32_t *__restrict__ gcount, int64_t nleaf,
                                                     int32_t *__restrict__ goff) {
    __shared__ int32_t s_w[16];
    __shared__ int32_t s_run;
    const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_run = 0;
    __syncthreads();
    for (int64_t base = 0; base < nleaf; base += 1024) {
        const int64_t i = base + tid;
        const int32_t v = i < nleaf ? gcount[(int64_t)t * nleaf + i] : 0;
        int32_t x = v;
        for (int o = 1; o < 64; o <<= 1) {
            int32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_w[w] = x;
        __syncthreads();
        int32_t wb = 0, tot = 0;
        for (int k = 0; k < 16; k++) {
            if (k < w) wb += s_w[k];
            tot += s_w[k];
        }
        if (i < nleaf) goff[(int64_t)t * nleaf + i] = s_run + wb + x - v;
        __syncthreads();
        if (tid == 0) s_run += tot;
        __syncthreads();
    }
}

__global__ void k_group_fill(const int32_t *__restrict__ qleaf, int64_t m, const int32_t *__restrict__ heap_leaf,
                             int64_t nleaf, const int32_t *__restrict__ goff, int32_t *__restrict__ gfill,
                             int32_t *__restrict__ qorder, int32_t *__restrict__ qgleaf) {
    const int t = blockIdx.y;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t li = heap_leaf[qleaf[(int64_t)t * m + q]];
        const int32_t pos = goff[(int64_t)t * nleaf + li] + atomicAdd(&gfill[(int64_t)t * nleaf + li], 1);
        qorder[(int64_t)t * m + pos] = (int32_t)q;
        qgleaf[(int64_t)t * m + pos] = li;
    }
}

// one tile job per (A chunk of a non-empty group) x (B tile of the leaf); the first trees -> list 0
__global__ void k_make_jobs(const int32_t *__restrict__ gcount, const int32_t *__restrict__ goff, int64_t nleaf,
                            const LeafDesc *__restrict__ leaves, int TR, int nfirst, int qs, TileJob *__restrict__ jobs0,
                            TileJob *__restrict__ jobs1, TileJob *__restrict__ sjobs0, TileJob *__restrict__ sjobs1,
                            int32_t *__restrict__ njobs) {
    // one (leaf, tree) group per lane; the jobs of a wave are reserved with one atomic per
    // list (MFMA tiles or the GEMV-shaped kernel) instead of one per job
    const int t = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const bool first = t < nfirst;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nleaf; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t li = base + threadIdx.x;
        const int32_t c = li < nleaf ? gcount[(int64_t)t * nleaf + li] : 0;
        LeafDesc lf{};
        int na = 0, nb = 0;
        if (c > 0) {
            lf = leaves[li];
            na = (c + TR - 1) / TR;
            nb = (lf.size + TR - 1) / TR;
        }
        const bool small = c <= qs;  // a few queries: the GEMV-shaped kernel
#pragma unroll
        for (int ls = 0; ls < 2; ls++) {  // ls = 1: the small-group list
            const int v = (c > 0 && small == (ls == 1)) ? na * nb : 0;
            int incl = v;
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o, 64);
                if (lane >= o) incl += y;
            }
            const int total = __shfl(incl, 63, 64);
            if (total == 0) continue;
            int slot0 = 0;
            if (lane == 63) slot0 = atomicAdd(&njobs[(first ? 0 : 1) + (ls ? 2 : 0)], total);
            slot0 = __shfl(slot0, 63, 64) + incl - v;
            if (v == 0) continue;
            TileJob *dst = ls ? (first ? sjobs0 : sjobs1) : (first ? jobs0 : jobs1);
            for (int I = 0; I < na; I++)
                for (int J = 0; J < nb; J++) {
                    TileJob j;
                    j.a_off = goff[(int64_t)t * nleaf + li] + (int64_t)I * TR;
                    j.b_off = lf.off + (int64_t)J * TR;
                    j.a_rows = min(TR, c - I * TR);
                    j.b_rows = min(TR, lf.size - J * TR);
                    j.tree = t;
                    j.same = 0;
                    j.b_pos = J * TR;
                    j.leaf_m = lf.size;
                    j.leaf = (int32_t)li;
                    j.pad = 0;
                    dst[slot0++] = j;
                }
        }
    }
}

// leaf-centred query copies in the tile precision, with the same norms as the data copies
template <typename T>
__global__ __launch_bounds__(256) void k_query_prep(const float *__restrict__ Q, int64_t m, int d, int dp,
                                                    const int32_t *__restrict__ qorder,
                                                    const int32_t *__restrict__ qgleaf,
                                                    const float *__restrict__ centroid, int64_t nleaf,
                                                    T *__restrict__ Qc, float2 *__restrict__ qnrm, float range_max) {
    const int t = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int64_t pos = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pos >= m) return;
    const int64_t q = qorder[(int64_t)t * m + pos];
    const float *mu = centroid + ((int64_t)t * nleaf + qgleaf[(int64_t)t * m + pos]) * d;
    T *out = Qc + ((int64_t)t * m + pos) * dp;
    float na = 0.f, ra = 0.f;
    bool over = false;
    for (int j = lane; j < dp; j += 64) {
        const float a = j < d ? Q[q * d + j] - mu[j] : 0.f;
        over |= fabsf(a) > range_max;
        const T v = (T)a;
        out[j] = v;
        const float vf = (float)v;
        na = __builtin_fmaf(vf, vf, na);
        ra = __builtin_fmaf(a, a, ra);
    }
    for (int o = 32; o > 0; o >>= 1) {
        na += __shfl_xor(na, o, 64);
        ra += __shfl_xor(ra, o, 64);
    }
    const uint64_t ov = __ballot(over);
    if (lane == 0) qnrm[(int64_t)t * m + pos] = make_float2(na, ov ? INFINITY : sqrtf(ra));
}

// ================================================================ host launch sequences

// Phase I trees: at most kFirstTrees, and K * B must leave room in the merge's small set
// trees of Phase I: at most kFirstTrees, and few enough that the K B smallest bounds fit the
// representative set and the B ML slots of a row fit one wave's registers
// Phase I slots per (row, tree): the largest leaf rounded up to a wave, so that the slots of a
// row's wave-wide column q all belong to one tree

// Bound coefficients of a tile precision (see pair_bounds).  Split bfloat16: the tiles hold
// the binary32 values a (norms and copy rounding as binary32), and the Gram product is
// sum(hi_a hi_b + hi_a lo_b + lo_a hi_b) over 3d exact products accumulated in binary32.
// With |lo| <= 2^-8 |a|, |a - hi - lo| <= 2^-16 |a|, the omitted lo.lo and residual terms
// are at most 3.0001 2^-16 |a||b| per column, the accumulation at most 1.0235 gamma_{3d+1}
// |a||b|; twice that (D = |a|^2 + |b|^2 - 2G) is at most (1.0235 gamma_{3d+1} + 3.0001
// 2^-16)(|a|^2 + |b|^2), beside 2 gamma_{d+2} for the two norms.  An input a flushed to zero
// by the MFMA moves each row by at most 2^-126 per column: eta covers it.
static BoundCoef bound_coef(int prec, int d) {
    const double u32 = ldexp(1.0, -24);
    const double ulp = prec == RPF_DIST_BF16 ? ldexp(1.0, -8) : prec == RPF_DIST_FP16 ? ldexp(1.0, -11) : 0.0;
    const double k = d + 2;
    const double gam = k * u32 / (1.0 - k * u32);
    BoundCoef bc;
    if (prec == RPF_DIST_BF16X3) {
        const double k3 = 3.0 * d + 2;
        const double gam3 = k3 * u32 / (1.0 - k3 * u32);
        bc.e = (float)((2.0 * gam + 1.0235 * gam3 + 3.0001 * ldexp(1.0, -16)) * 1.02);
        bc.c = (float)(u32 * (1.0 + (d + 4) * u32) * 1.01);
        bc.eta = (float)(2.0 * ldexp(1.0, -125) * sqrt((double)d) * 1.01);
        return bc;
    }
    bc.e = (float)(2.0 * 2.0 * gam * 1.01);
    bc.c = (float)((ulp + u32 + ulp * u32) * (1.0 + (d + 4) * u32) * 1.01);
    bc.eta = prec == RPF_DIST_FP16 ? (float)(2.0 * ldexp(1.0, -25) * sqrt((double)d) * 1.01) : 0.f;
    return bc;
}

static float rerank_window(int d) {
    const double u32 = ldexp(1.0, -24);
    const double eps = (ceil(d / 32.0) + 8.0) * u32;
    return (float)std::max(2e-6, 2.5 * eps + 4.0 * u32);
}

template <int MB, int PREC>
static void tile_launch(hipStream_t s, int64_t njobs, const TileJob *jobs, const void *A, const void *B, int dp,
                        int64_t as, int64_t bs, const float2 *an, const float2 *bn, const int32_t *ad,
                        const int32_t *bp, BoundCoef bc, int excl, const TileOut &out) {
    if (njobs <= 0) return;
    hipLaunchKernelGGL((k_tile<MB, PREC>), dim3((unsigned)(8 * ((njobs + 7) / 8))), dim3(64 * MB), 0, s, jobs, njobs, A,
                       B, dp, as, bs, an, bn, ad, bp, bc, excl, out);
    launch_check(s, "k_tile");
}

template <int PREC>
static void tile_dispatch_mb(int MB, hipStream_t s, int64_t njobs, const TileJob *jobs, const void *A, const void *B,
                             int dp, int64_t as, int64_t bs, const float2 *an, const float2 *bn, const int32_t *ad,
                             const int32_t *bp, BoundCoef bc, int excl, const TileOut &out) {
    switch (MB) {
    case 1: tile_launch<1, PREC>(s, njobs, jobs, A, B, dp, as, bs, an, bn, ad, bp, bc, excl, out); break;
    case 2: tile_launch<2, PREC>(s, njobs, jobs, A, B, dp, as, bs, an, bn, ad, bp, bc, excl, out); break;
    case 4: tile_launch<4, PREC>(s, njobs, jobs, A, B, dp, as, bs, an, bn, ad, bp, bc, excl, out); break;
    default: tile_launch<8, PREC>(s, njobs, jobs, A, B, dp, as, bs, an, bn, ad, bp, bc, excl, out); break;
    }
}

static void tile_dispatch(int prec, int MB, hipStream_t s, int64_t njobs, const TileJob *jobs, const void *A,
                          const void *B, int dp, int64_t as, int64_t bs, const float2 *an, const float2 *bn,
                          const int32_t *ad, const int32_t *bp, BoundCoef bc, int excl, const TileOut &out) {
    if (prec == RPF_DIST_BF16)
        tile_dispatch_mb<RPF_DIST_BF16>(MB, s, njobs, jobs, A, B, dp, as, bs, an, bn, ad, bp, bc, excl, out);
    else if (prec == RPF_DIST_FP16)
        tile_dispatch_mb<RPF_DIST_FP16>(MB, s, njobs, jobs, A, B, dp, as, bs, an, bn, ad, bp, bc, excl, out);
    else
        tile_dispatch_mb<RPF_DIST_FP32>(MB, s, njobs, jobs, A, B, dp, as, bs, an, bn, ad, bp, bc, excl, out);
}

// per-call workspace from the caching allocator; blocks go back ordered after the call's work
struct Workspace {
    hipStream_t s;
    std::vector<void *> ptrs;
    bool ok = true;
    explicit Workspace(hipStream_t st) : s(st) {}
    template <typename P>
    P *get(size_t bytes) {
        void *p = cache_alloc(bytes ? bytes : 16, s);
        if (!p) {
            ok = false;
            return nullptr;
        }
        ptrs.push_back(p);
        return static_cast<P *>(p);
    }
    ~Workspace() {
        for (void *p : ptrs) cache_free(p, s);
    }
};

// common candidate stage once the tile jobs, A rows and per-row metadata are known
struct CandStage {
    bool all_points = false;  // rows are the forest's points (Q = U)
    int shape = 0;            // Phase II symmetric tile shape (the tuner's; 0 = default)
    int bucket_S = 0;         // Phase II bucket size (the tuner's; 0 = the default rule)
    int64_t rows;          // number of result rows (n or m)
    const TileJob *jobs0;  // Phase I jobs (first tree)
    const TileJob *jobs1;  // Phase II jobs (other trees)
    int64_t njobs0, njobs1;
    const void *A;
    int64_t a_stride;
    const float2 *a_nrm;
    const int32_t *a_dest;
    const float *Qr;       // binary32 rows of the result rows
    const int32_t *row_leaf;  // [T][rows] heap ids (fallback)
    int excl;
    double flops0, flops1;  // useful Gram flops of the Phase I / Phase II tiles (0 if unknown)
    double bytes0, bytes1;  // tile-operand bytes of the two phases
    bool sym;               // all-points with one tile per leaf: symmetric kernel
    int B;                  // trees of Phase I
    const TileJob *sjobs0 = nullptr, *sjobs1 = nullptr;  // query groups of <= qs rows (GEMV-shaped)
    int64_t nsjobs0 = 0, nsjobs1 = 0;
};

// group size and chunks per lane of the GEMV-shaped query kernel (64 registers of query per
// lane); 0 = every job goes to the MFMA tiles
static int qtile_qs(int prec, int dp) {
    if (dp <= 128) return 4;
    if (dp <= 256) return 2;
    if (dp <= 512) return 1;
    return 0;
}

template <int PREC, int QS, int NCH>
static void qtile_launch(hipStream_t s, int64_t njobs, const TileJob *jobs, const void *A, const void *B, int dp,
                         int64_t as, int64_t bs, const float2 *an, const float2 *bn, const int32_t *ad,
                         const int32_t *bp, BoundCoef bc, const TileOut &out) {
    if (njobs <= 0) return;
    hipLaunchKernelGGL((k_qtile<PREC, QS, NCH>), dim3((unsigned)((njobs + 3) / 4)), dim3(256), 0, s, jobs, njobs, A, B,
                       dp, as, bs, an, bn, ad, bp, bc, out);
    launch_check(s, "k_qtile");
}

template <int PREC>
static void qtile_dispatch_p(int qs, hipStream_t s, int64_t njobs, const TileJob *jobs, const void *A, const void *B,
                             int dp, int64_t as, int64_t bs, const float2 *an, const float2 *bn, const int32_t *ad,
                             const int32_t *bp, BoundCoef bc, const TileOut &out) {
    constexpr int E = PREC == RPF_DIST_FP32 ? 4 : 8;  // elements per 16-byte chunk
    if (qs == 4)
        qtile_launch<PREC, 4, 128 / (8 * E)>(s, njobs, jobs, A, B, dp, as, bs, an, bn, ad, bp, bc, out);
    else if (qs == 2)
        qtile_launch<PREC, 2, 256 / (8 * E)>(s, njobs, jobs, A, B, dp, as, bs, an, bn, ad, bp, bc, out);
    else if (qs == 1)
        qtile_launch<PREC, 1, 512 / (8 * E)>(s, njobs, jobs, A, B, dp, as, bs, an, bn, ad, bp, bc, out);
}

static void qtile_dispatch(int prec, int qs, hipStream_t s, int64_t njobs, const TileJob *jobs, const void *A,
                           const void *B, int dp, int64_t as, int64_t bs, const float2 *an, const float2 *bn,
                           const int32_t *ad, const int32_t *bp, BoundCoef bc, const TileOut &out) {
    if (prec == RPF_DIST_BF16)
        qtile_dispatch_p<RPF_DIST_BF16>(qs, s, njobs, jobs, A, B, dp, as, bs, an, bn, ad, bp, bc, out);
    else if (prec == RPF_DIST_FP16)
        qtile_dispatch_p<RPF_DIST_FP16>(qs, s, njobs, jobs, A, B, dp, as, bs, an, bn, ad, bp, bc, out);
    else
        qtile_dispatch_p<RPF_DIST_FP32>(qs, s, njobs, jobs, A, B, dp, as, bs, an, bn, ad, bp, bc, out);
}

// the all-points tiles of one leaf each, staged from X and the leaf centroids
struct SymSrc {
    const float *X;
    int d, dp;
    const float *centroid;
    int nleaf;
    int64_t stride;  // points per tree (n)
};

static SymSrc sym_src(const ForestView &v) { return SymSrc{v.X, v.d, v.dp, v.centroid, (int)v.nleaf, v.n}; }

// Phase II into per-tree buckets with tile shape SH
template <int NB, int PREC, int SH>
static void sym_launch_p2(hipStream_t s, const dim3 g, const TileJob *jobs, const SymSrc &src, const float2 *nrm,
                          const int32_t *pt, BoundCoef bc, int excl, const TileOut &out) {
    hipLaunchKernelGGL((k_tile_sym<NB, PREC, 2, SH>), g, dim3(64 * sym_waves(NB, 2, SH)), 0, s, jobs, src.X, src.d,
                       src.dp, src.centroid, src.nleaf, src.stride, nrm, pt, bc, excl, out);
}

// the shapes a block-count NB offers: none at NB = 1, the chunk and queue bits at 2 and 4,
// all three at 8
constexpr int sym_shape_mask(int NB) { return NB == 1 ? 0 : NB == 8 ? 7 : 3; }

template <int NB, int PREC>
static void sym_launch(hipStream_t s, int64_t njobs, const TileJob *jobs, const SymSrc &src, const float2 *nrm,
                       const int32_t *pt, BoundCoef bc, int excl, const TileOut &out) {
    if (njobs <= 0) return;
    const int NT = 64 * sym_waves(NB, out.mode);
    const dim3 g((unsigned)njobs);
    if (out.mode == 0) {
        hipLaunchKernelGGL((k_tile_sym<NB, PREC, 0>), g, dim3(NT), 0, s, jobs, src.X, src.d, src.dp, src.centroid,
                           src.nleaf, src.stride, nrm, pt, bc, excl, out);
    } else if (out.bcnt) {  // Phase II into per-tree buckets
        switch (out.shape & sym_shape_mask(NB)) {
        case 1: sym_launch_p2<NB, PREC, 1 & sym_shape_mask(NB)>(s, g, jobs, src, nrm, pt, bc, excl, out); break;
        case 2: sym_launch_p2<NB, PREC, 2 & sym_shape_mask(NB)>(s, g, jobs, src, nrm, pt, bc, excl, out); break;
        case 3: sym_launch_p2<NB, PREC, 3 & sym_shape_mask(NB)>(s, g, jobs, src, nrm, pt, bc, excl, out); break;
        case 4: sym_launch_p2<NB, PREC, 4 & sym_shape_mask(NB)>(s, g, jobs, src, nrm, pt, bc, excl, out); break;
        case 5: sym_launch_p2<NB, PREC, 5 & sym_shape_mask(NB)>(s, g, jobs, src, nrm, pt, bc, excl, out); break;
        case 6: sym_launch_p2<NB, PREC, 6 & sym_shape_mask(NB)>(s, g, jobs, src, nrm, pt, bc, excl, out); break;
        case 7: sym_launch_p2<NB, PREC, 7 & sym_shape_mask(NB)>(s, g, jobs, src, nrm, pt, bc, excl, out); break;
        default: sym_launch_p2<NB, PREC, 0>(s, g, jobs, src, nrm, pt, bc, excl, out); break;
        }
    } else
        hipLaunchKernelGGL((k_tile_sym<NB, PREC, 1>), g, dim3(NT), 0, s, jobs, src.X, src.d, src.dp, src.centroid,
                           src.nleaf, src.stride, nrm, pt, bc, excl, out);
    launch_check(s, "k_tile_sym");
}

template <int PREC>
static void sym_dispatch_nb(int NB, hipStream_t s, int64_t njobs, const TileJob *jobs, const SymSrc &src,
                            const float2 *nrm, const int32_t *pt, BoundCoef bc, int excl, const TileOut &out) {
    switch (NB) {
    case 1: sym_launch<1, PREC>(s, njobs, jobs, src, nrm, pt, bc, excl, out); break;
    case 2: sym_launch<2, PREC>(s, njobs, jobs, src, nrm, pt, bc, excl, out); break;
    case 4: sym_launch<4, PREC>(s, njobs, jobs, src, nrm, pt, bc, excl, out); break;
    default: sym_launch<8, PREC>(s, njobs, jobs, src, nrm, pt, bc, excl, out); break;
    }
}

static void sym_dispatch(int prec, int NB, hipStream_t s, int64_t njobs, const TileJob *jobs, const SymSrc &src,
                         const float2 *nrm, const int32_t *pt, BoundCoef bc, int excl, const TileOut &out) {
    if (prec == RPF_DIST_BF16X3)
        sym_dispatch_nb<RPF_DIST_BF16X3>(NB, s, njobs, jobs, src, nrm, pt, bc, excl, out);
    else if (prec == RPF_DIST_BF16)
        sym_dispatch_nb<RPF_DIST_BF16>(NB, s, njobs, jobs, src, nrm, pt, bc, excl, out);
    else if (prec == RPF_DIST_FP16)
        sym_dispatch_nb<RPF_DIST_FP16>(NB, s, njobs, jobs, src, nrm, pt, bc, excl, out);
    else
        sym_dispatch_nb<RPF_DIST_FP32>(NB, s, njobs, jobs, src, nrm, pt, bc, excl, out);
}

// device buffers of the candidate stage (one call)
// Per-row record capacities of a candidate stage.  want2 sizes the wave merge (the Phase II
// records a row is expected to hold at most); cap2 is the row's Phase II record area.  In
// bucket mode (S > 0) the area is nT2 buckets of S records, one per Phase II tree, then an
// overflow list of capO records.
struct RecLayout {
    int lcap = 0, want2 = 0, cap2 = 0;
    int S = 0, nT2 = 0, capO = 0;
};

struct CandWs {
    int lcap = 0, cap1 = 0, cap2 = 0;
    RecLayout lay;
    uint8_t *region = nullptr;  // Phase I index / lb / ub arrays, then the Phase II records
    float *tau = nullptr;
    int32_t *cnt = nullptr, *lcnt = nullptr, *fb_list = nullptr, *fb_cnt = nullptr;
    Ent *list = nullptr;
    uint8_t *bcnt = nullptr;    // bucket mode: per-(row, Phase II tree) record counts
};

// Per-row capacities of the merged list and of the Phase II records, from K and the number
// of Phase II trees (about K (T - B) / 2 records per row were measured on mixtures; twice that
// plus a margin keeps overflow, which sends a row to the exhaustive path, rare).
//
// When that exceeds one wave's records (many trees, or a large K), the buffers take up to
// kBigCap records per row as long as the Phase II buffers of all rows stay within kBigBudget
// bytes: rows that outgrow the wave merge then go to the block-per-row merge rather than to
// the exhaustive path.
constexpr uint64_t kBigBudget = (uint64_t)32 << 30;
static void cand_caps(int K, int T, int B, int64_t rows, int &lcap, int &cap2) {
    lcap = std::min(kListCap, std::max(64, 8 * K));
    const int want = std::max(128, K * std::max(T - B, 0) + 64);
    cap2 = std::min(kFinalCap - lcap, want);
    if (want > kFinalCap - lcap) {
        const int big = std::min(kBigCap - lcap, want);
        if ((uint64_t)std::max<int64_t>(rows, 1) * big * sizeof(Ent) <= kBigBudget) cap2 = big;
    }
}

// Bucket mode: the all-points symmetric tiles, where one block holds every pair of a row in
// its tree, so a row's records of one tree are ranked in LDS and need no device-scope atomic.
// A row's records in one tree are about its neighbours among the leaf's rows, so they grow
// with K: S = the power of two at or above K within [16, 64], halved (to 4 at least) until
// the area fits kBucketBudget; the overflow list holds max(128, 2K).  Each bucket's count is
// a byte.
constexpr int kMaxBucketTrees = 128;   // buckets per row (two per lane of the merge's wave)
constexpr int kBucketOverflow = 128;   // overflow records per row, at least
constexpr uint64_t kBucketBudget = (uint64_t)40 << 30;

// RPF_BUCKET_S (1 .. 16) fixes the bucket size instead, so that tests can drive most records
// through the overflow list and its hand-over to the block merge and the exhaustive path.
static int bucket_size_override() {
    const char *e = getenv("RPF_BUCKET_S");
    const int v = e ? atoi(e) : 0;
    return v >= 1 && v <= 16 ? v : 0;
}

static RecLayout rec_layout(int K, int T, int B, int64_t rows, bool buckets, int want_S = 0) {
    RecLayout r;
    cand_caps(K, T, B, rows, r.lcap, r.cap2);
    r.want2 = r.cap2;
    const int nT2 = T - B;
    if (buckets && nT2 >= 1 && nT2 <= kMaxBucketTrees) {
        const int forced = bucket_size_override() ? bucket_size_override() : std::min(want_S, 64);
        const int capO = std::max(kBucketOverflow, 2 * K);
        int S0 = 16;
        while (S0 < K && S0 < 64) S0 *= 2;
        for (int S = forced ? forced : S0; S >= (forced ? forced : 4); S /= 2) {
            const int cap2 = nT2 * S + capO;
            if ((uint64_t)std::max<int64_t>(rows, 1) * cap2 * sizeof(Ent) <= kBucketBudget) {
                r.S = S;
                r.nT2 = nT2;
                r.capO = capO;
                r.cap2 = cap2;
                break;
            }
            if (forced) break;
        }
    }
    return r;
}

static bool phase2_buckets(const ForestView &v, const CandStage &cs) {
    return cs.all_points && cs.sym && v.sym_prec != RPF_DIST_U8GRID;
}

static RecLayout stage_layout(const ForestView &v, const CandStage &cs, int K) {
    return rec_layout(K, v.T, cs.B, cs.rows, phase2_buckets(v, cs), cs.bucket_S);
}

static void set_layout(CandWs &w, const RecLayout &lay) {
    w.lay = lay;
    w.lcap = lay.lcap;
    w.cap2 = lay.cap2;
}

// first-phase slots per (row, tree): the largest leaf, but at most the leaf size n0 (only a
// uniform-rule leaf kept whole at the depth cap or over duplicates exceeds it; the rows of
// such a leaf in a first-phase tree take the exhaustive path)
static int first_slot_leaf(const ForestView &v) { return std::min(v.max_leaf, std::max(v.n0, 1)); }
static int first_slot_stride(const ForestView &v) { return slot_stride(first_slot_leaf(v)); }


// Phase I keeps every pair of a row's first B leaves; Phase II keeps pairs below the
// threshold of the union of those leaves.  `get` hands out device bytes (nullptr = failure).
template <typename Get>
static bool cand_ws_alloc(const ForestView &v, const CandStage &cs, int K, Get get, CandWs &w) {
    const int64_t rows = cs.rows;
    set_layout(w, stage_layout(v, cs, K));
    w.cap1 = first_slot_stride(v) * cs.B;  // Phase I slots per row (bounds)
    // the Phase II records reuse the Phase I arrays, dead once the first merge has run
    const size_t first_bytes = (size_t)rows * w.cap1 * 4 + (size_t)rows * cs.B * 4;  // slots, leaf starts
    const size_t second_bytes = (size_t)rows * w.cap2 * sizeof(Ent);
    w.region = static_cast<uint8_t *>(get(std::max(first_bytes, second_bytes) + 256));
    w.tau = static_cast<float *>(get(rows * 4));
    w.cnt = static_cast<int32_t *>(get(rows * 4));
    w.list = static_cast<Ent *>(get((size_t)rows * w.lcap * sizeof(Ent)));
    w.lcnt = static_cast<int32_t *>(get(rows * 4));
    w.fb_list = static_cast<int32_t *>(get(rows * 8));  // fallback rows, then block-merge rows
    w.fb_cnt = static_cast<int32_t *>(get(16));
    if (w.lay.S) w.bcnt = static_cast<uint8_t *>(get((size_t)rows * w.lay.nT2));
    return w.region && w.tau && w.cnt && w.list && w.lcnt && w.fb_list && w.fb_cnt && (!w.lay.S || w.bcnt);
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t count, uint32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// a small fill kernel rather than a memset, so the launch sequence can be recorded in a graph
void fill_u32(void *p, int64_t count, uint32_t value, hipStream_t s) {
    if (count <= 0) return;
    const unsigned blocks = (unsigned)std::min<int64_t>((count + 255) / 256, 2048);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, static_cast<uint32_t *>(p), count, value);
    launch_check(s, "k_fill_u32");
}

__global__ void k_fill_u64(uint64_t *__restrict__ p, int64_t count, uint64_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

void fill_u64(void *p, int64_t count, uint64_t value, hipStream_t s) {
    if (count <= 0) return;
    const unsigned blocks = (unsigned)std::min<int64_t>((count + 255) / 256, 2048);
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks), dim3(256), 0, s, static_cast<uint64_t *>(p), count, value);
    launch_check(s, "k_fill_u64");
}

// Every tree has the same leaf shapes, so the all-points tile list of tree 0 (jobs[0, njt))
// is copied to trees 1 .. T - 1 with only the tree field changed.
__global__ void k_replicate_jobs(TileJob *__restrict__ jobs, int64_t njt, int T) {
    const int64_t total = njt * (T - 1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i / njt + 1, j = i - (t - 1) * njt;
        TileJob jb = jobs[j];
        jb.tree = (int32_t)t;
        jobs[t * njt + j] = jb;
    }
}

void replicate_jobs(TileJob *jobs, int64_t njt, int T, hipStream_t s) {
    if (njt <= 0 || T <= 1) return;
    const unsigned blocks = (unsigned)std::min<int64_t>((njt * (T - 1) + 255) / 256, 4096);
    hipLaunchKernelGGL(k_replicate_jobs, dim3(blocks), dim3(256), 0, s, jobs, njt, T);
    launch_check(s, "k_replicate_jobs");
}

// the candidate stage as launches only (no allocation, no synchronisation)
static void cand_launches(const ForestView &v, const CandStage &cs, int K, const CandWs &w, int32_t *out_idx,
                          float *out_dist, hipStream_t s) {
    const int64_t rows = cs.rows;
    const int lcap = w.lcap, cap1 = w.cap1, cap2 = w.cap2;
    uint8_t *region = w.region;
    float *tau = w.tau;
    int32_t *cnt = w.cnt, *lcnt = w.lcnt, *fb_list = w.fb_list, *fb_cnt = w.fb_cnt;
    Ent *list = w.list;
    Ent *ent = reinterpret_cast<Ent *>(region);
    uint32_t *plub = reinterpret_cast<uint32_t *>(region);
    int32_t *roff = reinterpret_cast<int32_t *>(region + (size_t)rows * cap1 * 4);
    fill_u32(cnt, rows, 0, s);
    fill_u32(fb_cnt, 4, 0, s);
    fill_u32(v.stats, kStatSlots * 8 * 2, 0, s);
    const BoundCoef bc = bound_coef(v.prec, v.d);
    // the all-points symmetric tiles may run split bfloat16 over a binary32 forest
    const BoundCoef bc_sym = v.sym_prec == v.prec ? bc : bound_coef(v.sym_prec, v.d);
    const int MB = v.job_mb;
    TileOut o1;
    o1.mode = 0;
    o1.t0 = 0;
    o1.ML = first_slot_stride(v);
    o1.cap = cap1;
    o1.ent = nullptr;
    o1.cnt = cnt;
    o1.tau = nullptr;
    o1.plub = plub;
    o1.roff = roff;
    o1.nrows = rows;
    o1.bcnt = nullptr;
    o1.t1 = 0;
    o1.S = 0;
    o1.nT2 = 0;
    o1.capO = 0;
    o1.shape = 0;
    const bool grid = v.sym_prec == RPF_DIST_U8GRID && cs.all_points;
    auto grid_launch = [&](const TileJob *jobs, int64_t njobs, const TileOut &o) {
        if (njobs <= 0) return;
        const dim3 g((unsigned)(8 * ((njobs + 7) / 8)));
        switch (v.job_mb) {
            case 1: hipLaunchKernelGGL(k_tile_q8<1>, g, dim3(64), 0, s, jobs, njobs, v.Xq, v.dq, v.qn, v.perm, v.n, cs.excl, o); break;
            case 2: hipLaunchKernelGGL(k_tile_q8<2>, g, dim3(128), 0, s, jobs, njobs, v.Xq, v.dq, v.qn, v.perm, v.n, cs.excl, o); break;
            case 4: hipLaunchKernelGGL(k_tile_q8<4>, g, dim3(256), 0, s, jobs, njobs, v.Xq, v.dq, v.qn, v.perm, v.n, cs.excl, o); break;
            default: hipLaunchKernelGGL(k_tile_q8<8>, g, dim3(512), 0, s, jobs, njobs, v.Xq, v.dq, v.qn, v.perm, v.n, cs.excl, o); break;
        }
        launch_check(s, "k_tile_q8");
    };
    {
        ProfScope ps(s, "tile_phase1", cs.bytes0, cs.flops0);
        if (grid)
            grid_launch(cs.jobs0, cs.njobs0, o1);
        else if (cs.sym)
            sym_dispatch(v.sym_prec, MB, s, cs.njobs0, cs.jobs0, sym_src(v), v.nrm, v.perm, bc_sym, cs.excl, o1);
        else
            tile_dispatch(v.prec, MB, s, cs.njobs0, cs.jobs0, cs.A, v.Xc, v.dp, cs.a_stride, v.n, cs.a_nrm, v.nrm,
                          cs.a_dest, v.perm, bc, cs.excl, o1);
        qtile_dispatch(v.prec, qtile_qs(v.prec, v.dp), s, cs.nsjobs0, cs.sjobs0, cs.A, v.Xc, v.dp, cs.a_stride, v.n,
                       cs.a_nrm, v.nrm, cs.a_dest, v.perm, bc, o1);
    }
    {
        ProfScope ps(s, "merge_first", 0, 0);
        // the smallest per-lane slot count that holds the row's B x max_leaf slots
        const dim3 mg((unsigned)((rows + 3) / 4));
        // hash table of the small set: room for twice its largest regular size (K B entries
        // plus ties)
        const bool big = K * cs.B > 128;
        const SlotIndex si{roff, v.perm, v.n};
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, mg, dim3(256), 0, s, rows, K, cs.B, first_slot_stride(v), plub, si, cap1, tau, list,
                               lcnt, lcap, cnt);
        };
        switch (merge_first_q(cap1)) {
            case 4: big ? go(k_merge_first<4, 1024>) : go(k_merge_first<4, 512>); break;
            case 8: big ? go(k_merge_first<8, 1024>) : go(k_merge_first<8, 512>); break;
            case 16: big ? go(k_merge_first<16, 1024>) : go(k_merge_first<16, 512>); break;
            default: big ? go(k_merge_first<kMergeCap / 64, 1024>) : go(k_merge_first<kMergeCap / 64, 512>); break;
        }
        launch_check(s, "k_merge_first");
    }
    if (cs.njobs1 > 0 || cs.nsjobs1 > 0) {
        TileOut o2 = o1;
        o2.mode = 1;
        o2.cap = cap2;
        o2.tau = tau;
        o2.ent = ent;
        if (w.lay.S) {  // rows' records in per-tree buckets (k_tile_sym only)
            o2.shape = cs.shape;
            o2.bcnt = w.bcnt;
            o2.t1 = cs.B;
            o2.S = w.lay.S;
            o2.nT2 = w.lay.nT2;
            o2.capO = w.lay.capO;
        }
        ProfScope ps(s, "tile_phase2", cs.bytes1, cs.flops1);
        if (grid)
            grid_launch(cs.jobs1, cs.njobs1, o2);
        else if (cs.sym)
            sym_dispatch(v.sym_prec, MB, s, cs.njobs1, cs.jobs1, sym_src(v), v.nrm, v.perm, bc_sym, cs.excl, o2);
        else
            tile_dispatch(v.prec, MB, s, cs.njobs1, cs.jobs1, cs.A, v.Xc, v.dp, cs.a_stride, v.n, cs.a_nrm, v.nrm,
                          cs.a_dest, v.perm, bc, cs.excl, o2);
        qtile_dispatch(v.prec, qtile_qs(v.prec, v.dp), s, cs.nsjobs1, cs.sjobs1, cs.A, v.Xc, v.dp, cs.a_stride, v.n,
                       cs.a_nrm, v.nrm, cs.a_dest, v.perm, bc, o2);
    }
    FinalArgs fa;
    fa.list = list; fa.lcnt = lcnt; fa.lcap = lcap; fa.cnt = cnt; fa.ent = ent; fa.cap = cap2; fa.K = K;
    fa.X = v.X; fa.Qr = cs.Qr; fa.d = v.d; fa.win = rerank_window(v.d); fa.out_idx = out_idx;
    fa.out_dist = out_dist; fa.fb_list = fb_list; fa.fb_cnt = fb_cnt; fa.npts = v.n;
    fa.stats = v.stats;
    fa.fault = v.fault;
    fa.bcnt = w.lay.S ? w.bcnt : nullptr;
    fa.S = w.lay.S;
    fa.nT2 = w.lay.nT2;
    fa.capO = w.lay.capO;
    const bool vec = (v.d % 4) == 0;
    {
        ProfScope ps(s, "final_rerank", 0, 0);
        const size_t lds = 4 * sizeof(float) * (size_t)((v.d + 3) & ~3);
        const dim3 grid((unsigned)((rows + 3) / 4));
        // the smallest per-lane record count that holds the list and the Phase II records
        // a row is expected to have (in bucket mode the record area is larger than that)
        const int need = lcap + w.lay.want2;
        // records per lane of the wave merge: the smallest that holds the capacity, at most 12;
        // 16 for bf16 / fp16 tiles when the capacity passes 1024 (their looser bounds emit more
        // records per row, which would otherwise send many rows to the slower block merge)
        const int wq = need <= 256 ? 4 : need <= 512 ? 8 : (need > 1024 && v.prec != RPF_DIST_FP32) ? 16 : 12;
        // second half of the row lists; in bucket mode any row may outgrow the wave merge
        fa.big_list = (need > 64 * wq || w.lay.S) ? fb_list + rows : nullptr;
        fa.big_cnt = fb_cnt + 1;
        if (need > kFinalCap && K > 64) {  // one block per row
            if (vec) hipLaunchKernelGGL((k_final_blk<true, false>), dim3((unsigned)rows), dim3(256), lds / 4, s, fa);
            else hipLaunchKernelGGL((k_final_blk<false, false>), dim3((unsigned)rows), dim3(256), lds / 4, s, fa);
        } else if (need <= 256) {
            if (vec) hipLaunchKernelGGL((k_final<true, 4>), grid, dim3(256), lds, s, fa, rows);
            else hipLaunchKernelGGL((k_final<false, 4>), grid, dim3(256), lds, s, fa, rows);
        } else if (need <= 512) {
            if (vec) hipLaunchKernelGGL((k_final<true, 8>), grid, dim3(256), lds, s, fa, rows);
            else hipLaunchKernelGGL((k_final<false, 8>), grid, dim3(256), lds, s, fa, rows);
        } else {
            if (wq == 16) {
                if (vec) hipLaunchKernelGGL((k_final<true, 16>), grid, dim3(256), lds, s, fa, rows);
                else hipLaunchKernelGGL((k_final<false, 16>), grid, dim3(256), lds, s, fa, rows);
            } else {
                if (vec) hipLaunchKernelGGL((k_final<true, kFinalQ>), grid, dim3(256), lds, s, fa, rows);
                else hipLaunchKernelGGL((k_final<false, kFinalQ>), grid, dim3(256), lds, s, fa, rows);
            }
            if (fa.big_list) {  // the rows the wave merge handed over
                const dim3 gb((unsigned)std::max<int64_t>(1, std::min<int64_t>(rows, 2048)));
                if (vec) hipLaunchKernelGGL((k_final_blk<true, true>), gb, dim3(256), lds / 4, s, fa);
                else hipLaunchKernelGGL((k_final_blk<false, true>), gb, dim3(256), lds / 4, s, fa);
            }
        }
        launch_check(s, "k_final");
    }
    FallbackArgs fb;
    fb.fb_list = fb_list; fb.fb_cnt = fb_cnt; fb.X = v.X; fb.Qr = cs.Qr; fb.d = v.d; fb.K = K; fb.T = v.T;
    fb.n = v.n; fb.perm = v.perm; fb.row_leaf = cs.row_leaf; fb.nrows = rows; fb.heap_leaf = v.heap_leaf;
    fb.leaves = v.leaves; fb.leaf_stride = v.leaf_stride; fb.exclude_self = cs.excl; fb.out_idx = out_idx;
    fb.out_dist = out_dist;
    {
        ProfScope ps(s, "fallback", 0, 0);
        const unsigned nb = (unsigned)std::min<int64_t>(rows, 1024);
        constexpr int NTH = kFallbackThreads;
        if (vec)
            hipLaunchKernelGGL((k_fallback<true, NTH>), dim3(nb), dim3(NTH), v.d * 4, s, fb);
        else
            hipLaunchKernelGGL((k_fallback<false, NTH>), dim3(nb), dim3(NTH), v.d * 4, s, fb);
        launch_check(s, "k_fallback");
    }
}

// the candidate stage with its buffers from `get` (device bytes, nullptr = failure)
template <typename Get>
static rpf_status run_cand_stage_get(const ForestView &v, const CandStage &cs, int K, int32_t *out_idx,
                                     float *out_dist, hipStream_t s, Get get) {
    CandWs w;
    if (!cand_ws_alloc(v, cs, K, get, w)) return fail(RPF_ENOMEM, "kNN workspace allocation failed");
    cand_launches(v, cs, K, w, out_idx, out_dist, s);
    const std::string le = take_launch_error();
    if (!le.empty()) return fail(RPF_EDEVICE, "kNN: " + le);
    return RPF_OK;
}

static rpf_status run_cand_stage(const ForestView &v, const CandStage &cs, int K, int32_t *out_idx,
                                 float *out_dist, hipStream_t s) {
    Workspace ws(s);
    return run_cand_stage_get(v, cs, K, out_idx, out_dist, s, [&](size_t b) { return ws.get<void>(b); });
}

// largest first-phase tree count the merge supports for this forest and K
static int max_first_trees(const ForestView &v, int K) { return max_first_trees_for(v.T, K, first_slot_leaf(v)); }

// Default first-phase trees of the all-points search: kFirstTrees, or twice that for bf16 /
// fp16 tiles over 64 trees or more.  Their looser bounds emit more Phase II records per row,
// and the tighter threshold of more first-phase trees pays for itself there (the plan tuner
// picks 8 at 10^6 points, K 20, T 80 in bf16, and 4 in fp32 or at T 32).
static int all_points_first_trees(const ForestView &v, int K) {
    int want = (v.prec != RPF_DIST_FP32 && v.T >= 64) ? 2 * kFirstTrees : kFirstTrees;
    // uniform-rule trees: leaves of every size up to n0 (at 10^6 x 128, n0 256, a median of
    // about 40 points), so four trees' leaves hold too few candidates for a tight threshold.
    // (The slot stride is capped at n0: a leaf above it, which a deep chain of uneven splits
    // can leave at the depth cap, sends its rows to the exhaustive path instead of limiting
    // the count.)
    if (v.leaf_stride > 0) want = 2 * kFirstTrees;
    return std::min(want, max_first_trees(v, K));
}

static CandStage all_points_stage(const ForestView &v, int K, int exclude_self, int B = 0) {
    CandStage cs;
    cs.rows = v.n;
    cs.B = B > 0 ? std::min(B, max_first_trees(v, K)) : all_points_first_trees(v, K);
    cs.jobs0 = v.jobs;
    if (v.job_off) {  // trees with leaves of their own: tree t's tiles are jobs[job_off[t], job_off[t + 1])
        cs.jobs1 = v.jobs + v.job_off[cs.B];
        cs.njobs0 = v.job_off[cs.B];
        cs.njobs1 = v.job_off[v.T] - v.job_off[cs.B];
    } else {
        cs.jobs1 = v.jobs + v.n_jobs_tree * cs.B;
        cs.njobs0 = v.n_jobs_tree * cs.B;
        cs.njobs1 = v.n_jobs_tree * (v.T - cs.B);
    }
    cs.A = v.Xc;
    cs.a_stride = v.n;
    cs.a_nrm = v.nrm;
    cs.a_dest = v.perm;
    cs.Qr = v.X;
    cs.row_leaf = v.leaf_of;
    cs.excl = exclude_self;
    const double esz = v.prec == RPF_DIST_FP32 ? 4.0 : 2.0;
    cs.flops0 = v.flops_off ? v.flops_off[cs.B] : v.tile_flops_tree * cs.B;
    cs.flops1 = v.flops_off ? v.flops_off[v.T] - v.flops_off[cs.B] : v.tile_flops_tree * (v.T - cs.B);
    cs.bytes0 = (double)v.n * v.dp * esz * cs.B;
    cs.bytes1 = (double)v.n * v.dp * esz * (v.T - cs.B);
    cs.sym = v.max_leaf <= 32 * v.job_mb;  // every leaf is a single diagonal tile
    cs.all_points = true;
    if (v.sym_prec == RPF_DIST_U8GRID) {  // int8 rows
        cs.bytes0 = (double)v.n * v.dq * cs.B;
        cs.bytes1 = (double)v.n * v.dq * (v.T - cs.B);
    }
    return cs;
}

rpf_status knn_all(const rpf_forest *f, int K, int exclude_self, int32_t *out_idx, float *out_dist, hipStream_t s) {
    ForestView v = view(f);
    const CandStage cs = all_points_stage(v, K, exclude_self);
    if (!cs.sym && !v.Xc && v.sym_prec != RPF_DIST_U8GRID) {  // leaves of more than one tile read the centred copy
        const rpf_status st = ensure_leaf_copies(f, s);
        if (st != RPF_OK) return st;
        v = view(f);
        return run_cand_stage(v, all_points_stage(v, K, exclude_self), K, out_idx, out_dist, s);
    }
    return run_cand_stage(v, cs, K, out_idx, out_dist, s);
}

// All-points search of several forests (parts) run one after the other with one workspace,
// sized for the largest part and the largest first-phase tree count it will be given: the
// launches can be recorded once and replayed.
struct KnnShared {
    int K = 0, excl = 0;
    std::vector<void *> blocks;
    CandWs w;  // base pointers; each part derives its capacities
};

KnnShared *knn_shared_create(const std::vector<const rpf_forest *> &parts, const std::vector<int> &maxB, int K,
                             int exclude_self, hipStream_t s) {
    KnnShared *p = new KnnShared();
    p->K = K;
    p->excl = exclude_self;
    size_t b_region = 0, b_rows = 0, b_list = 0, b_bcnt = 0;
    for (size_t i = 0; i < parts.size(); i++) {
        const ForestView v = view(parts[i]);
        const CandStage cs = all_points_stage(v, K, exclude_self, maxB[i]);
        // capacities grow with B for cap1 and shrink for cap2: take each over 1..B
        for (int B = 1; B <= cs.B; B++) {
            CandStage cb = cs;
            cb.B = B;
            const RecLayout lay = stage_layout(v, cb, K);
            const size_t cap1 = (size_t)first_slot_stride(v) * B;
            b_region = std::max(b_region, std::max((size_t)v.n * cap1 * 4 + (size_t)v.n * B * 4,
                                                   (size_t)v.n * lay.cap2 * sizeof(Ent)) + 256);
            b_list = std::max(b_list, (size_t)v.n * lay.lcap * sizeof(Ent));
            if (lay.S) b_bcnt = std::max(b_bcnt, (size_t)v.n * lay.nT2);
        }
        b_rows = std::max(b_rows, (size_t)v.n * 4);
    }
    auto get = [&](size_t b) {
        void *q = cache_alloc(b ? b : 16, s);
        if (q) p->blocks.push_back(q);
        return q;
    };
    CandWs &w = p->w;
    w.region = static_cast<uint8_t *>(get(b_region));
    w.tau = static_cast<float *>(get(b_rows));
    w.cnt = static_cast<int32_t *>(get(b_rows));
    w.list = static_cast<Ent *>(get(b_list));
    w.lcnt = static_cast<int32_t *>(get(b_rows));
    w.fb_list = static_cast<int32_t *>(get(2 * b_rows));  // fallback rows, then block-merge rows
    w.fb_cnt = static_cast<int32_t *>(get(16));
    if (b_bcnt) w.bcnt = static_cast<uint8_t *>(get(b_bcnt));
    if (!w.region || !w.tau || !w.cnt || !w.list || !w.lcnt || !w.fb_list || !w.fb_cnt || (b_bcnt && !w.bcnt)) {
        knn_shared_destroy(p, s);
        return nullptr;
    }
    return p;
}

// first-phase tree count actually used for a part (B = 0: the default rule)
int knn_part_first_trees(const rpf_forest *f, int K, int B) {
    const ForestView v = view(f);
    return all_points_stage(v, K, 0, B).B;
}

// the Phase II tile shapes the part's symmetric tiles offer (0: none but the default)
int knn_part_shape_mask(const rpf_forest *f, int K) {
    const ForestView v = view(f);
    const CandStage cs = all_points_stage(v, K, 0);
    if (!cs.sym || v.sym_prec == RPF_DIST_U8GRID) return 0;
    return v.job_mb == 1 ? sym_shape_mask(1) : v.job_mb == 2 ? sym_shape_mask(2) : v.job_mb == 4 ? sym_shape_mask(4)
                                                                                             : sym_shape_mask(8);
}

// the Phase II bucket size the default rule gives a part (0: no buckets)
int knn_part_bucket_size(const rpf_forest *f, int K, int B) {
    const ForestView v = view(f);
    const CandStage cs = all_points_stage(v, K, 0, B);
    return stage_layout(v, cs, K).S;
}

void knn_part_launch(const KnnShared *p, const rpf_forest *f, int B, int shape, int bucket_S, int32_t *out_idx,
                     float *out_dist, hipStream_t s) {
    const ForestView v = view(f);
    CandStage cs = all_points_stage(v, p->K, p->excl, B);
    cs.shape = shape;
    cs.bucket_S = bucket_S;
    CandWs w = p->w;
    set_layout(w, stage_layout(v, cs, p->K));
    w.cap1 = first_slot_stride(v) * cs.B;
    cand_launches(v, cs, p->K, w, out_idx, out_dist, s);
}

void knn_shared_destroy(KnnShared *p, hipStream_t s) {
    if (!p) return;
    for (void *q : p->blocks) cache_free(q, s);
    delete p;
}

rpf_status route(const rpf_forest *f, const float *Q, int64_t m, int32_t *out_leaf, hipStream_t s) {
    const ForestView v = view(f);
    const bool vec = (v.d % 4) == 0 && ((uintptr_t)Q % 16) == 0;
    dim3 grid((unsigned)((m + 31) / 32), v.T);
    ProfScope ps(s, "route", (double)m * v.T * (v.L * (8.0 * v.d + 16)), 0);
    if (vec)
        hipLaunchKernelGGL(k_route<true>, grid, dim3(256), 0, s, Q, m, v.d, v.R, v.H, v.n_try, v.chosen, v.split, v.n,
                           v.n0, out_leaf);
    else
        hipLaunchKernelGGL(k_route<false>, grid, dim3(256), 0, s, Q, m, v.d, v.R, v.H, v.n_try, v.chosen, v.split,
                           v.n, v.n0, out_leaf);
    launch_check(s, "k_route");
    const std::string le = take_launch_error();
    if (!le.empty()) return fail(RPF_EDEVICE, "route: " + le);
    return RPF_OK;
}

// The query search with every device buffer taken from `get` (device bytes, nullptr =
// failure): the library's cache (knn_query) or a fixed scratch area (rpf_query_noalloc).
// may_copy: the forest's leaf copies may be made (allocated) here on its first query.
template <typename Get>
static rpf_status knn_query_get(const rpf_forest *f, const float *Q, int64_t m, int K, int32_t *out_idx,
                                float *out_dist, hipStream_t s, Get get, bool may_copy) {
    {
        const rpf_status st = ensure_leaf_copies(f, s, may_copy);  // query tiles read the leaf-ordered copy
        if (st != RPF_OK) return st;
    }
    const ForestView v = view(f);
    {   // queries must be finite (one synchronisation)
        int32_t *flag = static_cast<int32_t *>(get(16));
        if (!flag) return fail(RPF_ENOMEM, "rpf_query: allocation");
        fill_u32(flag, 4, 0, s);
        launch_nonfinite(s, Q, m * v.d, flag);
        int32_t h = 0;
        hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, s);
        rpf_status st = check_hip(hipStreamSynchronize(s), "rpf_query input check");
        if (st != RPF_OK) return st;
        if (h) return fail(RPF_EINVAL, "rpf_query: Q holds NaN or Inf");
    }
    bool ok = true;
    auto take = [&](size_t bytes) {
        void *p = get(bytes ? bytes : 16);
        ok = ok && p;
        return p;
    };
    const int T = v.T;
    const int64_t nleaf = v.nleaf;
    const int TR = 32 * v.job_mb;
    const size_t esz = v.prec == RPF_DIST_FP32 ? 4 : 2;
    int32_t *qleaf = static_cast<int32_t *>(take((size_t)T * m * 4));
    int32_t *gcount = static_cast<int32_t *>(take((size_t)T * nleaf * 4));
    int32_t *goff = static_cast<int32_t *>(take((size_t)T * nleaf * 4));
    int32_t *gfill = static_cast<int32_t *>(take((size_t)T * nleaf * 4));
    int32_t *qorder = static_cast<int32_t *>(take((size_t)T * m * 4));
    int32_t *qgleaf = static_cast<int32_t *>(take((size_t)T * m * 4));
    void *Qc = take((size_t)T * m * v.dp * esz);
    float2 *qnrm = static_cast<float2 *>(take((size_t)T * m * 8));
    const int nbt = (v.max_leaf + TR - 1) / TR;
    const int nfirst = first_trees(T, K, first_slot_leaf(v));
    const int64_t jcap_tree = (m / TR + std::min<int64_t>(m, nleaf) + 1) * nbt;
    const int64_t jcap0 = jcap_tree * nfirst;
    const int64_t jcap1 = jcap_tree * (T > nfirst ? T - nfirst : 1);
    TileJob *jobs0 = static_cast<TileJob *>(take((size_t)jcap0 * sizeof(TileJob)));
    TileJob *jobs1 = static_cast<TileJob *>(take((size_t)jcap1 * sizeof(TileJob)));
    const int qs = qtile_qs(v.prec, v.dp);
    TileJob *sjobs0 = qs ? static_cast<TileJob *>(take((size_t)jcap0 * sizeof(TileJob))) : nullptr;
    TileJob *sjobs1 = qs ? static_cast<TileJob *>(take((size_t)jcap1 * sizeof(TileJob))) : nullptr;
    int32_t *njobs = static_cast<int32_t *>(take(16));
    if (!ok) return fail(RPF_ENOMEM, "rpf_query: workspace allocation failed");
    rpf_status st = route(f, Q, m, qleaf, s);
    if (st != RPF_OK) return st;
    fill_u32(gcount, (int64_t)T * nleaf, 0, s);
    fill_u32(gfill, (int64_t)T * nleaf, 0, s);
    fill_u32(njobs, 4, 0, s);
    const unsigned qb = (unsigned)std::min<int64_t>((m + 255) / 256, 1024);
    hipLaunchKernelGGL(k_group_count, dim3(qb, T), dim3(256), 0, s, qleaf, m, v.heap_leaf, nleaf, gcount);
    hipLaunchKernelGGL(k_group_scan, dim3(T), dim3(1024), 0, s, gcount, nleaf, goff);
    hipLaunchKernelGGL(k_group_fill, dim3(qb, T), dim3(256), 0, s, qleaf, m, v.heap_leaf, nleaf, goff, gfill, qorder,
                       qgleaf);
    const unsigned lb_ = (unsigned)std::min<int64_t>((nleaf + 255) / 256, 1024);
    hipLaunchKernelGGL(k_make_jobs, dim3(lb_, T), dim3(256), 0, s, gcount, goff, nleaf, v.leaves, TR, nfirst, qs,
                       jobs0, jobs1, sjobs0, sjobs1, njobs);
    launch_check(s, "query grouping");
    {
        dim3 g((unsigned)((m + 3) / 4), T);
        if (v.prec == RPF_DIST_BF16)
            hipLaunchKernelGGL(k_query_prep<__bf16>, g, dim3(256), 0, s, Q, m, v.d, v.dp, qorder, qgleaf, v.centroid,
                               nleaf, (__bf16 *)Qc, qnrm, 3.0e38f);
        else if (v.prec == RPF_DIST_FP16)
            hipLaunchKernelGGL(k_query_prep<_Float16>, g, dim3(256), 0, s, Q, m, v.d, v.dp, qorder, qgleaf,
                               v.centroid, nleaf, (_Float16 *)Qc, qnrm, 60000.f);
        else
            hipLaunchKernelGGL(k_query_prep<float>, g, dim3(256), 0, s, Q, m, v.d, v.dp, qorder, qgleaf, v.centroid,
                               nleaf, (float *)Qc, qnrm, 3.0e38f);
    }
    // the job counts are needed to size the tile grids: read them back (small, one sync)
    launch_check(s, "k_query_prep");
    int32_t nj[4] = {0, 0, 0, 0};
    hipMemcpyAsync(nj, njobs, 16, hipMemcpyDeviceToHost, s);
    st = check_hip(hipStreamSynchronize(s), "rpf_query grouping");
    if (st != RPF_OK) return st;
    {
        const std::string le = take_launch_error();
        if (!le.empty()) return fail(RPF_EDEVICE, "rpf_query: " + le);
    }
    CandStage cs;
    cs.rows = m;
    cs.jobs0 = jobs0;
    cs.jobs1 = jobs1;
    cs.B = nfirst;
    cs.njobs0 = nj[0];
    cs.njobs1 = T > nfirst ? nj[1] : 0;
    cs.sjobs0 = sjobs0;
    cs.sjobs1 = sjobs1;
    cs.nsjobs0 = nj[2];
    cs.nsjobs1 = T > nfirst ? nj[3] : 0;
    cs.A = Qc;
    cs.a_stride = m;
    cs.a_nrm = qnrm;
    cs.a_dest = qorder;
    cs.Qr = Q;
    cs.row_leaf = qleaf;
    cs.excl = 0;
    cs.flops0 = cs.flops1 = cs.bytes0 = cs.bytes1 = 0;
    cs.sym = false;
    return run_cand_stage_get(v, cs, K, out_idx, out_dist, s, get);
}

rpf_status knn_query(const rpf_forest *f, const float *Q, int64_t m, int K, int32_t *out_idx, float *out_dist,
                     hipStream_t s) {
    Workspace ws(s);
    return knn_query_get(f, Q, m, K, out_idx, out_dist, s, [&](size_t b) { return ws.get<void>(b); }, true);
}

// device bytes one knn_query call of m queries takes from the allocator (its workspace)
uint64_t query_workspace_bytes(const rpf_forest *f, int64_t m, int K) {
    const ForestView v = view(f);
    const int64_t T = v.T, nleaf = v.nleaf;
    const int TR = 32 * v.job_mb;
    const uint64_t esz = v.prec == RPF_DIST_FP32 ? 4 : 2;
    const int nbt = (v.max_leaf + TR - 1) / TR;
    const int B = first_trees(v.T, K, first_slot_leaf(v));
    const int64_t jcap_tree = (m / TR + std::min<int64_t>(m, nleaf) + 1) * nbt;
    uint64_t b = 0;
    b += (uint64_t)T * m * 4 * 3;                  // leaf per tree, order, group leaf
    b += (uint64_t)T * nleaf * 4 * 3;              // group counts, offsets, fill
    b += (uint64_t)T * m * v.dp * esz + (uint64_t)T * m * 8;  // centred queries and norms
    b += (uint64_t)jcap_tree * (B + (T > B ? T - B : 1)) * sizeof(TileJob) * (qtile_qs(v.prec, v.dp) ? 2 : 1);
    int lcap = 0, cap2 = 0;
    cand_caps(K, v.T, B, m, lcap, cap2);
    const uint64_t cap1 = (uint64_t)first_slot_stride(v) * B;
    b += std::max(m * cap1 * 4 + m * (uint64_t)B * 4, m * (uint64_t)cap2 * sizeof(Ent)) + 256;
    b += (uint64_t)m * 4 * 5 + (uint64_t)m * lcap * sizeof(Ent) + 16 * 3;
    return b + (uint64_t)16 * 4096;  // allocator rounding of the ~16 blocks
}

}  // namespace rpf

// ---------------------------------------------------------------- allocation-free queries

// A fixed scratch area per device for callers that cannot allocate device memory: the
// workspace of rpf_query_noalloc is carved from it.  The name `scratch` is a host-side
// stand-in for the device array; host code uses only the device address obtained for it
// with hipGetSymbolAddress, per device, on the first call made on that device.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace rpf {
namespace {

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// the device address of this device's scratch array (nullptr on failure, with the error)
void *scratch_of(int dev, hipError_t &err) {
    std::call_once(g_scratch_once[dev], [dev] {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_err[dev] = e;
        g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
    });
    err = g_scratch_err[dev];
    return g_scratch_ptr[dev];
}

// bump allocation from the scratch area, 256-byte aligned
struct Arena {
    uint8_t *base;
    size_t cap, used = 0;
    void *get(size_t bytes) {
        const size_t at = (used + 255) & ~(size_t)255;
        if (at + bytes > cap) return nullptr;
        used = at + bytes;
        return base + at;
    }
};

}  // namespace
}  // namespace rpf

extern "C" rpf_status rpf_query_noalloc(const rpf_forest *f, const float *Q, int64_t m, int32_t K, int32_t *out_idx,
                                        float *out_dist, void *stream) {
    using namespace rpf;
    if (!f) return fail(RPF_EINVAL, "rpf_query_noalloc: forest is NULL");
    if (m < 0) return fail(RPF_EINVAL, "rpf_query_noalloc: m must be >= 0");
    if (m == 0) return RPF_OK;
    if (!Q || !out_idx || !out_dist) return fail(RPF_EINVAL, "rpf_query_noalloc: NULL pointer");
    if (K < 1 || K > forest_points(f)) return fail(RPF_EINVAL, "rpf_query_noalloc: K must be in [1, n]");
    if (K > 256) return fail(RPF_EINVAL, "rpf_query_noalloc: K above 256 is not supported");
    if (forest_batch_count(f) > 1) return fail(RPF_EINVAL, "rpf_query_noalloc: the forest holds several data sets");
    if (forest_uniform(f)) return fail(RPF_EINVAL, "rpf_query_noalloc: queries need a median-rule forest");
    if (forest_fault_seen(f)) return fault_error(f, "rpf_query_noalloc");
    const uint64_t need = query_workspace_bytes(f, m, K);  // an upper bound of the carve below
    if (need > kScratchBytes)
        return fail(RPF_EINVAL, "rpf_query_noalloc: m = " + std::to_string(m) + " queries at K = " + std::to_string(K) +
                                    " need " + std::to_string(need) + " bytes of workspace, above the " +
                                    std::to_string(kScratchBytes) + "-byte scratch area: use fewer queries per call");
    int dev = 0;
    rpf_status st = check_hip(hipGetDevice(&dev), "rpf_query_noalloc");
    if (st != RPF_OK) return st;
    if (dev < 0 || dev >= kMaxDevices) return fail(RPF_EINVAL, "rpf_query_noalloc: device index out of range");
    hipError_t err = hipSuccess;
    void *base = scratch_of(dev, err);
    if (!base) return check_hip(err == hipSuccess ? hipErrorInvalidSymbol : err, "rpf_query_noalloc: scratch address");
    Arena ar{static_cast<uint8_t *>(base), kScratchBytes};
    hipStream_t s = (hipStream_t)stream;
    st = knn_query_get(f, Q, m, K, out_idx, out_dist, s, [&](size_t b) { return ar.get(b); }, false);
    if (st == RPF_ENOMEM) return fail(RPF_EINTERNAL, "rpf_query_noalloc: the scratch carve exceeded its bound");
    return st != RPF_OK ? st : search_tail(f, s, "rpf_query_noalloc");
}
