// Exact kNN by brute force: the plain definition of the problem the forest approximates
// (Sec. 1: the K points of U nearest to each query), used as the ground truth of the
// accuracy measures of Sec. 5.1 at full data size.
//
// Every (query, point) pair gets its canonical binary64 squared distance D (32 classes of
// fma(delta, delta, s), the same tree as the rest of the library), and each query keeps the
// K points of smallest key (D, index).  Two kernels per chunk of queries:
//   k_exact_dist    D for a chunk of queries against all n points, written to a
//                   [chunk][n] binary64 buffer (a point row is read once per 8 x QL queries:
//                   it stays in registers while the lane group walks the chunk's queries,
//                   which sit in LDS);
//   k_exact_select  one 1024-thread block per query: radix select of the K-th smallest
//                   96-bit key (D bits, index) with 11-bit digits and LDS histograms, stopping
//                   once the key's bucket holds at most 2048 entries; one more pass gathers the
//                   entries below the bucket and the bucket itself; a bitonic sort in LDS
//                   orders the bucket and then the K results.
// Both are HBM / fp64-bound: per pair d binary64 subtractions and fmas; per query a few
// 8-byte reads of its n distances.
#include <math.h>

#include <algorithm>
#include <string>

#include "rpf_internal.h"

namespace rpf {
namespace {

constexpr int kQL = 64;          // most queries of a distance block held in LDS (8 per pass)
constexpr int kSelThreads = 1024;
constexpr int kSelBins = 2048;   // 11-bit digits
constexpr int kSelCand = 2048;   // bucket size at which the select gathers and sorts
constexpr uint64_t kInfBits = 0x7ff0000000000000ull;

// D[r][j] for queries q0 + r (r < nq) of this launch and every point j.  NR > 0: d <= 32 NR,
// d % 4 == 0 and 16-byte rows: each lane holds its NR float4 of the point row in registers.
// NR == 0: any d, the row is re-read (from cache) per group of 8 queries.
template <int NR>
__global__ __launch_bounds__(256) void k_exact_dist(const float *__restrict__ X, int64_t n, int d,
                                                    const float *__restrict__ Q, int64_t nq, int ql,
                                                    const int64_t *__restrict__ self, double *__restrict__ D,
                                                    int64_t ldD) {
    extern __shared__ float s_q[];  // [ql][dq], dq = d rounded up to 32, zero-padded; ql % 8 == 0
    const int dq = (d + 31) & ~31;
    const int64_t qb = (int64_t)blockIdx.y * ql;
    const int nql = (int)std::min<int64_t>(ql, nq - qb);
    for (int i = threadIdx.x; i < ql * dq; i += blockDim.x) {
        const int r = i / dq, c = i - r * dq;
        s_q[i] = (r < nql && c < d) ? Q[(qb + r) * d + c] : 0.f;
    }
    __syncthreads();
    const int g = threadIdx.x & 7;
    const int grp = threadIdx.x >> 3;  // 32 point slots per block
    const int nqg = (nql + 7) >> 3;
    for (int64_t j = (int64_t)blockIdx.x * 32 + grp; j < n; j += (int64_t)gridDim.x * 32) {
        const float *xr = X + j * d;
        float4 row[NR > 0 ? NR : 1];
        if (NR > 0) {
#pragma unroll
            for (int k = 0; k < NR; k++) {
                const int c = 4 * g + 32 * k;
                row[k] = c < d ? *reinterpret_cast<const float4 *>(xr + c) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
        for (int t = 0; t < nqg; t++) {
            double s[8][4];
#pragma unroll
            for (int r = 0; r < 8; r++) s[r][0] = s[r][1] = s[r][2] = s[r][3] = 0.0;
            // one column step: the canonical class of column c is c mod 32, held by lane
            // (c mod 32) / 4 in component c mod 4 -- as in every distance of the library
            auto step = [&](const float4 xv, int c) {
#pragma unroll
                for (int r = 0; r < 8; r++) {
                    const float4 qv = *reinterpret_cast<const float4 *>(&s_q[(t * 8 + r) * dq + c]);
                    const double e0 = (double)qv.x - (double)xv.x, e1 = (double)qv.y - (double)xv.y;
                    const double e2 = (double)qv.z - (double)xv.z, e3 = (double)qv.w - (double)xv.w;
                    s[r][0] = __builtin_fma(e0, e0, s[r][0]);
                    s[r][1] = __builtin_fma(e1, e1, s[r][1]);
                    s[r][2] = __builtin_fma(e2, e2, s[r][2]);
                    s[r][3] = __builtin_fma(e3, e3, s[r][3]);
                }
            };
            if (NR > 0) {
#pragma unroll
                for (int k = 0; k < NR; k++) step(row[k], 4 * g + 32 * k);
            } else {
                for (int c = 4 * g; c < d; c += 32) {
                    // columns past d hold 0 in the query row and are read as 0 here, so they
                    // add fma(0, 0, s) = s (s is never -0: it starts at +0 and adds squares)
                    float4 xv;
                    xv.x = xr[c];
                    xv.y = c + 1 < d ? xr[c + 1] : 0.f;
                    xv.z = c + 2 < d ? xr[c + 2] : 0.f;
                    xv.w = c + 3 < d ? xr[c + 3] : 0.f;
                    step(xv, c);
                }
            }
            double mine = 0.0;
#pragma unroll
            for (int r = 0; r < 8; r++) {
                double v = (s[r][0] + s[r][1]) + (s[r][2] + s[r][3]);
                v = v + shfl_xor_d(v, 1);
                v = v + shfl_xor_d(v, 2);
                v = v + shfl_xor_d(v, 4);
                if (r == g) mine = v;
            }
            const int qr = t * 8 + g;  // this lane writes query qr of the block
            if (qr < nql) {
                const int64_t q = qb + qr;
                if (self && self[q] == j) mine = __longlong_as_double((long long)kInfBits);
                D[q * ldD + j] = mine;
            }
        }
    }
}

// 96-bit key of an entry: (bits of D >= 0, point index); order = (D, index) order
__device__ inline unsigned __int128 ekey(uint64_t dbits, uint32_t j) { return ((unsigned __int128)dbits << 32) | j; }

// bitonic sort of s_k[0, m) (m a power of two <= 2 kSelThreads) ascending, by the whole block
__device__ inline void block_bitonic(uint64_t *s_hi, uint32_t *s_lo, int m) {
    for (int size = 2; size <= m; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < (m >> 1); i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const unsigned __int128 a = ekey(s_hi[lo], s_lo[lo]), b = ekey(s_hi[hi], s_lo[hi]);
                if ((a > b) == up) {
                    const uint64_t th = s_hi[lo];
                    const uint32_t tl = s_lo[lo];
                    s_hi[lo] = s_hi[hi];
                    s_lo[lo] = s_lo[hi];
                    s_hi[hi] = th;
                    s_lo[hi] = tl;
                }
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(kSelThreads) void k_exact_select(const double *__restrict__ D, int64_t n, int64_t ldD,
                                                             int K, int32_t *__restrict__ out_idx,
                                                             float *__restrict__ out_dist) {
    __shared__ uint32_t s_hist[kSelBins];
    __shared__ uint64_t s_ch[kSelCand];  // bucket entries (D bits, index), then the results
    __shared__ uint32_t s_cl[kSelCand];
    __shared__ uint64_t s_rh[256];       // entries below the bucket
    __shared__ uint32_t s_rl[256];
    __shared__ int s_state[4];
    const int64_t q = blockIdx.x;
    const uint64_t *row = reinterpret_cast<const uint64_t *>(D + q * ldD);
    const int tid = threadIdx.x;
    // the K-th smallest finite key: digits of 11 bits from the top of the 96-bit key (the
    // last digit 8 bits); after each histogram the prefix grows by the digit whose bucket
    // holds the rank
    unsigned __int128 prefix = 0;
    int nbits = 0;
    int need = K;       // entries still to take at or above the prefix
    int below = 0;      // entries known to lie below the prefix (all of them results)
    int bucket = 0;     // entries matching the prefix
    bool all = false;   // fewer finite entries than K: every finite entry is a result
    for (int lev = 0; lev < 9; lev++) {
        const int w = lev < 8 ? 11 : 8;
        const int shift = 96 - nbits - w;
        const unsigned __int128 mask = nbits ? (~(unsigned __int128)0) << (96 - nbits) : 0;
        for (int i = tid; i < kSelBins; i += kSelThreads) s_hist[i] = 0;
        __syncthreads();
        for (int64_t j = tid; j < n; j += kSelThreads) {
            const uint64_t b = row[j];
            if (b >= kInfBits) continue;
            const unsigned __int128 k = ekey(b, (uint32_t)j);
            if ((k & mask) == prefix) atomicAdd(&s_hist[(uint32_t)(k >> shift) & ((1u << w) - 1)], 1u);
        }
        __syncthreads();
        if (tid == 0) {  // the bucket of the rank (2048 bins, one thread: cheap next to the pass)
            uint32_t cum = 0;
            int b = -1;
            for (int i = 0; i < (1 << w); i++) {
                if (cum + s_hist[i] >= (uint32_t)need) {
                    b = i;
                    break;
                }
                cum += s_hist[i];
            }
            s_state[0] = b;
            s_state[1] = (int)cum;
            s_state[2] = b >= 0 ? (int)s_hist[b] : 0;
        }
        __syncthreads();
        const int b = s_state[0];
        if (b < 0) {  // fewer than `need` finite entries match: all of them are results
            all = true;
            break;
        }
        below += s_state[1];
        need -= s_state[1];
        bucket = s_state[2];
        prefix |= (unsigned __int128)b << shift;
        nbits += w;
        __syncthreads();
        if (bucket <= kSelCand) break;
    }
    // gather: entries below the prefix are results; entries matching it are sorted
    if (tid == 0) s_state[0] = s_state[1] = 0;
    __syncthreads();
    const unsigned __int128 mask = nbits ? (~(unsigned __int128)0) << (96 - nbits) : 0;
    for (int64_t j = tid; j < n; j += kSelThreads) {
        const uint64_t b = row[j];
        if (b >= kInfBits) continue;
        const unsigned __int128 k = ekey(b, (uint32_t)j) & mask;
        if (all || k < prefix) {
            const int at = atomicAdd(&s_state[0], 1);
            if (at < 256) {
                s_rh[at] = b;
                s_rl[at] = (uint32_t)j;
            }
        } else if (k == prefix) {
            const int at = atomicAdd(&s_state[1], 1);
            if (at < kSelCand) {
                s_ch[at] = b;
                s_cl[at] = (uint32_t)j;
            }
        }
    }
    __syncthreads();
    const int nr = min(s_state[0], 256), nc = all ? 0 : min(s_state[1], kSelCand);
    int m2 = 1;
    while (m2 < nc) m2 <<= 1;
    for (int i = nc + tid; i < m2; i += kSelThreads) {
        s_ch[i] = ~0ull;
        s_cl[i] = ~0u;
    }
    __syncthreads();
    if (nc > 1) block_bitonic(s_ch, s_cl, m2);
    // results: the nr entries below, then the first `need` of the bucket, sorted together
    const int take = all ? 0 : min(need, nc);
    const int tot = nr + take;
    __syncthreads();
    for (int i = tid; i < take; i += kSelThreads) {  // move the bucket's head behind the below-entries
        s_rh[nr + i] = s_ch[i];
        s_rl[nr + i] = s_cl[i];
    }
    __syncthreads();
    int m3 = 1;
    while (m3 < tot) m3 <<= 1;
    for (int i = tot + tid; i < m3; i += kSelThreads) {
        s_rh[i] = ~0ull;
        s_rl[i] = ~0u;
    }
    __syncthreads();
    if (tot > 1) block_bitonic(s_rh, s_rl, m3);
    for (int i = tid; i < K; i += kSelThreads) {
        if (i < tot) {
            out_idx[q * K + i] = (int32_t)s_rl[i];
            out_dist[q * K + i] = (float)sqrt(__longlong_as_double((long long)s_rh[i]));
        } else {
            out_idx[q * K + i] = -1;
            out_dist[q * K + i] = INFINITY;
        }
    }
    (void)below;
}

}  // namespace
}  // namespace rpf

using namespace rpf;

extern "C" rpf_status rpf_exact_knn(const float *X, int64_t n, int32_t d, const float *Q, int64_t m,
                                    const int64_t *self, int32_t K, int32_t *out_idx, float *out_dist, void *stream) {
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(RPF_EINVAL, "rpf_exact_knn: n must be in [1, 2^31)");
    if (d < 1 || d > 2048) return fail(RPF_EINVAL, "rpf_exact_knn: d must be in [1, 2048]");
    if (m < 0) return fail(RPF_EINVAL, "rpf_exact_knn: m must be >= 0");
    if (K < 1 || K > 256) return fail(RPF_EINVAL, "rpf_exact_knn: K must be in [1, 256]");
    if (m == 0) return RPF_OK;
    if (!X || !Q || !out_idx || !out_dist) return fail(RPF_EINVAL, "rpf_exact_knn: NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    {   // finite inputs only (one synchronisation)
        int32_t *flag = static_cast<int32_t *>(cache_alloc(16, s));
        if (!flag) return fail(RPF_ENOMEM, "rpf_exact_knn: allocation");
        fill_u32(flag, 4, 0, s);
        launch_nonfinite(s, X, n * d, flag);
        launch_nonfinite(s, Q, m * d, flag + 1);
        int32_t h[2] = {0, 0};
        hipMemcpyAsync(h, flag, 8, hipMemcpyDeviceToHost, s);
        cache_free(flag, s);
        const rpf_status st = check_hip(hipStreamSynchronize(s), "rpf_exact_knn input check");
        if (st != RPF_OK) return st;
        if (h[0] || h[1]) return fail(RPF_EINVAL, "rpf_exact_knn: X or Q holds NaN or Inf");
    }
    // queries of a distance block (a multiple of 8, LDS within 64 KiB), and per chunk: the
    // distance buffer stays within 4 GiB (at least one block of queries)
    const int dq = (d + 31) & ~31;
    const int ql = std::max(8, std::min(kQL, 16384 / dq / 8 * 8));
    const size_t lds = (size_t)ql * dq * 4;
    const int64_t chunk = std::max<int64_t>(ql, std::min<int64_t>(((int64_t)1 << 29) / n / ql * ql, m));
    double *Dbuf = static_cast<double *>(cache_alloc((size_t)std::min(chunk, m) * n * 8, s));
    if (!Dbuf) return fail(RPF_ENOMEM, "rpf_exact_knn: distance buffer allocation failed");
    const bool vec = (d % 4) == 0 && ((uintptr_t)X % 16) == 0;
    const int nr = vec && d <= 256 ? (d + 31) / 32 : 0;
    for (int64_t q0 = 0; q0 < m; q0 += chunk) {
        const int64_t nq = std::min(chunk, m - q0);
        const unsigned gy = (unsigned)((nq + ql - 1) / ql);
        const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 31) / 32, std::max<int64_t>(1, 16384 / gy)));
        {
            ProfScope ps(s, "exact_dist", (double)nq * n * 8 + (double)gy * n * d * 4, 2.0 * nq * n * d);
            const float *Qc = Q + q0 * d;
            const int64_t *sc = self ? self + q0 : nullptr;
            switch (nr) {
                case 1: hipLaunchKernelGGL(k_exact_dist<1>, dim3(gx, gy), dim3(256), lds, s, X, n, d, Qc, nq, ql, sc, Dbuf, n); break;
                case 2: hipLaunchKernelGGL(k_exact_dist<2>, dim3(gx, gy), dim3(256), lds, s, X, n, d, Qc, nq, ql, sc, Dbuf, n); break;
                case 3: hipLaunchKernelGGL(k_exact_dist<3>, dim3(gx, gy), dim3(256), lds, s, X, n, d, Qc, nq, ql, sc, Dbuf, n); break;
                case 4: hipLaunchKernelGGL(k_exact_dist<4>, dim3(gx, gy), dim3(256), lds, s, X, n, d, Qc, nq, ql, sc, Dbuf, n); break;
                case 5: hipLaunchKernelGGL(k_exact_dist<5>, dim3(gx, gy), dim3(256), lds, s, X, n, d, Qc, nq, ql, sc, Dbuf, n); break;
                case 6: hipLaunchKernelGGL(k_exact_dist<6>, dim3(gx, gy), dim3(256), lds, s, X, n, d, Qc, nq, ql, sc, Dbuf, n); break;
                case 7: hipLaunchKernelGGL(k_exact_dist<7>, dim3(gx, gy), dim3(256), lds, s, X, n, d, Qc, nq, ql, sc, Dbuf, n); break;
                case 8: hipLaunchKernelGGL(k_exact_dist<8>, dim3(gx, gy), dim3(256), lds, s, X, n, d, Qc, nq, ql, sc, Dbuf, n); break;
                default: hipLaunchKernelGGL(k_exact_dist<0>, dim3(gx, gy), dim3(256), lds, s, X, n, d, Qc, nq, ql, sc, Dbuf, n); break;
            }
            launch_check(s, "k_exact_dist");
        }
        {
            ProfScope ps(s, "exact_select", (double)nq * n * 8 * 3, 0);
            hipLaunchKernelGGL(k_exact_select, dim3((unsigned)nq), dim3(kSelThreads), 0, s, Dbuf, n, n, K,
                               out_idx + q0 * K, out_dist + q0 * K);
            launch_check(s, "k_exact_select");
        }
    }
    cache_free(Dbuf, s);
    const std::string le = take_launch_error();
    if (!le.empty()) return fail(RPF_EDEVICE, "rpf_exact_knn: " + le);
    return RPF_OK;
}
