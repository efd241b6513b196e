// Host-only replay of the first-phase merge's reads (Alg. 3, union of the first B trees'
// leaves).  For a problem shape it derives the merge geometry with the library's own
// functions (merge_index.h), enumerates every (row, lane, slot column) read the merge kernel
// makes over every leaf start of the closed-form tree shape, and checks each against the
// extents of the buffers it reads:
//   slot   in [a * cap1, a * cap1 + B * ML)  and  < rows * cap1  (the slot array)
//   leaf   lane index of the leaf-start read in [0, B)            (the [B][rows] array)
//   perm   in [0, T * n)                                          (the permutation)
// `--old` replays instead the arithmetic before slot columns past the row were masked (every
// lane read Q columns), as a negative control: it must fail where that fault was seen.
//
// usage: merge_index_replay n T n0 K rows [--old] [--B b]    prints "ok ..." or "FAIL ..." lines
// (--B: the first-phase tree count asked for, capped as the library caps it; default: the
// library's default)
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../paper_1812_11689_amd/csrc/merge_index.h"

using namespace rpf;

// leaves of the median-rule tree over n points (a node of m > n0 points splits into
// floor(m/2) and ceil(m/2)): their starts in the leaf-ordered permutation and sizes
static void leaves(int64_t off, int64_t m, int64_t n0, std::vector<int64_t> &start, std::vector<int64_t> &size) {
    if (m <= n0) {
        start.push_back(off);
        size.push_back(m);
        return;
    }
    leaves(off, m / 2, n0, start, size);
    leaves(off + m / 2, m - m / 2, n0, start, size);
}

int main(int argc, char **argv) {
    if (argc < 6) {
        fprintf(stderr, "usage: %s n T n0 K rows [--old]\n", argv[0]);
        return 2;
    }
    const int64_t n = atoll(argv[1]);
    const int T = atoi(argv[2]);
    const int64_t n0 = atoll(argv[3]);
    const int K = atoi(argv[4]);
    const int64_t rows = atoll(argv[5]);
    bool old = false;
    int want_b = 0;
    for (int i = 6; i < argc; i++) {
        if (strcmp(argv[i], "--old") == 0) old = true;
        if (strcmp(argv[i], "--B") == 0 && i + 1 < argc) want_b = atoi(argv[++i]);
    }
    std::vector<int64_t> start, size;
    leaves(0, n, n0, start, size);
    int max_leaf = 0;
    for (int64_t s : size) max_leaf = s > max_leaf ? (int)s : max_leaf;
    const int B = want_b > 0 ? imin_(want_b, max_first_trees_for(T, K, max_leaf)) : first_trees(T, K, max_leaf);
    const int ML = slot_stride(max_leaf);
    const int cap1 = ML * B;  // slots per row, as the workspace is sized
    const int Q = merge_first_q(cap1);
    const int c = B * ML;
    const int ncol = first_slot_cols(B, ML);
    printf("geometry n=%lld T=%d n0=%lld K=%d rows=%lld: leaves=%zu max_leaf=%d B=%d ML=%d cap1=%d Q=%d ncol=%d\n",
           (long long)n, T, (long long)n0, K, (long long)rows, start.size(), max_leaf, B, ML, cap1, Q, ncol);
    if (c > 64 * Q) {  // the kernel sends the row to the exhaustive path and reads nothing
        printf("ok (rows take the exhaustive path: %d slots > %d)\n", c, 64 * Q);
        return 0;
    }
    // rows whose slot reads are checked: every row of a small problem, else both ends and a
    // spread; the address depends on the row only through a * cap1
    std::vector<int64_t> rs;
    if (rows <= 4096) {
        for (int64_t a = 0; a < rows; a++) rs.push_back(a);
    } else {
        for (int64_t a = 0; a < 64; a++) rs.push_back(a);
        for (int64_t a = rows - 64; a < rows; a++) rs.push_back(a);
        for (int64_t k = 1; k < 1024; k++) rs.push_back(rows * k / 1024);
    }
    int64_t bad_slot = 0, bad_perm = 0, bad_lane = 0, reads = 0;
    for (int64_t a : rs) {
        FirstSlotCursor cur;
        for (int q = 0; q < Q; q++) {
            const bool in = old ? true : q < ncol;
            for (int lane = 0; lane < 64; lane++) {
                if (!in) continue;
                const int64_t addr = first_slot_addr(a, cap1, lane, q);
                reads++;
                if (addr < a * (int64_t)cap1 || addr >= a * (int64_t)cap1 + c || addr >= rows * (int64_t)cap1) {
                    if (bad_slot++ < 3)
                        printf("  slot read out of the row: row %lld lane %d col %d addr %lld (row range [%lld, %lld))\n",
                               (long long)a, lane, q, (long long)addr, (long long)(a * cap1), (long long)(a * cap1 + c));
                }
            }
            const int tl = in ? cur.tree : 0;  // lane whose leaf start the column reads
            if (tl < 0 || tl >= B) bad_lane++;
            first_slot_next(cur, ML);
        }
    }
    // permutation reads: every leaf start of the shape, every column in the row, every lane
    {
        FirstSlotCursor cur;
        for (int q = 0; q < Q; q++) {
            const bool in = old ? true : q < ncol;
            if (in) {
                for (size_t l = 0; l < start.size(); l++)
                    for (int lane = 0; lane < 64; lane++) {
                        const int32_t pos = first_slot_perm_pos((int32_t)start[l], cur.col0, lane, n);
                        const int64_t at = (int64_t)cur.tree * n + pos;
                        reads++;
                        if (pos < 0 || pos >= n || at < 0 || at >= (int64_t)T * n) {
                            if (bad_perm++ < 3)
                                printf("  permutation read out of range: tree %d leaf start %lld col0 %d lane %d -> %lld\n",
                                       cur.tree, (long long)start[l], cur.col0, lane, (long long)at);
                        }
                    }
            }
            first_slot_next(cur, ML);
        }
    }
    if (bad_slot || bad_perm || bad_lane) {
        printf("FAIL %lld slot reads, %lld permutation reads, %lld leaf-start lanes out of range (of %lld reads)\n",
               (long long)bad_slot, (long long)bad_perm, (long long)bad_lane, (long long)reads);
        return 1;
    }
    printf("ok %lld reads in range\n", (long long)reads);
    return 0;
}
