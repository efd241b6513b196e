// Geometry and index arithmetic of the first-phase merge (the union of a row's leaves in the
// first B trees, Alg. 3), kept free of HIP so that a host-only build can replay every read the
// merge kernel makes for a given problem shape and check it against the buffers' extents.
//
// Layout of the first-phase slots: row a owns slots [a * cap1, a * cap1 + B * ML), where
// ML = the largest leaf rounded up to a wave (64) and cap1 = B * ML.  Slot (a, t, j) holds the
// packed bounds of the pair (row a, member j of the row's leaf in tree t), j < ML; slots past
// the leaf's size hold the empty pattern.  The member's point index is read from the tree's
// leaf-ordered permutation at the leaf's start + j, clamped into [0, n).
#pragma once

#include <stdint.h>

#ifdef __HIPCC__
#define RPF_HD __host__ __device__
#else
#define RPF_HD
#endif

namespace rpf {

constexpr int kFirstTrees = 4;   // default first-phase trees (their leaves are kept whole)
constexpr int kMergeCap = 2048;  // first-phase slots per row one merge wave holds
constexpr int kSetCap = 512;     // bounds the small set of the merge: K * B <= kSetCap - 64

RPF_HD inline int imin_(int a, int b) { return a < b ? a : b; }
RPF_HD inline int imax_(int a, int b) { return a > b ? a : b; }

// first-phase slots per (row, tree): the largest leaf rounded up to a wave, so that the
// slots of a row's wave-wide column q all belong to one tree
RPF_HD inline int slot_stride(int max_leaf) { return (imax_(max_leaf, 1) + 63) & ~63; }

// largest first-phase tree count the merge supports: K * B leaves room in the small set and
// the row's B * ML slots fit one wave's registers
RPF_HD inline int max_first_trees_for(int T, int K, int max_leaf) {
    return imax_(1, imin_(imin_(T, (kSetCap - 64) / K), kMergeCap / slot_stride(max_leaf)));
}

RPF_HD inline int first_trees(int T, int K, int max_leaf) {
    return imin_(kFirstTrees, max_first_trees_for(T, K, max_leaf));
}

// slots per lane of the merge instantiation that holds cap1 = B * ML slots (4, 8, 16 or 32)
RPF_HD inline int merge_first_q(int cap1) {
    return cap1 <= 256 ? 4 : cap1 <= 512 ? 8 : cap1 <= 1024 ? 16 : kMergeCap / 64;
}

// The read of slot column q by one lane (the kernel walks q = 0, 1, ... with the cursor).
struct FirstSlotCursor {
    int tree = 0;  // tree of column q
    int col0 = 0;  // position in the leaf of the column's first slot
};

RPF_HD inline void first_slot_next(FirstSlotCursor &c, int ML) {
    c.col0 += 64;
    if (c.col0 == ML) {
        c.col0 = 0;
        c.tree++;
    }
}

// wave-wide slot columns of a row; a column past them is not read
RPF_HD inline int first_slot_cols(int B, int ML) { return B * (ML >> 6); }

// address of the lane's slot in column q of row a (valid only when q < first_slot_cols)
RPF_HD inline int64_t first_slot_addr(int64_t a, int cap1, int lane, int q) {
    return a * (int64_t)cap1 + lane + 64 * (int64_t)q;
}

// position in the tree's permutation of the member a slot names: leaf start + column
// position + lane, clamped into [0, n) (a slot past the leaf's size is dropped by its
// bounds, and its clamped index read is never used)
RPF_HD inline int32_t first_slot_perm_pos(int32_t leaf_start, int col0, int lane, int64_t n) {
    const int64_t p = (int64_t)leaf_start + col0 + lane;
    return (int32_t)(p < 0 ? 0 : p < n - 1 ? p : n - 1);
}

}  // namespace rpf
