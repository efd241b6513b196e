"""Pure-Python twin of the C oracle, for tiny inputs -- TEST INFRASTRUCTURE ONLY.

Written separately from `rpf_oracle.c` (recursive rather than work-list driven, Python
floats rather than C doubles, exact integer arithmetic for fused multiply-add) so that the
two can pin each other bit for bit on small problems.  It follows the same canonical
reading of the paper (Sec. 2 projections, Alg. 1 median split on the key (p, index),
Alg. 2 direction choice by the largest S2, Alg. 3 union of leaves and exact distances; the
uniform split point of Alg. 1 with the SplitMix64 generator keyed by (seed, tree, node)):

  canon_sum: +0.0-padding to a power of two, then adjacent pairs summed level by level;
  projection: 32 partial sums by j mod 32 of exact binary64 products, canon_sum, + 0.0;
  distance: 32 partial sums of fma(delta, delta, s) with delta = a_j - b_j in binary64.
"""

from __future__ import annotations

import numpy as np

NCLASS = 32


def canon_sum(v) -> float:
    vals = [float(a) for a in v]
    if not vals:
        return 0.0
    p = 1
    while p < len(vals):
        p *= 2
    vals += [0.0] * (p - len(vals))
    while len(vals) > 1:
        vals = [vals[i] + vals[i + 1] for i in range(0, len(vals), 2)]
    return vals[0]


def fma(a: float, b: float, c: float) -> float:
    """a*b + c with one rounding, via exact integer arithmetic (denominators are powers of
    two) and CPython's correctly rounded int/int division."""
    na, da = float(a).as_integer_ratio()
    nb, db = float(b).as_integer_ratio()
    nc, dc = float(c).as_integer_ratio()
    n1, d1 = na * nb, da * db
    if d1 >= dc:
        num, den = n1 + nc * (d1 // dc), d1
    else:
        num, den = n1 * (dc // d1) + nc, dc
    return num / den


def canon_dot64(x, r) -> float:
    xs = [float(v) for v in np.asarray(x, dtype=np.float32)]
    rs = [float(v) for v in np.asarray(r, dtype=np.float32)]
    s = [0.0] * NCLASS
    for j, (a, b) in enumerate(zip(xs, rs)):
        s[j % NCLASS] = s[j % NCLASS] + a * b  # a*b is exact: 24+24 significant bits
    return canon_sum(s) + 0.0


def canon_dist64(a, b) -> float:
    aa = [float(v) for v in np.asarray(a, dtype=np.float32)]
    bb = [float(v) for v in np.asarray(b, dtype=np.float32)]
    s = [0.0] * NCLASS
    for j, (u, v) in enumerate(zip(aa, bb)):
        delta = u - v
        s[j % NCLASS] = fma(delta, delta, s[j % NCLASS])
    return canon_sum(s)


def depth(n: int, n0: int) -> int:
    L = 0
    while -(-n // (1 << L)) > n0:
        L += 1
    return L


def _which_projection(x, members, Rnode, n_try):
    if n_try == 1:
        return 0
    best, best_try = 0.0, None
    for k in range(n_try):
        p = [canon_dot64(x[i], Rnode[k]) for i in members]
        mu = canon_sum(p) / len(p)
        s2 = canon_sum([(v - mu) * (v - mu) for v in p])
        if s2 > best:
            best, best_try = s2, k
    return 0 if best_try is None else best_try


def build_tree(x, Rt, n0: int, n_try: int = 1):
    """One tree (Alg. 1, median split).  Returns dict(split, split_idx, chosen, perm,
    leaf_of) with the same conventions as the C oracle."""
    x = np.asarray(x, dtype=np.float32)
    n = x.shape[0]
    L = depth(n, n0)
    H = (1 << L) - 1
    split = np.full(H, np.nan)
    split_idx = np.full(H, -1, np.int32)
    chosen = np.full(H, -1, np.int32)
    leaf_of = np.zeros(n, np.int32)

    def grow(members, h):
        if len(members) <= n0:
            for i in members:
                leaf_of[i] = h
            return list(members)
        ch = _which_projection(x, members, Rt[h - 1], n_try)
        keys = sorted((canon_dot64(x[i], Rt[h - 1][ch]), i) for i in members)
        c = keys[len(members) // 2]
        split[h - 1], split_idx[h - 1], chosen[h - 1] = c[0], c[1], ch
        left = [i for i in members if (canon_dot64(x[i], Rt[h - 1][ch]), i) < c]
        right = [i for i in members if (canon_dot64(x[i], Rt[h - 1][ch]), i) >= c]
        return grow(left, 2 * h) + grow(right, 2 * h + 1)

    perm = np.asarray(grow(list(range(n)), 1), dtype=np.int32)
    return dict(split=split, split_idx=split_idx, chosen=chosen, perm=perm, leaf_of=leaf_of, L=L)


def build_forest(x, R, n_trees: int, n0: int, n_try: int = 1):
    return [build_tree(x, R[t], n0, n_try) for t in range(n_trees)]


def route_one(q, tree, Rt, n: int, n0: int) -> int:
    h, size = 1, n
    while size > n0:
        p = canon_dot64(q, Rt[h - 1][tree["chosen"][h - 1]])
        right = p >= tree["split"][h - 1]
        size = size - size // 2 if right else size // 2
        h = 2 * h + int(right)
    return h


def knn_union(x, trees, leaves_of_query, q, K: int, self_idx=None):
    """K closest members of the union of the given leaves (one heap id per tree)."""
    cand = set()
    for tree, h in zip(trees, leaves_of_query):
        cand.update(np.nonzero(tree["leaf_of"] == h)[0].tolist())
    if self_idx is not None:
        cand.discard(int(self_idx))
    ranked = sorted((canon_dist64(q, x[j]), j) for j in cand)[:K]
    idx = [j for _, j in ranked] + [-1] * (K - len(ranked))
    dist = [float(np.sqrt(D)) for D, _ in ranked] + [np.inf] * (K - len(ranked))
    return np.asarray(idx, np.int32), np.asarray(dist)


def all_knn(x, trees, K: int, exclude_self: bool = True):
    x = np.asarray(x, dtype=np.float32)
    n = x.shape[0]
    idx = np.empty((n, K), np.int32)
    dist = np.empty((n, K))
    for i in range(n):
        idx[i], dist[i] = knn_union(x, trees, [t["leaf_of"][i] for t in trees], x[i], K,
                                    i if exclude_self else None)
    return idx, dist


# ---- uniform split rule (Alg. 1 as printed: c uniform in [a, b]) --------------------------
# SplitMix64 (Steele, Lea and Flood 2014) in Python integers: output i of the stream with
# seed s is mix64(s + (i + 1) * GAMMA) mod 2^64.

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
UNIFORM_DEPTH = 62


def mix64(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def stream(seed: int, i: int) -> int:
    return mix64(seed + (i + 1) * GAMMA)


def node_key(seed: int, t: int, h: int) -> int:
    return stream(stream(seed, t), h)


def node_u(key: int) -> float:
    return (stream(key, 0) >> 11) * 2.0 ** -53


def node_direction(key: int, try_i: int, d: int) -> np.ndarray:
    out = []
    for j in range(d):
        total = 0
        for q in range(6):
            w = stream(key, 1 + 6 * (try_i * d + j) + q)
            total += (w >> 32) + (w & 0xFFFFFFFF)
        out.append(total * 2.0 ** -32 - 6.0)  # exact: fewer than 53 significant bits
    return np.asarray(out, dtype=np.float64).astype(np.float32)


def build_tree_uniform(x, seed: int, t: int, n0: int, n_try: int = 1):
    """Tree t by the uniform rule, recursively.  Returns dict(perm, leaf_of (ordinals),
    nleaf, max_depth, nodes) with the C oracle's conventions; nodes lists (heap, a, b, c,
    size, left size, try, depth) of every node where a split was attempted, in the order
    the recursion visits them (pre-order, left first)."""
    x = np.asarray(x, dtype=np.float32)
    n, d = x.shape
    leaf_of = np.zeros(n, np.int32)
    nodes = []
    state = {"nleaf": 0, "depth": 0}

    def leaf(members, depth):
        for i in members:
            leaf_of[i] = state["nleaf"]
        state["nleaf"] += 1
        state["depth"] = max(state["depth"], depth)
        return list(members)

    def grow(members, h, depth):
        if len(members) <= n0 or depth >= UNIFORM_DEPTH:
            return leaf(members, depth)
        key = node_key(seed, t, h)
        R = [node_direction(key, i, d) for i in range(n_try)]
        ch = _which_projection(x, members, R, n_try)
        p = [canon_dot64(x[i], R[ch]) for i in members]
        a, b = min(p), max(p)
        c = a + node_u(key) * (b - a)
        left = [i for i, v in zip(members, p) if v < c]
        right = [i for i, v in zip(members, p) if v >= c]
        nodes.append((h, a, b, c, len(members), len(left), ch, depth))
        if not left or not right:
            return leaf(members, depth)
        return grow(left, 2 * h, depth + 1) + grow(right, 2 * h + 1, depth + 1)

    perm = np.asarray(grow(list(range(n)), 1, 0), dtype=np.int32)
    return dict(perm=perm, leaf_of=leaf_of, nleaf=state["nleaf"], max_depth=state["depth"], nodes=nodes)


def build_forest_uniform(x, n_trees: int, n0: int, seed: int, n_try: int = 1):
    return [build_tree_uniform(x, seed, t, n0, n_try) for t in range(n_trees)]
