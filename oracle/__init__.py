"""CPU oracle for rpForests kNN search -- TEST INFRASTRUCTURE ONLY.

`rpf_oracle.c` is a plain C implementation of the paper's Algorithms 1-3 (median split
point of Sec. 2, and the uniform split point of Alg. 1 with a counter-based generator) plus
brute-force kNN; `mini.py` is an independent pure-Python/numpy twin
for tiny inputs.  Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this package.  It shares no code with the HIP library and never imports it.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rpf_oracle.c")
_LIB = os.path.join(_HERE, "librpf_oracle.so")
_lib = None

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (binary64, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        vp = ctypes.c_void_p
        lib.rpfo_canon_sum.restype = dbl
        lib.rpfo_canon_sum.argtypes = [vp, i64]
        lib.rpfo_canon_dot64.restype = dbl
        lib.rpfo_canon_dot64.argtypes = [vp, vp, i32]
        lib.rpfo_canon_dist64.restype = dbl
        lib.rpfo_canon_dist64.argtypes = [vp, vp, i32]
        lib.rpfo_depth.restype = i32
        lib.rpfo_depth.argtypes = [i64, i64]
        lib.rpfo_node_range.restype = i64
        lib.rpfo_node_range.argtypes = [i64, i64, i64, vp]
        lib.rpfo_build.restype = i32
        lib.rpfo_build.argtypes = [vp, i64, i32, vp, i32, i32, i64, vp, vp, vp, vp, vp]
        lib.rpfo_route.restype = None
        lib.rpfo_route.argtypes = [vp, i32, i32, i32, i64, i64, vp, vp, vp, i64, vp]
        lib.rpfo_knn.restype = None
        lib.rpfo_knn.argtypes = [vp, i64, i32, i32, i64, vp, vp, i64, vp, vp, i32, vp, vp]
        lib.rpfo_bruteforce.restype = None
        lib.rpfo_bruteforce.argtypes = [vp, i64, i32, vp, i64, vp, i32, vp, vp]
        u64 = ctypes.c_uint64
        lib.rpfo_mix64.restype = u64
        lib.rpfo_mix64.argtypes = [u64]
        lib.rpfo_stream.restype = u64
        lib.rpfo_stream.argtypes = [u64, u64]
        lib.rpfo_node_key.restype = u64
        lib.rpfo_node_key.argtypes = [u64, i32, i64]
        lib.rpfo_node_u.restype = dbl
        lib.rpfo_node_u.argtypes = [u64]
        lib.rpfo_node_direction.restype = None
        lib.rpfo_node_direction.argtypes = [u64, i32, i32, vp]
        lib.rpfo_build_uniform.restype = None
        lib.rpfo_build_uniform.argtypes = [vp, i64, i32, i32, i32, i64, u64, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.rpfo_knn_ordinal.restype = None
        lib.rpfo_knn_ordinal.argtypes = [vp, i64, i32, i32, vp, vp, vp, i64, vp, vp, i32, vp, vp]
        lib.rpfo_threads.restype = i32
        lib.rpfo_threads.argtypes = []
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def threads() -> int:
    return _load().rpfo_threads()


def canon_sum(v) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return _load().rpfo_canon_sum(_p(v), v.size)


def canon_dot64(x, r) -> float:
    x, r = _f32(x), _f32(r)
    return _load().rpfo_canon_dot64(_p(x), _p(r), x.size)


def canon_dist64(a, b) -> float:
    a, b = _f32(a), _f32(b)
    return _load().rpfo_canon_dist64(_p(a), _p(b), a.size)


def depth(n: int, n0: int) -> int:
    return _load().rpfo_depth(n, n0)


def node_range(n: int, n0: int, h: int):
    off = ctypes.c_int64(0)
    m = _load().rpfo_node_range(n, n0, h, ctypes.byref(off))
    return (off.value, m) if m >= 0 else None


class Forest:
    """Output of the oracle build: per tree split value, split index, chosen try, leaf
    order (perm) and leaf heap id of every point."""

    def __init__(self, x, R, n_trees, n_try, n0, split, split_idx, chosen, perm, leaf_of, L):
        self.x, self.R = x, R
        self.n_trees, self.n_try, self.n0, self.L = n_trees, n_try, n0, L
        self.split, self.split_idx, self.chosen = split, split_idx, chosen
        self.perm, self.leaf_of = perm, leaf_of

    @property
    def n(self):
        return self.x.shape[0]

    @property
    def d(self):
        return self.x.shape[1]


def build_forest(x, R, n_trees: int, n0: int, n_try: int = 1) -> Forest:
    """Alg. 3 (forest growth) with Alg. 1/2: grow `n_trees` trees over x with directions R
    [T][2^L-1][n_try][d] (R may hold more trees; the first n_trees are used)."""
    x = _f32(x)
    n, d = x.shape
    L = depth(n, n0)
    H = (1 << L) - 1
    R = _f32(R)
    assert R.shape[1:] == (H, n_try, d) and R.shape[0] >= n_trees, (R.shape, H, n_try, d)
    R = np.ascontiguousarray(R[:n_trees])
    split = np.empty((n_trees, H), np.float64)
    split_idx = np.empty((n_trees, H), np.int32)
    chosen = np.empty((n_trees, H), np.int32)
    perm = np.empty((n_trees, n), np.int32)
    leaf_of = np.empty((n_trees, n), np.int32)
    got = _load().rpfo_build(_p(x), n, d, _p(R), n_trees, n_try, n0, _p(split), _p(split_idx),
                             _p(chosen), _p(perm), _p(leaf_of))
    assert got == L
    return Forest(x, R, n_trees, n_try, n0, split, split_idx, chosen, perm, leaf_of, L)


def route(f: Forest, q, n_trees: int | None = None) -> np.ndarray:
    """Leaf heap id of each query in each tree, int32 [T][m]."""
    T = f.n_trees if n_trees is None else n_trees
    q = _f32(q)
    m = q.shape[0]
    out = np.empty((T, m), np.int32)
    R = np.ascontiguousarray(f.R[:T])
    H = R.shape[1]
    chosen = np.ascontiguousarray(f.chosen[:T])
    split = np.ascontiguousarray(f.split[:T])
    assert H == (1 << f.L) - 1
    _load().rpfo_route(_p(R), T, f.n_try, f.d, f.n, f.n0, _p(chosen), _p(split), _p(q), m,
                       _p(out))
    return out


def knn_from_leaves(f: Forest, q, qleaf, K: int, self_idx=None, n_trees: int | None = None):
    """K nearest in the union of the leaves qleaf[t][:] over the first n_trees trees."""
    T = f.n_trees if n_trees is None else n_trees
    q = _f32(q)
    m = q.shape[0]
    qleaf = np.ascontiguousarray(qleaf[:T], dtype=np.int32)
    perm = np.ascontiguousarray(f.perm[:T])
    out_idx = np.empty((m, K), np.int32)
    out_dist = np.empty((m, K), np.float64)
    self_arr = None if self_idx is None else np.ascontiguousarray(self_idx, dtype=np.int64)
    _load().rpfo_knn(_p(f.x), f.n, f.d, T, f.n0, _p(perm), _p(q), m, _p(qleaf),
                     None if self_arr is None else _p(self_arr), K, _p(out_idx), _p(out_dist))
    return out_idx, out_dist


def all_knn(f: Forest, K: int, points=None, exclude_self: bool = True,
            n_trees: int | None = None):
    """Q = U (Alg. 3 with Q the data set): every point's leaves are its own leaves."""
    T = f.n_trees if n_trees is None else n_trees
    pts = np.arange(f.n) if points is None else np.asarray(points, dtype=np.int64)
    qleaf = f.leaf_of[:T][:, pts]
    return knn_from_leaves(f, f.x[pts], qleaf, K, pts if exclude_self else None, T)


def query_knn(f: Forest, q, K: int, n_trees: int | None = None):
    """External queries: route each through every tree, then kNN over the leaf union."""
    qleaf = route(f, q, n_trees)
    return knn_from_leaves(f, q, qleaf, K, None, n_trees)


# ---- uniform split rule (Alg. 1 as printed: c ~ runif[a, b]) -----------------------------

def mix64(z: int) -> int:
    """SplitMix64's finaliser (Steele, Lea and Flood 2014)."""
    return _load().rpfo_mix64(z & (2**64 - 1))


def stream(seed: int, i: int) -> int:
    """Output i of the SplitMix64 stream with the given seed: mix64(seed + (i + 1) GAMMA)."""
    return _load().rpfo_stream(seed & (2**64 - 1), i & (2**64 - 1))


def node_key(seed: int, t: int, h: int) -> int:
    """Seed of the stream of node h (heap id) of tree t: stream(stream(seed, t), h)."""
    return _load().rpfo_node_key(seed & (2**64 - 1), t, h)


def node_u(key: int) -> float:
    """The node's split fraction u in [0, 1)."""
    return _load().rpfo_node_u(key)


def node_direction(key: int, try_i: int, d: int) -> np.ndarray:
    """Direction `try_i` of the node whose stream seed is `key` (binary32 [d])."""
    r = np.empty(d, np.float32)
    _load().rpfo_node_direction(key, try_i, d, _p(r))
    return r


class UniformForest:
    """Output of the oracle's uniform-rule build: per tree the leaf order (perm), the leaf
    ordinal of every point (leaf_of), the leaf count and depth, and optionally the list of
    nodes where a split was attempted (heap id, (a, b, c), (size, left size, try, depth))."""

    def __init__(self, x, n_trees, n_try, n0, seed, perm, leaf_of, nleaf, max_depth, nodes):
        self.x, self.n_trees, self.n_try, self.n0, self.seed = x, n_trees, n_try, n0, seed
        self.perm, self.leaf_of, self.nleaf, self.max_depth, self.nodes = perm, leaf_of, nleaf, max_depth, nodes

    @property
    def n(self):
        return self.x.shape[0]

    @property
    def d(self):
        return self.x.shape[1]


def build_uniform(x, n_trees: int, n0: int, seed: int, n_try: int = 1, nodes: bool = False) -> UniformForest:
    """Alg. 3 forest growth with Alg. 1's uniform split point and Alg. 2's direction choice;
    the random numbers come from the counter-based generator keyed by (seed, tree, node)."""
    x = _f32(x)
    n, d = x.shape
    perm = np.empty((n_trees, n), np.int32)
    leaf_of = np.empty((n_trees, n), np.int32)
    nleaf = np.empty(n_trees, np.int32)
    max_depth = np.empty(n_trees, np.int32)
    nn = np.zeros(n_trees, np.int64)
    heap = abc = info = None
    if nodes:
        heap = np.zeros((n_trees, n), np.int64)
        abc = np.zeros((n_trees, n, 3), np.float64)
        info = np.zeros((n_trees, n, 4), np.int32)
    _load().rpfo_build_uniform(_p(x), n, d, n_trees, n_try, n0, seed & (2**64 - 1), _p(perm), _p(leaf_of),
                               _p(nleaf), _p(max_depth), _p(nn), None if heap is None else _p(heap),
                               None if abc is None else _p(abc), None if info is None else _p(info))
    node_lists = None
    if nodes:
        node_lists = [dict(heap=heap[t, :nn[t]], a=abc[t, :nn[t], 0], b=abc[t, :nn[t], 1], c=abc[t, :nn[t], 2],
                           size=info[t, :nn[t], 0], left=info[t, :nn[t], 1], chosen=info[t, :nn[t], 2],
                           depth=info[t, :nn[t], 3]) for t in range(n_trees)]
    return UniformForest(x, n_trees, n_try, n0, seed, perm, leaf_of, nleaf, max_depth, node_lists)


def knn_ordinal(x, perm, leaf_of, q, qleaf, K: int, self_idx=None):
    """K nearest in the union of leaves given by ordinals (qleaf [T][m]) of trees whose
    leaf order is perm [T][n] and leaf ordinals leaf_of [T][n]."""
    x, q = _f32(x), _f32(q)
    n, d = x.shape
    m = q.shape[0]
    T = perm.shape[0]
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    leaf_of = np.ascontiguousarray(leaf_of, dtype=np.int32)
    qleaf = np.ascontiguousarray(qleaf, dtype=np.int32)
    out_idx = np.empty((m, K), np.int32)
    out_dist = np.empty((m, K), np.float64)
    self_arr = None if self_idx is None else np.ascontiguousarray(self_idx, dtype=np.int64)
    _load().rpfo_knn_ordinal(_p(x), n, d, T, _p(perm), _p(leaf_of), _p(q), m, _p(qleaf),
                             None if self_arr is None else _p(self_arr), K, _p(out_idx), _p(out_dist))
    return out_idx, out_dist


def all_knn_uniform(f: UniformForest, K: int, points=None, exclude_self: bool = True, n_trees: int | None = None):
    """Q = U over a uniform-rule forest: every point's leaves are its own leaves."""
    T = f.n_trees if n_trees is None else n_trees
    pts = np.arange(f.n) if points is None else np.asarray(points, dtype=np.int64)
    return knn_ordinal(f.x, f.perm[:T], f.leaf_of[:T], f.x[pts], f.leaf_of[:T][:, pts], K,
                       pts if exclude_self else None)


def bruteforce(x, q, K: int, self_idx=None):
    """Exact K nearest neighbours of each query over all of x, ordered by (D, index)."""
    x, q = _f32(x), _f32(q)
    n, d = x.shape
    m = q.shape[0]
    out_idx = np.empty((m, K), np.int32)
    out_dist = np.empty((m, K), np.float64)
    self_arr = None if self_idx is None else np.ascontiguousarray(self_idx, dtype=np.int64)
    _load().rpfo_bruteforce(_p(x), n, d, _p(q), m, None if self_arr is None else _p(self_arr),
                            K, _p(out_idx), _p(out_dist))
    return out_idx, out_dist


def missing_rate(found_idx, true_idx) -> float:
    """Average missing rate m_k = (1/(nK)) sum_i |TrueK(i) minus Found(i)| (Sec. 5.1)."""
    found_idx = np.asarray(found_idx)
    true_idx = np.asarray(true_idx)
    miss = 0
    for f, t in zip(found_idx, true_idx):
        miss += len(set(t.tolist()) - set(f.tolist()))
    return miss / true_idx.size


def missing_counts(found_idx, true_idx) -> np.ndarray:
    return np.array([len(set(t.tolist()) - set(f.tolist())) for f, t in zip(found_idx, true_idx)])
