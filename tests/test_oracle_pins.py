"""Pins for the CPU oracle: each test checks it against something other than itself --
hand-worked values, closed forms, special cases that reduce to textbook routines (brute
force, the median kd-tree), exact rational arithmetic, invariants of the method and an
independent pure-Python twin.  CPU only."""

import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import mini
from paper_1812_11689_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _heap_count(n, n0):
    return (1 << oracle.depth(n, n0)) - 1


def _forest(x, T, n0, n_try=1, seed=3):
    n, d = x.shape
    R = W.directions(seed, T, _heap_count(n, n0), n_try, d)
    return oracle.build_forest(x, R, T, n0, n_try), R


# ---------------------------------------------------------------- canonical arithmetic


def _golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln for ln in fh.read().splitlines() if ln.strip() and not ln.startswith("#")]


def test_canonical_arithmetic_hand_values():
    rows = [[c.strip() for c in ln.split("|")] for ln in _golden_lines("canonical_arithmetic.txt")]
    assert len(rows) >= 8
    for kind, inputs, expected, _why in rows:
        exp = float(expected)
        if kind == "sum":
            v = [float(t) for t in inputs.split()]
            assert oracle.canon_sum(v) == exp, inputs
            assert mini.canon_sum(v) == exp, inputs
        elif kind == "dot":
            head, _ = inputs.split(",")
            toks = head.replace(":", " ").split()
            d = int(toks[0].split("=")[1])
            x = np.zeros(d, np.float32)
            for tok in toks[1:]:
                k, v = tok.split("=")
                x[int(k[1:])] = float(v)
            r = np.ones(d, np.float32)
            assert oracle.canon_dot64(x, r) == exp, inputs
            assert mini.canon_dot64(x, r) == exp, inputs
        elif kind == "dist":
            a = np.zeros(2, np.float32)
            b = np.zeros(2, np.float32)
            a[0], b[1] = 3, 4
            assert oracle.canon_dist64(a, b) == exp
            assert mini.canon_dist64(a, b) == exp


@pytest.mark.parametrize("d", [1, 3, 7, 31, 32, 33, 64, 100, 257])
def test_projection_exact_on_integers(d):
    # small integers: every partial sum is exact, so the canonical value is the exact dot
    rng = np.random.default_rng(d)
    x = rng.integers(-1000, 1000, d).astype(np.float32)
    r = rng.integers(-1000, 1000, d).astype(np.float32)
    exact = sum(int(a) * int(b) for a, b in zip(x, r))
    assert oracle.canon_dot64(x, r) == float(exact)
    assert oracle.canon_dist64(x, r) == float(sum((int(a) - int(b)) ** 2 for a, b in zip(x, r)))


@pytest.mark.parametrize("d", [1, 5, 16, 33, 128, 784])
def test_projection_within_rounding_bound(d):
    # binary32 products are exact in binary64; the canonical sum differs from the exactly
    # rounded dot product by at most gamma_{ceil(d/32)+5} * sum |x_j r_j|
    rng = np.random.default_rng(100 + d)
    for _ in range(20):
        x = (rng.standard_normal(d) * np.exp(rng.uniform(-20, 20, d))).astype(np.float32)
        r = rng.standard_normal(d).astype(np.float32)
        prods = [Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, r)]
        exact = sum(prods, Fraction(0))
        absum = float(sum((abs(p) for p in prods), Fraction(0)))
        k = math.ceil(d / 32) + 5
        u = 2.0 ** -53
        bound = k * u / (1 - k * u) * absum
        got = oracle.canon_dot64(x, r)
        assert abs(Fraction(got) - exact) <= Fraction(bound) * (1 + 1e-9)
        assert got == mini.canon_dot64(x, r)


def test_projection_sign_of_zero_and_symmetry():
    x = np.array([-1.0, 2.0], np.float32)
    r = np.array([0.0, 0.0], np.float32)
    p = oracle.canon_dot64(x, r)
    assert p == 0.0 and math.copysign(1.0, p) == 1.0
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal((2, 77)).astype(np.float32)
    assert oracle.canon_dist64(a, b) == oracle.canon_dist64(b, a)
    assert oracle.canon_dist64(a, a) == 0.0


def test_fma_twin_is_exact():
    # the twin's fused multiply-add against exact rationals
    rng = np.random.default_rng(9)
    for _ in range(200):
        a, c = rng.standard_normal(2) * np.exp(rng.uniform(-30, 30, 2))
        exact = Fraction(float(a)) * Fraction(float(a)) + Fraction(float(c))
        got = mini.fma(float(a), float(a), float(c))
        lo, hi = np.nextafter(got, -np.inf), np.nextafter(got, np.inf)
        assert abs(Fraction(got) - exact) <= abs(Fraction(float(hi)) - Fraction(float(lo))) / 4


# ---------------------------------------------------------------- tree shape (median rule)


@pytest.mark.parametrize("n,n0", [(1, 1), (5, 5), (6, 5), (7, 3), (100, 10), (1000, 50),
                                  (1023, 64), (1025, 64), (4096, 256), (10000, 50)])
def test_shape_closed_form(n, n0):
    x = W.gaussian_mixture(n + n0, n, 4, 3)
    f, _ = _forest(x, 2, n0)
    L = oracle.depth(n, n0)
    assert L == (0 if n <= n0 else math.ceil(math.log2(n / n0)))
    for t in range(2):
        assert np.array_equal(np.sort(f.perm[t]), np.arange(n))  # leaves partition U
        heaps, sizes = np.unique(f.leaf_of[t], return_counts=True)
        assert sizes.sum() == n
        for h, m in zip(heaps, sizes):
            dep = int(h).bit_length() - 1
            assert dep in (L - 1, L) or (L == 0 and dep == 0)
            assert m <= n0
            assert m in (n // (1 << dep), -(-n // (1 << dep)))
            off, m2 = oracle.node_range(n, n0, int(h))
            assert m2 == m
            assert np.all(f.leaf_of[t][f.perm[t][off:off + m]] == h)
            # members of a leaf are listed in ascending original index
            assert np.all(np.diff(f.perm[t][off:off + m]) > 0)


def test_split_orders_children():
    n, n0 = 700, 20
    x = W.gaussian_mixture(4, n, 9, 4)
    f, R = _forest(x, 3, n0)
    for t in range(3):
        for h in range(1, (1 << f.L)):
            rng_ = oracle.node_range(n, n0, h)
            if rng_ is None or rng_[1] <= n0:
                continue
            off, m = rng_
            members = np.sort(f.perm[t][off:off + m])
            r = R[t, h - 1, 0]
            # projections by an independent, exactly rounded dot product
            p = np.array([math.fsum(float(a) * float(b) for a, b in zip(x[i], r)) for i in members])
            loff, lm = oracle.node_range(n, n0, 2 * h)
            left = set(f.perm[t][loff:loff + lm].tolist())
            assert lm == m // 2
            is_left = np.array([i in left for i in members])
            c = f.split[t, h - 1]
            tol = 1e-12 * (1 + np.abs(p).max())
            assert p[is_left].max() <= c + tol and p[~is_left].min() >= c - tol
            assert f.split_idx[t, h - 1] in members[~is_left]


def test_hand_worked_tree():
    g = {}
    for ln in _golden_lines("median_tree_1d.txt"):
        k, v = ln.split("=")
        g[k.strip()] = [float(t) for t in v.split()]
    x = np.array(g["x"], np.float32)[:, None]
    R = np.array(g["directions"], np.float32).reshape(1, 3, 1, 1)
    f = oracle.build_forest(x, R, 1, int(g["n0"][0]))
    assert f.split[0].tolist() == g["split"]
    assert f.split_idx[0].tolist() == [int(v) for v in g["split_idx"]]
    assert f.perm[0].tolist() == [int(v) for v in g["perm"]]
    assert f.leaf_of[0].tolist() == [int(v) for v in g["leaf_of"]]
    t = mini.build_tree(x, R[0], int(g["n0"][0]))
    assert t["perm"].tolist() == [int(v) for v in g["perm"]]


def _kd_tree_leaves(x, axes, n0):
    """Textbook median kd-tree: split on coordinate axes[h-1] at the element of rank
    floor(m/2) in (x_j, index) order; independent of the oracle."""
    out = {}

    def grow(members, h):
        if len(members) <= n0:
            out[h] = sorted(members)
            return
        j = axes[h - 1]
        mem = np.asarray(sorted(members))
        order = np.lexsort((mem, x[mem, j]))
        k = len(mem) // 2
        grow(mem[order[:k]].tolist(), 2 * h)
        grow(mem[order[k:]].tolist(), 2 * h + 1)

    grow(list(range(x.shape[0])), 1)
    return out


@pytest.mark.parametrize("n,d,n0", [(500, 3, 16), (1000, 8, 40), (333, 5, 7)])
def test_axis_directions_give_median_kd_tree(n, d, n0):
    x = W.gaussian_mixture(n * d, n, d, 3)
    x[1::7] = x[0]  # duplicate rows: their projections tie and the index decides
    H = _heap_count(n, n0)
    R = W.axis_directions(2, H, 1, d, seed=n)
    f = oracle.build_forest(x, R, 2, n0)
    for t in range(2):
        axes = R[t, :, 0].argmax(axis=1)
        kd = _kd_tree_leaves(x, axes, n0)
        got = {}
        for i, h in enumerate(f.leaf_of[t]):
            got.setdefault(int(h), []).append(i)
        assert got == kd


def test_one_dimension_leaves_are_sorted_blocks():
    n, n0 = 999, 30
    x = W.gaussian_mixture(1, n, 1, 2)
    f, R = _forest(x, 3, n0)
    assert set(np.unique(np.abs(R))) == {1.0}  # unit directions in 1-d are +-1
    rank = np.empty(n, int)
    rank[np.argsort(x[:, 0], kind="stable")] = np.arange(n)
    for t in range(3):
        for h in np.unique(f.leaf_of[t]):
            rk = np.sort(rank[f.leaf_of[t] == h])
            assert rk[-1] - rk[0] == len(rk) - 1  # a contiguous block of the sorted order


# ---------------------------------------------------------------- Alg. 2 (whichProjection)


def test_which_projection_picks_largest_spread():
    n, d, n0, n_try = 600, 6, 25, 4
    x = W.gaussian_mixture(8, n, d, 3, anisotropic=True)
    f, R = _forest(x, 2, n0, n_try)
    assert (f.chosen[f.chosen >= 0] > 0).any()
    for t in range(2):
        for h in range(1, (1 << f.L)):
            rr = oracle.node_range(n, n0, h)
            if rr is None or rr[1] <= n0:
                continue
            off, m = rr
            mem = np.sort(f.perm[t][off:off + m])  # node h's members: its leaves' union
            spreads = [np.var(x[mem].astype(np.float64) @ R[t, h - 1, k].astype(np.float64))
                       for k in range(n_try)]
            assert f.chosen[t, h - 1] == int(np.argmax(spreads))


# ---------------------------------------------------------------- Alg. 3 (kNN over unions)


def _numpy_knn(x, q, K, self_idx=None):
    D = ((q[:, None, :].astype(np.float64) - x[None, :, :].astype(np.float64)) ** 2).sum(-1)
    if self_idx is not None:
        D[np.arange(len(q)), self_idx] = np.inf
    idx = np.empty((len(q), K), np.int64)
    for i in range(len(q)):
        order = np.lexsort((np.arange(x.shape[0]), D[i]))
        idx[i] = order[:K]
    return idx, np.sqrt(np.take_along_axis(D, idx, 1))


def test_bruteforce_matches_numpy():
    x = W.gaussian_mixture(21, 800, 7, 5)
    q = W.gaussian_mixture(22, 50, 7, 5)
    bi, bd = oracle.bruteforce(x, q, 8)
    ni, nd = _numpy_knn(x, q, 8)
    assert np.array_equal(bi, ni)
    np.testing.assert_allclose(bd, nd, rtol=1e-12)


@pytest.mark.parametrize("n0", [400, 10_000])
def test_single_leaf_forest_is_brute_force(n0):
    # n0 >= n: every tree is one leaf, N_q = U, so the forest kNN is exact (any T)
    x = W.gaussian_mixture(30, 400, 5, 3)
    f, _ = _forest(x, 3, n0)
    assert f.L == 0
    fi, fd = oracle.all_knn(f, 7)
    ni, nd = _numpy_knn(x, x, 7, np.arange(400))
    assert np.array_equal(fi, ni)
    np.testing.assert_allclose(fd, nd, rtol=1e-12)


def test_tiny_exhaustive():
    # n <= 64: leaf sets enumerated by hand, distances as exact rationals
    n, d, n0, T, K = 48, 3, 5, 3, 4
    x = W.gaussian_mixture(40, n, d, 2)
    f, _ = _forest(x, T, n0)
    fi, _ = oracle.all_knn(f, K)
    for i in range(n):
        cand = set()
        for t in range(T):
            cand |= set(np.nonzero(f.leaf_of[t] == f.leaf_of[t][i])[0].tolist())
        cand.discard(i)
        exact = sorted((sum((Fraction(float(a)) - Fraction(float(b))) ** 2
                            for a, b in zip(x[i], x[j])), j) for j in cand)
        want = [j for _, j in exact[:K]] + [-1] * (K - min(K, len(exact)))
        assert fi[i].tolist() == want


def test_fewer_candidates_than_k_pads():
    x = W.gaussian_mixture(50, 10, 2, 2)
    f, _ = _forest(x, 1, 3)
    fi, fd = oracle.all_knn(f, 5)
    counts = np.bincount(f.leaf_of[0])[f.leaf_of[0]] - 1
    for i in range(10):
        assert (fi[i] >= 0).sum() == counts[i]
        assert np.all(fi[i][counts[i]:] == -1) and np.all(np.isinf(fd[i][counts[i]:]))


def test_twin_agrees_bit_for_bit():
    for (n, d, n0, T, n_try) in [(300, 12, 20, 3, 1), (257, 5, 9, 2, 3), (130, 40, 33, 2, 2)]:
        x = W.gaussian_mixture(n + d, n, d, 3)
        f, R = _forest(x, T, n0, n_try)
        trees = mini.build_forest(x, R, T, n0, n_try)
        for t in range(T):
            assert np.array_equal(trees[t]["perm"], f.perm[t])
            assert np.array_equal(trees[t]["leaf_of"], f.leaf_of[t])
            assert np.array_equal(trees[t]["split"], f.split[t], equal_nan=True)
            assert np.array_equal(trees[t]["chosen"], f.chosen[t])
        mi, md = mini.all_knn(x, trees, 6)
        oi, od = oracle.all_knn(f, 6)
        assert np.array_equal(mi, oi) and np.array_equal(md, od)
        q = W.gaussian_mixture(n + d + 1, 20, d, 3)
        lv = oracle.route(f, q)
        for j in range(20):
            for t in range(T):
                assert lv[t, j] == mini.route_one(q[j], trees[t], R[t], n, n0)


def test_points_route_to_their_own_leaf():
    # a data point falling through a tree lands in the leaf that holds it (no exact ties)
    x = W.gaussian_mixture(60, 3000, 10, 6)
    f, _ = _forest(x, 4, 30)
    assert np.array_equal(oracle.route(f, x), f.leaf_of)


def test_query_union_matches_brute_force_on_union():
    x = W.gaussian_mixture(61, 2000, 8, 4)
    q = W.gaussian_mixture(62, 40, 8, 4)
    f, _ = _forest(x, 5, 40)
    qi, qd = oracle.query_knn(f, q, 6)
    lv = oracle.route(f, q)
    for j in range(40):
        cand = sorted(set(np.concatenate([np.nonzero(f.leaf_of[t] == lv[t, j])[0] for t in range(5)])))
        ni, nd = _numpy_knn(x[cand], q[j:j + 1], 6)
        assert qi[j].tolist() == [cand[k] for k in ni[0]]


# ---------------------------------------------------------------- properties of the ensemble


def test_missing_rate_non_increasing_in_trees():
    # nested forests (tree t depends only on (seed, t)): N_q grows with T, so each point's
    # number of missed true neighbours and its k-th found distance cannot increase
    n, K = 3000, 10
    x = W.gaussian_mixture(70, n, 12, 8)
    f, _ = _forest(x, 8, 40)
    ti, td = oracle.bruteforce(x, x, K, np.arange(n))
    prev_miss, prev_dk = None, None
    rates = []
    for T in range(1, 9):
        fi, fd = oracle.all_knn(f, K, n_trees=T)
        miss = oracle.missing_counts(fi, ti)
        dk = fd[:, -1]
        assert np.all(dk >= td[:, -1])  # the estimated k-th distance never undercuts the truth
        if prev_miss is not None:
            assert np.all(miss <= prev_miss) and np.all(dk <= prev_dk)
        prev_miss, prev_dk = miss, dk
        rates.append(miss.mean() / K)
    assert rates[-1] < rates[0]


def test_pair_separation_decays_as_power():
    # trees are i.i.d. given the data, so P(pair separated in all of T trees) = P1^T
    n, n0, S = 120, 8, 3000
    x = W.gaussian_mixture(80, n, 4, 2)
    D = ((x[:, None] - x[None]) ** 2).sum(-1)
    np.fill_diagonal(D, np.inf)
    i, j = 0, int(np.argmin(D[0]))
    H = _heap_count(n, n0)
    sep = np.empty((S, 3), bool)
    for s in range(S):
        R = W.directions(10_000 + s, 3, H, 1, 4)
        f = oracle.build_forest(x, R, 3, n0)
        sep[s] = f.leaf_of[:, i] != f.leaf_of[:, j]
    p = sep.mean(axis=0)
    assert np.all(np.abs(p - p.mean()) < 4 * np.sqrt(p.mean() * (1 - p.mean()) / S))
    for T in (2, 3):
        joint = np.all(sep[:, :T], axis=1).mean()
        expect = np.prod(p[:T])
        sd = np.sqrt(expect * (1 - expect) / S)
        assert abs(joint - expect) < 4 * sd + 1e-3, (T, joint, expect)
