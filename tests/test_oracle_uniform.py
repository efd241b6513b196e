"""Pins for the oracle's uniform split rule (Alg. 1 as printed: the split point c is drawn
uniformly between the smallest and the largest projection of the node).  The random numbers
come from SplitMix64, pinned to its published outputs; the rest is checked against
distributional facts (u and the split fraction uniform on [0, 1), direction coordinates with
the Irwin-Hall moments), special cases that fix the answer (identical points make one leaf;
on a line every leaf is an interval of the sorted values; a single leaf makes the search a
brute force), invariants of the partition, and the independent pure-Python twin.  CPU only."""

import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import mini

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _vectors():
    out = []
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as fh:
        for ln in fh:
            if ln.strip() and not ln.startswith("#"):
                s, i, v = [c.strip() for c in ln.split("|")]
                out.append((int(s), int(i), int(v, 16)))
    return out


@pytest.mark.parametrize("impl", ["c", "python"])
def test_splitmix64_published_outputs(impl):
    fn = oracle.stream if impl == "c" else mini.stream
    vec = _vectors()
    assert len(vec) >= 3
    for s, i, v in vec:
        assert fn(s, i) == v


def _unmix64(z):
    """Inverse of mix64: each xor-shift and odd multiplication is undone in turn."""
    M = (1 << 64) - 1

    def unxorshift(y, k):
        x = y
        for _ in range(64 // k + 1):
            x = y ^ (x >> k)
        return x & M

    z = unxorshift(z, 31)
    z = (z * pow(0x94D049BB133111EB, -1, 1 << 64)) & M
    z = unxorshift(z, 27)
    z = (z * pow(0xBF58476D1CE4E5B9, -1, 1 << 64)) & M
    return unxorshift(z, 30)


def test_mix64_is_a_bijection():
    rng = np.random.default_rng(0)
    for v in [0, 1, (1 << 64) - 1] + [int(a) for a in rng.integers(0, 2**63, 200, dtype=np.int64)]:
        assert _unmix64(oracle.mix64(v)) == v
        assert oracle.mix64(v) == mini.mix64(v)


def test_node_streams_are_keyed_by_seed_tree_and_node():
    # distinct (seed, tree, node) give distinct stream seeds; the C and Python keys agree
    keys = {}
    for seed in (0, 1, 2**63 + 5):
        for t in range(4):
            for h in (1, 2, 3, 1 << 40, (1 << 62) + 7):
                k = oracle.node_key(seed, t, h)
                assert k == mini.node_key(seed, t, h)
                assert k not in keys
                keys[k] = (seed, t, h)


def test_split_fraction_u_is_uniform():
    u = np.array([oracle.node_u(oracle.node_key(11, t, h)) for t in range(8) for h in range(1, 2001)])
    assert u.min() >= 0.0 and u.max() < 1.0
    # 53-bit grid
    assert np.all(u * 2.0**53 == np.floor(u * 2.0**53))
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    assert np.array_equal(u[:50], [mini.node_u(mini.node_key(11, 0, h)) for h in range(1, 51)])


def test_direction_coordinates_have_irwin_hall_moments():
    d = 64
    R = np.stack([oracle.node_direction(oracle.node_key(5, t, h), i, d)
                  for t in range(3) for h in range(1, 301) for i in range(2)]).astype(np.float64)
    v = R.ravel()
    assert abs(v.mean()) < 0.01
    assert abs(v.var() - 1.0) < 0.01
    # Irwin-Hall(12) - 6: kurtosis 3 - 6 / (5 * 12) = 2.9; support [-6, 6]
    assert abs(stats.kurtosis(v, fisher=False) - 2.9) < 0.03
    assert np.abs(v).max() <= 6.0
    # coordinates and tries are uncorrelated
    c = np.corrcoef(R[:, :8].T)
    assert np.abs(c - np.eye(8)).max() < 0.05
    # the C and Python draws agree bit for bit
    for t, h, i in [(0, 1, 0), (2, 77, 1), (1, 5000, 3)]:
        k = oracle.node_key(5, t, h)
        assert np.array_equal(oracle.node_direction(k, i, d), mini.node_direction(k, i, d))


def _check_partition(f):
    """Every tree: perm is a permutation, leaves sit together in perm with ascending members,
    ordinals run 0..nleaf-1 left to right, and a leaf above n0 comes from an empty child."""
    n = f.n
    for t in range(f.n_trees):
        perm, lo = f.perm[t], f.leaf_of[t]
        assert np.array_equal(np.sort(perm), np.arange(n))
        seq = lo[perm]
        assert seq[0] == 0 and np.all(np.diff(seq) >= 0) and np.all(np.diff(seq) <= 1)
        assert seq[-1] == f.nleaf[t] - 1
        starts = np.flatnonzero(np.r_[True, np.diff(seq) > 0])
        ends = np.r_[starts[1:], n]
        for s, e in zip(starts, ends):
            assert np.all(np.diff(perm[s:e]) > 0)
        sizes = ends - starts
        if f.nodes is not None:
            nd = f.nodes[t]
            stuck = int(np.sum((nd["left"] == 0) | (nd["left"] == nd["size"])))
            assert int(np.sum(sizes > f.n0)) <= stuck
        yield t, starts, ends


def test_identical_points_make_one_leaf():
    x = np.full((500, 7), 0.25, np.float32)
    f = oracle.build_uniform(x, 3, 20, seed=9, n_try=2, nodes=True)
    for t in range(3):
        assert f.nleaf[t] == 1 and f.max_depth[t] == 0
        assert np.array_equal(f.perm[t], np.arange(500))
        nd = f.nodes[t]
        assert list(nd["heap"]) == [1] and nd["a"][0] == nd["b"][0] == nd["c"][0] and nd["left"][0] == 0
    list(_check_partition(f))


def test_on_a_line_every_leaf_is_an_interval():
    rng = np.random.default_rng(4)
    x = rng.permutation(np.arange(3000, dtype=np.float32) * 0.5 + 1.0)[:, None]
    f = oracle.build_uniform(x, 4, 25, seed=21, nodes=True)
    v = x[:, 0]
    for t, starts, ends in _check_partition(f):
        assert np.all(ends - starts <= 25)
        for s, e in zip(starts, ends):
            mem = v[f.perm[t][s:e]]
            lo, hi = mem.min(), mem.max()
            inside = np.count_nonzero((v >= lo) & (v <= hi))
            assert inside == e - s


def test_split_point_is_uniform_between_min_and_max():
    rng = np.random.default_rng(8)
    x = rng.standard_normal((20000, 6)).astype(np.float32)
    f = oracle.build_uniform(x, 4, 10, seed=77, n_try=3, nodes=True)
    frac = []
    for t, _, _ in _check_partition(f):
        nd = f.nodes[t]
        a, b, c = nd["a"], nd["b"], nd["c"]
        assert np.all((a <= c) & (c <= b))
        ok = (b - a) > 1e-9 * np.maximum(np.abs(a), np.abs(b))
        frac.append(((c - a) / (b - a))[ok])
        assert np.all(nd["chosen"] < 3)
        # children are one level down and every heap id is unique
        assert len(set(nd["heap"].tolist())) == len(nd["heap"])
    frac = np.concatenate(frac)
    assert frac.size > 5000
    assert stats.kstest(frac, "uniform").pvalue > 1e-3


def test_left_sizes_match_a_numpy_replay_on_exact_data():
    # points on a coarse integer grid in d = 3 and one try: every product x_j r_j is exact in
    # binary64 and so is the sum of three of them (at most 24 + 4 + 2 significant bits), so
    # numpy's x @ r equals the canonical projection and the partition can be replayed
    rng = np.random.default_rng(12)
    x = rng.integers(-8, 8, (400, 3)).astype(np.float32)
    f = oracle.build_uniform(x, 2, 12, seed=5, nodes=True)
    for t in range(2):
        nd = f.nodes[t]
        members = {1: np.arange(400)}
        for h, a, b, c, m, nl in zip(nd["heap"], nd["a"], nd["b"], nd["c"], nd["size"], nd["left"]):
            mem = members.pop(int(h))
            assert mem.size == m
            r = mini.node_direction(mini.node_key(5, t, int(h)), 0, 3).astype(np.float64)
            p = x[mem].astype(np.float64) @ r
            assert p.min() == a and p.max() == b
            assert c == a + mini.node_u(mini.node_key(5, t, int(h))) * (b - a)
            left = mem[p < c]
            assert left.size == nl
            if 0 < nl < m:
                members[2 * int(h)] = left
                members[2 * int(h) + 1] = mem[p >= c]
            else:
                members[-int(h)] = mem  # an empty child: the node stays whole, as a leaf
        # what the replay left unsplit are exactly the oracle's leaves
        leaves = sorted(tuple(sorted(v.tolist())) for v in members.values())
        got = sorted(tuple(np.flatnonzero(f.leaf_of[t] == k).tolist()) for k in range(f.nleaf[t]))
        assert leaves == got


@pytest.mark.parametrize("n,d,T,n0,n_try,seed,dup", [
    (200, 3, 3, 8, 1, 0, 0),
    (300, 5, 2, 10, 3, 1234, 0),
    (250, 33, 2, 16, 2, 2**64 - 1, 0),
    (240, 4, 2, 6, 1, 7, 3),     # every third point repeated
])
def test_c_oracle_equals_python_twin(n, d, T, n0, n_try, seed, dup):
    rng = np.random.default_rng(n + d)
    x = rng.standard_normal((n, d)).astype(np.float32)
    if dup:
        x[::dup] = x[0]
    f = oracle.build_uniform(x, T, n0, seed, n_try=n_try, nodes=True)
    for t in range(T):
        m = mini.build_tree_uniform(x, seed, t, n0, n_try)
        assert np.array_equal(m["perm"], f.perm[t])
        assert np.array_equal(m["leaf_of"], f.leaf_of[t])
        assert m["nleaf"] == f.nleaf[t] and m["max_depth"] == f.max_depth[t]
        nd = f.nodes[t]
        got = list(zip(nd["heap"].tolist(), nd["a"].tolist(), nd["b"].tolist(), nd["c"].tolist(),
                       nd["size"].tolist(), nd["left"].tolist(), nd["chosen"].tolist(), nd["depth"].tolist()))
        assert got == [tuple(v) for v in m["nodes"]]
    list(_check_partition(f))


def test_single_leaf_search_is_brute_force():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((60, 9)).astype(np.float32)
    f = oracle.build_uniform(x, 3, 60, seed=1)
    assert np.all(f.nleaf == 1)
    gi, gd = oracle.all_knn_uniform(f, 7)
    bi, bd = oracle.bruteforce(x, x, 7, np.arange(60))
    assert np.array_equal(gi, bi) and np.array_equal(gd, bd)


def test_search_over_uniform_leaves_matches_twin_union():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((180, 4)).astype(np.float32)
    f = oracle.build_uniform(x, 5, 9, seed=31, n_try=2)
    gi, gd = oracle.all_knn_uniform(f, 5)
    trees = [dict(leaf_of=f.leaf_of[t]) for t in range(5)]
    for i in range(180):
        ei, ed = mini.knn_union(x, trees, [f.leaf_of[t][i] for t in range(5)], x[i], 5, i)
        assert np.array_equal(ei, gi[i])
        np.testing.assert_array_equal(ed, gd[i])


def test_more_trees_miss_fewer_neighbours():
    # Sec. 5: the missing rate falls as trees are added (here on a fixed uniform forest grown
    # once and searched over its first T trees)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3000, 8)).astype(np.float32)
    f = oracle.build_uniform(x, 40, 20, seed=3, n_try=3)
    ti, _ = oracle.bruteforce(x, x, 5, np.arange(3000))
    rates = [oracle.missing_rate(oracle.all_knn_uniform(f, 5, n_trees=T)[0], ti) for T in (1, 5, 20, 40)]
    assert all(b <= a for a, b in zip(rates, rates[1:]))
    assert rates[-1] < 0.5 * rates[0]
