"""GPU parity of the uniform split rule (Alg. 1 as printed: c drawn uniformly between the
smallest and the largest projection of the node).  Tree growth: every leaf order and leaf
ordinal, and every attempted split (heap id, split value bit for bit in binary64, size, left
size, chosen try, depth), equals the oracle's for the same data and seed.  All-points search
over the resulting forests: indices bit-exact against the oracle's union of each point's
leaves, distances within 1e-5 relative, in every tile precision.  Queries are refused."""

import numpy as np
import pytest
import torch

import oracle
from tests.helpers import problem

pytestmark = pytest.mark.gpu

BUILD_CASES = [
    # name, n, d, T, n0, n_try, seed, kind, dup
    ("block_d16", 3000, 16, 4, 20, 1, 11, "mixture", 0),           # one block per node
    ("block_d33_ntry3", 4000, 33, 3, 25, 3, 12, "aniso", 0),        # scalar projection path
    ("chunked_d8_ntry2", 20_000, 8, 3, 10, 2, 13, "mixture", 0),   # roots above one chunk
    ("chunked_d128", 50_000, 128, 2, 30, 1, 14, "aniso", 0),
    ("ntry5_wide_seed", 9000, 12, 2, 16, 5, 2**64 - 3, "aniso", 0),
    ("duplicates", 6000, 4, 3, 20, 1, 15, "mixture", 2),           # 3000 copies: a leaf of 3000
    ("wide_exponents", 5000, 24, 2, 30, 1, 16, "wide", 0),
    ("quantized_d784", 3000, 784, 2, 40, 1, 17, "quant", 0),
    ("single_leaf", 200, 5, 2, 200, 1, 18, "mixture", 0),
    ("one_point", 1, 3, 2, 1, 1, 19, "mixture", 0),
    ("n0_1", 300, 3, 2, 1, 2, 20, "mixture", 0),
]


def _x(case):
    name, n, d, T, n0, n_try, seed, kind, dup = case
    x, _ = problem(n, d, 1, max(n0, 1), 1, seed=len(name) + 900, kind=kind, dup_every=dup)
    return x


def _gpu(x, T, n0, n_try, seed, prec="fp32"):
    from paper_1812_11689_amd import rpf
    return rpf.build(torch.from_numpy(x).cuda(), T, n0, None, n_try=n_try, dist_prec=prec, split_rule="uniform",
                     seed=seed)


@pytest.mark.parametrize("case", BUILD_CASES, ids=[c[0] for c in BUILD_CASES])
def test_uniform_build_matches_oracle(case):
    name, n, d, T, n0, n_try, seed, kind, dup = case
    print(f"[uniform build] {name} n={n} d={d} T={T} n0={n0} nTry={n_try}", flush=True)
    x = _x(case)
    ref = oracle.build_uniform(x, T, n0, seed, n_try=n_try, nodes=True)
    f = _gpu(x, T, n0, n_try, seed)
    info = f.info()
    assert info["split_rule"] == 1
    assert info["depth"] == int(ref.max_depth.max())
    assert info["n_leaves"] == int(ref.nleaf.max())
    for t in range(T):
        g = {k: v.cpu().numpy() for k, v in f.tree_dump(t).items()}
        np.testing.assert_array_equal(g["perm"], ref.perm[t])
        np.testing.assert_array_equal(g["leaf_of"], ref.leaf_of[t])
        nodes = sorted(f.tree_nodes(t), key=lambda r: r["heap"])
        rn = ref.nodes[t]
        order = np.argsort(rn["heap"])
        assert [r["heap"] for r in nodes] == rn["heap"][order].tolist()
        got_c = np.array([r["split"] for r in nodes], np.float64)
        assert np.array_equal(got_c.view(np.uint64), rn["c"][order].view(np.uint64))
        for key, col in (("size", "size"), ("left", "left"), ("chosen", "chosen"), ("depth", "depth")):
            assert [r[key] for r in nodes] == rn[col][order].tolist(), key
    f.free()


KNN_CASES = [
    # name, n, d, T, n0, n_try, seed, kind, dup, K, prec, exclude_self
    ("fp32_k10", 6000, 16, 8, 20, 1, 31, "mixture", 0, 10, "fp32", True),
    ("bf16_k5", 6000, 32, 6, 24, 2, 32, "aniso", 0, 5, "bf16", True),
    ("fp16_k7", 5000, 20, 6, 30, 1, 33, "mixture", 0, 7, "fp16", False),
    ("bf16x3_k20", 8000, 64, 10, 40, 1, 34, "aniso", 0, 20, "bf16x3", True),
    ("u8grid_k10", 4000, 96, 8, 30, 1, 35, "quant", 0, 10, "u8grid", True),
    ("chunked_k8", 24_000, 8, 6, 16, 1, 36, "mixture", 0, 8, "fp32", True),
    ("duplicates_big_leaf", 3000, 4, 4, 20, 1, 37, "mixture", 2, 6, "fp32", True),
    ("k_above_leaves", 2000, 6, 3, 8, 1, 38, "mixture", 0, 40, "fp32", True),
]


@pytest.mark.parametrize("case", KNN_CASES, ids=[c[0] for c in KNN_CASES])
def test_uniform_all_knn_matches_oracle(case):
    name, n, d, T, n0, n_try, seed, kind, dup, K, prec, excl = case
    print(f"[uniform knn] {name} n={n} d={d} T={T} n0={n0} K={K} {prec}", flush=True)
    x, _ = problem(n, d, 1, n0, 1, seed=len(name) + 950, kind=kind, dup_every=dup)
    ref = oracle.build_uniform(x, T, n0, seed, n_try=n_try)
    ri, rd = oracle.all_knn_uniform(ref, K, exclude_self=excl)
    f = _gpu(x, T, n0, n_try, seed, prec)
    gi, gd = f.all_knn(K, exclude_self=excl)
    torch.cuda.synchronize()
    st = f.knn_stats()
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    np.testing.assert_array_equal(gi, ri)
    fin = np.isfinite(rd)
    assert np.array_equal(np.isfinite(gd), fin)
    np.testing.assert_allclose(gd[fin], rd[fin], rtol=1e-5, atol=0)
    assert st["rows"] == n
    f.free()


def test_uniform_forest_refuses_queries():
    from paper_1812_11689_amd import rpf
    x, _ = problem(500, 8, 1, 20, 1, seed=3)
    f = _gpu(x, 2, 20, 1, 7)
    q = torch.from_numpy(x[:10]).cuda()
    for call in (lambda: f.query(q, 5), lambda: f.route(q)):
        with pytest.raises(rpf.RpfError) as e:
            call()
        assert e.value.status == rpf.RPF_EINVAL
    f.free()


def test_uniform_seed_changes_trees_and_same_seed_repeats():
    x, _ = problem(4000, 10, 1, 20, 1, seed=4)
    a, b, c = _gpu(x, 2, 20, 1, 100), _gpu(x, 2, 20, 1, 100), _gpu(x, 2, 20, 1, 101)
    pa, pb, pc = (f.tree_dump(0)["perm"].cpu().numpy() for f in (a, b, c))
    assert np.array_equal(pa, pb) and not np.array_equal(pa, pc)
    for f in (a, b, c):
        f.free()
