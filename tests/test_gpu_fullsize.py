"""Oracle parity at the full sizes of the measured workloads (Alg. 1-3):

  - 10^6 x 128 anisotropic mixture, T 32, n0 256 (the benchmark's forest): every tree's split
    values, split indices, leaf order and leaf membership bit-exact; all-points kNN (K 20) at
    binary32 and bfloat16 tiles on a seeded sample of 20 000 rows, indices bit-exact and
    distances within 1e-5 relative;
  - the served forest, 4 * 10^6 x 96, T 64, n0 256, float16 tiles: 5 000 mixture queries (5 %
    uniform outliers) at K 1, 10 and 100;
  - 10^5 x 784 quantised (70 % zeros, 1/255 grid), T 48, n0 512, bfloat16 tiles (leaves of
    390/391 points take the copied-leaf tiles) and int8 grid tiles: the whole build and kNN on
    5 000 sampled rows.

The oracle runs on the host cores (OpenMP); these cases take about a minute each."""

import numpy as np
import pytest
import torch

import oracle
from paper_1812_11689_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]

RTOL = 1e-5


def _compare(gi, gd, ri, rd, what):
    np.testing.assert_array_equal(gi, ri, err_msg=what)
    fin = np.isfinite(rd)
    assert np.array_equal(np.isfinite(gd), fin), what
    np.testing.assert_allclose(gd[fin], rd[fin], rtol=RTOL, atol=0, err_msg=what)


def _check_trees(f, ref, T):
    for t in range(T):
        dump = f.tree_dump(t)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(dump["perm"].cpu().numpy(), ref.perm[t], err_msg=f"perm of tree {t}")
        np.testing.assert_array_equal(dump["leaf_of"].cpu().numpy(), ref.leaf_of[t], err_msg=f"leaf_of of tree {t}")
        g = dump["split"].cpu().numpy()
        assert np.array_equal(g.view(np.uint64), ref.split[t].view(np.uint64)) or \
            np.array_equal(g, ref.split[t], equal_nan=True), f"split of tree {t}"
        np.testing.assert_array_equal(dump["split_idx"].cpu().numpy(), ref.split_idx[t],
                                      err_msg=f"split_idx of tree {t}")


def _build(x, R, T, n0, prec):
    from paper_1812_11689_amd import rpf
    return rpf.build(torch.from_numpy(x).cuda(), T, n0, torch.from_numpy(np.ascontiguousarray(R[:T])).cuda(),
                     dist_prec=prec)


def _sample(seed, n, m):
    return np.sort(np.random.default_rng(seed).choice(n, size=m, replace=False))


def test_1M_d128_T32_build_and_all_knn():
    w = W.make_config(2)
    x, T, n0, K = w.x, w.n_trees, w.leaf_size, w.k
    n, d = x.shape
    L = oracle.depth(n, n0)
    print(f"[fullsize] {w.name}: n={n} d={d} T={T} n0={n0} K={K} L={L}", flush=True)
    R = W.directions(w.dir_seed, T, (1 << L) - 1, 1, d)
    ref = oracle.build_forest(x, R, T, n0)
    print("    oracle forest built", flush=True)
    pts = _sample(W.SEED_BASE + 302, n, 20_000)
    ri, rd = oracle.all_knn(ref, K, points=pts)
    print("    oracle kNN of 20000 sampled rows done", flush=True)
    for prec in ("fp32", "bf16"):
        f = _build(x, R, T, n0, prec)
        if prec == "fp32":
            _check_trees(f, ref, T)
            print(f"    {T} trees bit-exact", flush=True)
        gi, gd = f.all_knn(K)
        torch.cuda.synchronize()
        st = f.knn_stats()
        print(f"    {prec} stats {st}", flush=True)
        sel = torch.from_numpy(pts).cuda().long()
        _compare(gi[sel].cpu().numpy(), gd[sel].cpu().numpy(), ri, rd, f"all_knn {prec}")
        print(f"    {prec} all_knn sample matches", flush=True)
        f.free()
        del gi, gd


def test_4M_d96_T64_served_queries():
    w = W.make_config(4)
    x, T, n0 = w.x, w.n_trees, w.leaf_size
    n, d = x.shape
    L = oracle.depth(n, n0)
    print(f"[fullsize] {w.name}: n={n} d={d} T={T} n0={n0} L={L} fp16", flush=True)
    R = W.directions(w.dir_seed, T, (1 << L) - 1, 1, d)
    q = W.mixture_queries(W.SEED_BASE + 204, x, 5000, 1000, mean_seed=W.SEED_BASE + 4)
    ref = oracle.build_forest(x, R, T, n0)
    print("    oracle forest built", flush=True)
    f = _build(x, R, T, n0, "fp16")
    Q = torch.from_numpy(q).cuda()
    leaf = f.route(Q)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(leaf.cpu().numpy(), oracle.route(ref, q), err_msg="routing")
    print("    routing of 5000 queries through 64 trees matches", flush=True)
    for K in (1, 10, 100):
        ri, rd = oracle.query_knn(ref, q, K)
        gi, gd = f.query(Q, K)
        torch.cuda.synchronize()
        f.knn_stats()
        _compare(gi.cpu().numpy(), gd.cpu().numpy(), ri, rd, f"query K={K}")
        print(f"    K={K} matches", flush=True)
    f.free()


@pytest.mark.parametrize("prec", ["bf16", "u8grid"])
def test_100k_d784_T48_quantised(prec):
    n, d, T, n0, K = 100_000, 784, 48, 512, 10
    x = W.sparse_quantized(W.SEED_BASE + 3, n, d)
    L = oracle.depth(n, n0)
    print(f"[fullsize] quantised n={n} d={d} T={T} n0={n0} K={K} L={L} {prec}", flush=True)
    R = W.directions(W.SEED_BASE + 103, T, (1 << L) - 1, 1, d)
    ref = oracle.build_forest(x, R, T, n0)
    f = _build(x, R, T, n0, prec)
    _check_trees(f, ref, T)
    print(f"    {T} trees bit-exact", flush=True)
    pts = _sample(W.SEED_BASE + 303, n, 5000)
    ri, rd = oracle.all_knn(ref, K, points=pts)
    gi, gd = f.all_knn(K)
    torch.cuda.synchronize()
    st = f.knn_stats()
    print(f"    stats {st}", flush=True)
    sel = torch.from_numpy(pts).cuda().long()
    _compare(gi[sel].cpu().numpy(), gd[sel].cpu().numpy(), ri, rd, f"all_knn {prec} quantised")
    print("    all_knn sample matches", flush=True)
    f.free()
