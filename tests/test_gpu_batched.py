"""GPU tests of forests over many data sets grown together (rpf_build_batched): every data
set's trees and all-points kNN equal those of a forest grown over that data set alone with
the same directions, and the oracle's."""

import numpy as np
import pytest
import torch

import oracle
from paper_1812_11689_amd import workloads as W
from tests.helpers import heap_count

pytestmark = pytest.mark.gpu


def _sets(seed, sizes, d, clusters=6):
    return [W.gaussian_mixture(seed + i, n, d, clusters) for i, n in enumerate(sizes)]


@pytest.mark.parametrize("prec,d,sizes,subtrees", [
    ("fp16", 24, [300, 1500, 4000, 77, 2500, 10_000, 41], False),
    ("fp32", 8, [2000, 130, 6000, 999], False),
    ("bf16", 64, [5000, 800, 3000], False),
    # the one-block levels of every data set in one persistent launch
    ("fp16", 24, [300, 1500, 4000, 77, 2500, 10_000, 41], True),
    ("fp32", 33, [9000, 130, 6000, 40, 999], True),
])
def test_batched_equals_each_alone(prec, d, sizes, subtrees):
    from paper_1812_11689_amd import rpf
    T, n0, K = 3, 40, 9
    print(f"[batched] {prec} d={d} sizes={sizes} subtrees={subtrees}", flush=True)
    xs = _sets(700 + d, sizes, d)
    Rs = [W.directions(800 + d + i, T, heap_count(n, n0), 1, d) for i, n in enumerate(sizes)]
    R = torch.from_numpy(np.concatenate(Rs, axis=1)).cuda()
    Xs = [torch.from_numpy(x).cuda() for x in xs]
    bf = rpf.build_batched(Xs, T, n0, R, dist_prec=prec, subtrees=subtrees)
    parts = bf.all_knn_split(K)
    bf.knn_stats()  # raises on an out-of-range candidate index (internal error)
    ents = bf.entries()
    dumps = [bf.tree_dump(t) for t in range(T)]
    torch.cuda.synchronize()
    for i, (x, Ri) in enumerate(zip(xs, Rs)):
        f = rpf.build(Xs[i], T, n0, torch.from_numpy(Ri).cuda(), dist_prec=prec)
        k = min(K, len(x) - 1)
        ai, ad = f.all_knn(k)
        torch.cuda.synchronize()
        gi, gd = parts[i]
        assert torch.equal(gi[:, :k], ai) and torch.equal(gd[:, :k], ad), f"data set {i}"
        if k < K:  # fewer candidates than K: padded tail
            assert bool((gi[:, k:] == -1).all()) and bool(torch.isinf(gd[:, k:]).all())
        e = ents[i]
        H = heap_count(len(x), n0)
        for t in range(T):
            alone = f.tree_dump(t)
            hb = e["heap_base"]
            a, b = dumps[t]["split"][hb:hb + H], alone["split"]
            assert bool(((a == b) | (torch.isnan(a) & torch.isnan(b))).all())
            assert torch.equal(dumps[t]["chosen"][hb:hb + H], alone["chosen"])
            lo = e["offset"]
            assert torch.equal(dumps[t]["leaf_of"][lo:lo + len(x)] - e["leaf_heap_base"], alone["leaf_of"])
            assert torch.equal(dumps[t]["perm"][lo:lo + len(x)] - lo, alone["perm"])
        f.free()
    # the smallest and the largest data set against the oracle
    for i in (int(np.argmin(sizes)), int(np.argmax(sizes))):
        ref = oracle.build_forest(xs[i], Rs[i], T, n0)
        k = min(K, len(xs[i]) - 1)
        ri, rd = oracle.all_knn(ref, k)
        np.testing.assert_array_equal(parts[i][0][:, :k].cpu().numpy(), ri)
        np.testing.assert_allclose(parts[i][1][:, :k].cpu().numpy(), rd, rtol=1e-5)
    assert bf.info()["batch_count"] == len(sizes)
    bf.free()


def test_batched_forest_rejects_queries():
    from paper_1812_11689_amd import rpf
    xs = _sets(900, [500, 700], 16)
    Rs = [W.directions(901 + i, 2, heap_count(len(x), 30), 1, 16) for i, x in enumerate(xs)]
    bf = rpf.build_batched([torch.from_numpy(x).cuda() for x in xs], 2, 30,
                           torch.from_numpy(np.concatenate(Rs, axis=1)).cuda())
    with pytest.raises(rpf.RpfError):
        bf.query(torch.from_numpy(xs[0][:5]).cuda(), 3)
    bf.free()
