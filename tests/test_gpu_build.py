"""GPU parity of tree growth (Alg. 1 / Alg. 2, median split): every split value (bit for
bit in binary64), split index, chosen direction, leaf order and leaf membership of every
tree equals the oracle's on the same data and directions."""

import numpy as np
import pytest
import torch

import oracle
from tests.helpers import problem

pytestmark = pytest.mark.gpu

CASES = [
    # name, n, d, T, n0, n_try, kind, dup
    ("mixture_10k_d16", 10_000, 16, 4, 50, 1, "mixture", 0),      # one multi-block level
    ("aniso_20k_d128", 20_000, 128, 3, 256, 1, "aniso", 0),
    ("d1", 3000, 1, 2, 20, 1, "mixture", 0),
    ("d33_scalar_path", 5000, 33, 2, 40, 1, "mixture", 0),
    ("ntry3_small", 3000, 12, 2, 30, 3, "aniso", 0),
    ("ntry4_large", 12_000, 20, 2, 64, 4, "aniso", 0),
    ("duplicates", 9000, 8, 3, 30, 1, "mixture", 7),
    ("wide_exponents", 6000, 24, 2, 50, 1, "wide", 0),
    ("quantized_d784", 5000, 784, 2, 512, 1, "quant", 0),
    ("single_leaf", 300, 5, 2, 300, 1, "mixture", 0),
    ("n0_plus_1", 51, 5, 2, 50, 1, "mixture", 0),
    ("tiny_n0_1", 37, 3, 2, 1, 1, "mixture", 0),
]


def _gpu_forest(x, R, T, n0, n_try):
    from paper_1812_11689_amd import rpf
    X = torch.from_numpy(x).cuda()
    Rd = torch.from_numpy(np.ascontiguousarray(R[:T])).cuda()
    return rpf.build(X, T, n0, Rd, n_try=n_try)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_build_matches_oracle(case):
    name, n, d, T, n0, n_try, kind, dup = case
    print(f"[build] {name} n={n} d={d} T={T} n0={n0} nTry={n_try}", flush=True)
    x, R = problem(n, d, T, n0, n_try, seed=len(name), kind=kind, dup_every=dup)
    ref = oracle.build_forest(x, R, T, n0, n_try)
    f = _gpu_forest(x, R, T, n0, n_try)
    info = f.info()  # synchronises and surfaces device-side invariant failures
    assert info["depth"] == ref.L
    for t in range(T):
        g = {k: v.cpu().numpy() for k, v in f.tree_dump(t).items()}
        np.testing.assert_array_equal(g["perm"], ref.perm[t])
        np.testing.assert_array_equal(g["leaf_of"], ref.leaf_of[t])
        assert np.array_equal(g["split"].view(np.uint64), ref.split[t].view(np.uint64)) or \
            np.array_equal(g["split"], ref.split[t], equal_nan=True)
        np.testing.assert_array_equal(g["split_idx"], ref.split_idx[t])
        np.testing.assert_array_equal(g["chosen"], ref.chosen[t])
    f.free()


GRID_CASES = [
    # points on the 1/255 grid, built with RPF_DIST_U8GRID: the projections read each row from
    # the int8 copy (k - 128) instead of X and must give the same splits bit for bit
    # name, n, d, T, n0, n_try
    ("grid_d784", 5000, 784, 2, 512, 1),
    ("grid_d50_multiblock", 40_000, 50, 3, 64, 1),
    ("grid_d7_ntry3", 6000, 7, 2, 30, 3),
]


@pytest.mark.parametrize("case", GRID_CASES, ids=[c[0] for c in GRID_CASES])
def test_grid_build_matches_oracle(case):
    from paper_1812_11689_amd import rpf
    name, n, d, T, n0, n_try = case
    print(f"[build] {name} n={n} d={d} T={T} n0={n0} nTry={n_try} (int8 grid rows)", flush=True)
    x, R = problem(n, d, T, n0, n_try, seed=len(name) + 50, kind="quant")
    ref = oracle.build_forest(x, R, T, n0, n_try)
    f = rpf.build(torch.from_numpy(x).cuda(), T, n0, torch.from_numpy(np.ascontiguousarray(R[:T])).cuda(),
                  n_try=n_try, dist_prec="u8grid")
    f.info()
    for t in range(T):
        g = {k: v.cpu().numpy() for k, v in f.tree_dump(t).items()}
        np.testing.assert_array_equal(g["perm"], ref.perm[t])
        np.testing.assert_array_equal(g["leaf_of"], ref.leaf_of[t])
        assert np.array_equal(g["split"].view(np.uint64), ref.split[t].view(np.uint64))
        np.testing.assert_array_equal(g["split_idx"], ref.split_idx[t])
        np.testing.assert_array_equal(g["chosen"], ref.chosen[t])
    f.free()


SUBTREE_CASES = [c for c in CASES if c[5] == 1 and c[0] not in ("single_leaf", "n0_plus_1")] + [
    # every level one-block from the root; levels of mixed leaf and internal nodes
    ("all_small_levels", 3000, 6, 3, 10, 1, "mixture", 0),
    ("n0_3_deep", 4000, 9, 2, 3, 1, "aniso", 0),
]


@pytest.mark.parametrize("case", SUBTREE_CASES, ids=[c[0] for c in SUBTREE_CASES])
def test_subtree_schedule_matches_oracle(case):
    # RPF_BUILD_SUBTREES: the one-block levels run as one persistent launch; the forest must be
    # the same, bit for bit
    from paper_1812_11689_amd import rpf
    name, n, d, T, n0, n_try, kind, dup = case
    print(f"[subtree] {name} n={n} d={d} T={T} n0={n0}", flush=True)
    x, R = problem(n, d, T, n0, n_try, seed=len(name) + 50, kind=kind, dup_every=dup)
    ref = oracle.build_forest(x, R, T, n0, n_try)
    rpf.profile_reset()
    rpf.profile_enable(True)
    f = rpf.build(torch.from_numpy(x).cuda(), T, n0, torch.from_numpy(np.ascontiguousarray(R[:T])).cuda(),
                  n_try=n_try, subtrees=True)
    info = f.info()
    rpf.profile_enable(False)
    prof = rpf.profile_read()
    if ref.L >= 2:
        assert "subtree_levels" in prof, "the persistent launch did not run"
    for t in range(T):
        g = {k: v.cpu().numpy() for k, v in f.tree_dump(t).items()}
        np.testing.assert_array_equal(g["perm"], ref.perm[t])
        np.testing.assert_array_equal(g["leaf_of"], ref.leaf_of[t])
        assert np.array_equal(g["split"].view(np.uint64), ref.split[t].view(np.uint64)) or \
            np.array_equal(g["split"], ref.split[t], equal_nan=True)
        np.testing.assert_array_equal(g["split_idx"], ref.split_idx[t])
    assert info["depth"] == ref.L
    f.free()


def test_build_twice_bit_identical():
    x, R = problem(8000, 32, 3, 40, seed=5)
    a = _gpu_forest(x, R, 3, 40, 1)
    b = _gpu_forest(x, R, 3, 40, 1)
    for t in range(3):
        da, db = a.tree_dump(t), b.tree_dump(t)
        for k in da:
            assert torch.equal(da[k].view(torch.int64) if da[k].dtype == torch.float64 else da[k],
                               db[k].view(torch.int64) if db[k].dtype == torch.float64 else db[k]), k


def test_routing_matches_oracle():
    x, R = problem(12_000, 24, 4, 60, seed=9)
    q, _ = problem(3000, 24, 1, 60, seed=19)
    ref = oracle.build_forest(x, R, 4, 60)
    f = _gpu_forest(x, R, 4, 60, 1)
    got = f.route(torch.from_numpy(q).cuda()).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.route(ref, q))
    # data points fall into their own leaves
    got_self = f.route(torch.from_numpy(x).cuda()).cpu().numpy()
    np.testing.assert_array_equal(got_self, ref.leaf_of)


def test_nonfinite_input_rejected():
    from paper_1812_11689_amd import rpf
    x, R = problem(500, 4, 2, 20, seed=3)
    x[17, 2] = np.nan
    with pytest.raises(rpf.RpfError) as e:
        _gpu_forest(x, R, 2, 20, 1)
    assert e.value.status == rpf.RPF_EINVAL


@pytest.mark.parametrize("shift", [0, 1], ids=["aligned", "unaligned"])
def test_input_copy_check_edges(shift):
    """The input copy and its non-finite check, on 16-byte aligned and unaligned inputs whose
    length is not a multiple of four: a NaN or an infinity anywhere (first value, middle, the
    last value) is rejected, and a finite input grows the same forest as the oracle."""
    from paper_1812_11689_amd import rpf
    n, d, T, n0 = 333, 3, 2, 20
    x, R = problem(n, d, T, n0, 1, seed=11)
    print(f"[build] input copy check shift={shift} n={n} d={d}", flush=True)
    Rd = torch.from_numpy(np.ascontiguousarray(R[:T])).cuda()

    def as_dev(a):
        buf = torch.zeros(n * d + 4, dtype=torch.float32, device="cuda")
        buf[shift:shift + n * d] = torch.from_numpy(a.reshape(-1)).cuda()
        return buf[shift:shift + n * d].view(n, d)

    for pos, bad in [(0, np.nan), (n * d // 2, np.inf), (n * d - 1, np.nan), (n * d - 2, -np.inf)]:
        xb = x.copy().reshape(-1)
        xb[pos] = bad
        with pytest.raises(rpf.RpfError) as e:
            rpf.build(as_dev(xb.reshape(n, d)), T, n0, Rd)
        assert e.value.status == rpf.RPF_EINVAL
    ref = oracle.build_forest(x, R, T, n0, 1)
    f = rpf.build(as_dev(x), T, n0, Rd)
    try:
        for t in range(T):
            g = {k: v.cpu().numpy() for k, v in f.tree_dump(t).items()}
            np.testing.assert_array_equal(g["perm"], ref.perm[t])
            np.testing.assert_array_equal(g["leaf_of"], ref.leaf_of[t])
            assert np.array_equal(g["split"].view(np.uint64), ref.split[t].view(np.uint64)) or \
                np.array_equal(g["split"], ref.split[t], equal_nan=True)
    finally:
        f.free()
