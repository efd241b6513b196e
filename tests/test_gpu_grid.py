"""GPU parity of the all-points search over points on the 1/255 grid with the int8 tiles
(RPF_DIST_U8GRID: exact integer grid distances on the int8 MFMA, bounds off only by the
binary32 rounding of k / 255): neighbour indices bit-exact against the oracle (binary64
ranking, ties by index) and distances within 1e-5 relative, for copied-leaf and one-tile
leaf shapes, d not a multiple of 64, include/exclude self, exact duplicates (small d on the
grid), K 100, tile lists several times longer than the resident grid; queries on such a forest (binary32 tiles); data off the grid is rejected."""

import numpy as np
import pytest
import torch

import oracle
from paper_1812_11689_amd import workloads as W
from tests.helpers import problem

pytestmark = pytest.mark.gpu

CASES = [
    # name, n, d, T, n0, K, excl
    ("leaves312_d784", 20_000, 784, 4, 512, 10, 1),
    ("leaves244_d96", 7800, 96, 8, 256, 20, 1),
    ("leaves244_self", 7800, 96, 8, 256, 20, 0),
    ("leaves40_d16", 10_000, 16, 6, 50, 10, 1),
    ("d33_padding", 4000, 33, 5, 40, 7, 1),
    ("duplicates_d4", 6000, 4, 5, 60, 8, 1),
    ("big_k", 12_000, 24, 12, 200, 100, 1),
    ("leaves390_d200", 25_000, 200, 6, 400, 16, 0),
    # many more tiles than resident blocks at 64- and 128-row tiles: each block runs
    # several jobs, the next one's rows loaded during the current one
    ("many_tiles_mb2", 60_000, 8, 8, 64, 10, 1),
    ("many_tiles_mb4", 40_000, 12, 6, 128, 10, 1),
]


def _compare(gi, gd, ri, rd):
    np.testing.assert_array_equal(gi, ri)
    fin = np.isfinite(rd)
    assert np.array_equal(np.isfinite(gd), fin)
    np.testing.assert_allclose(gd[fin], rd[fin], rtol=1e-5, atol=0)


def _forest(x, R, T, n0, prec):
    from paper_1812_11689_amd import rpf
    return rpf.build(torch.from_numpy(x).cuda(), T, n0, torch.from_numpy(np.ascontiguousarray(R[:T])).cuda(),
                     dist_prec=prec)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_grid_all_knn_matches_oracle(case):
    name, n, d, T, n0, K, excl = case
    print(f"[grid] {name} n={n} d={d} T={T} n0={n0} K={K}", flush=True)
    x, R = problem(n, d, T, n0, seed=len(name) + 700, kind="quant")
    ref = oracle.build_forest(x, R, T, n0)
    ri, rd = oracle.all_knn(ref, K, exclude_self=bool(excl))
    f = _forest(x, R, T, n0, "u8grid")
    gi, gd = f.all_knn(K, exclude_self=bool(excl))
    torch.cuda.synchronize()
    st = f.knn_stats()
    print(f"    stats {st}", flush=True)
    _compare(gi.cpu().numpy(), gd.cpu().numpy(), ri, rd)
    f.free()


def test_grid_forest_queries_and_rejection():
    from paper_1812_11689_amd import rpf
    n, d, T, n0 = 9000, 48, 5, 300
    print("[grid] queries on a grid forest; off-grid data rejected", flush=True)
    x, R = problem(n, d, T, n0, seed=777, kind="quant")
    q = W.gaussian_mixture(778, 400, d, 4) * 0.1 + 0.5  # queries need not lie on the grid
    ref = oracle.build_forest(x, R, T, n0)
    ri, rd = oracle.query_knn(ref, q, 9)
    f = _forest(x, R, T, n0, "u8grid")
    gi, gd = f.query(torch.from_numpy(q.astype(np.float32)).cuda(), 9)
    torch.cuda.synchronize()
    _compare(gi.cpu().numpy(), gd.cpu().numpy(), ri, rd)
    f.free()
    bad = x.copy()
    bad[17, 3] = 0.3  # not k / 255
    with pytest.raises(rpf.RpfError) as e:
        _forest(bad, R, T, n0, "u8grid")
    assert e.value.status == rpf.RPF_EINVAL
