"""GPU tests of the recorded build + search (rpf_plan_*): every replay of the graph, with
eager work and synchronisations between replays and new data between some of them, equals
the eager build and search over the same inputs."""

import numpy as np
import pytest
import torch

from paper_1812_11689_amd import workloads as W
from tests.helpers import heap_count

pytestmark = pytest.mark.gpu


def _inputs(seed, sizes, d, T, n0):
    xs = [W.gaussian_mixture(seed + i, n, d, 5) for i, n in enumerate(sizes)]
    Rs = [W.directions(seed + 50 + i, T, heap_count(n, n0), 1, d) for i, n in enumerate(sizes)]
    return xs, Rs


def _eager(xs, Rs, T, n0, K, prec):
    from paper_1812_11689_amd import rpf
    Xs = [torch.from_numpy(x).cuda() for x in xs]
    R = torch.from_numpy(np.concatenate(Rs, axis=1)).cuda()
    if len(xs) == 1:
        f = rpf.build(Xs[0], T, n0, R, dist_prec=prec)
    else:
        f = rpf.build_batched(Xs, T, n0, R, dist_prec=prec)
    i, dd = f.all_knn(K)
    torch.cuda.synchronize()
    f.free()
    return i, dd


@pytest.mark.parametrize("prec,d,sizes", [("fp16", 16, [900, 3000, 150, 5000, 64]), ("fp32", 40, [7000])])
def test_plan_replays_equal_eager(prec, d, sizes):
    from paper_1812_11689_amd import rpf
    T, n0, K = 3, 32, 7
    print(f"[plan] {prec} d={d} sizes={sizes}", flush=True)
    plan = rpf.Plan(sizes, d, T, n0, K, dist_prec=prec)
    for rep, seed in enumerate([1000, 1000, 2000, 1000]):
        xs, Rs = _inputs(seed, sizes, d, T, n0)
        plan.X.copy_(torch.from_numpy(np.concatenate(xs)).cuda())
        plan.directions.copy_(torch.from_numpy(np.concatenate(Rs, axis=1)).cuda())
        plan.launch()
        plan.check()
        gi, gd = plan.idx.clone(), plan.dist.clone()
        # eager work of the program between replays
        ei, ed = _eager(xs, Rs, T, n0, K, prec)
        assert torch.equal(gi, ei) and torch.equal(gd, ed), f"replay {rep}"
        dump = plan.forest.tree_dump(0)
        assert int(dump["leaf_of"].min()) >= 1
        torch.cuda.synchronize()
    plan.close()


def test_plan_reports_nonfinite_input():
    from paper_1812_11689_amd import rpf
    sizes, d, T, n0 = [500, 800], 8, 2, 30
    print("[plan] non-finite input", flush=True)
    plan = rpf.Plan(sizes, d, T, n0, 5)
    xs, Rs = _inputs(3000, sizes, d, T, n0)
    X = np.concatenate(xs)
    X[123, 4] = np.nan
    plan.X.copy_(torch.from_numpy(X).cuda())
    plan.directions.copy_(torch.from_numpy(np.concatenate(Rs, axis=1)).cuda())
    plan.launch()
    with pytest.raises(rpf.RpfError) as e:
        plan.check()
    assert e.value.status == rpf.RPF_EINVAL
    # the same plan with finite data afterwards
    X[123, 4] = 0.5
    plan.X.copy_(torch.from_numpy(X).cuda())
    plan.launch()
    plan.check()
    plan.close()
