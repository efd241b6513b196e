"""GPU tests of the recorded build + search of many data sets (rpf_plan_*): every replay of
the graph -- with eager work and synchronisations between replays, new data between some of
them, and a re-recording by the tuner -- gives every data set the same trees and all-points
kNN as a forest grown over it alone."""

import numpy as np
import pytest
import torch

from paper_1812_11689_amd import workloads as W
from tests.helpers import heap_count

pytestmark = pytest.mark.gpu


def _inputs(seed, sizes, dims, T, n0):
    xs = [W.gaussian_mixture(seed + i, n, d, 5) for i, (n, d) in enumerate(zip(sizes, dims))]
    Rs = [W.directions(seed + 50 + i, T, heap_count(n, n0), 1, d) for i, (n, d) in enumerate(zip(sizes, dims))]
    return xs, Rs


def _alone(x, R, T, n0, K, prec):
    from paper_1812_11689_amd import rpf
    f = rpf.build(torch.from_numpy(x).cuda(), T, n0, torch.from_numpy(R).cuda(), dist_prec=prec)
    i, d = f.all_knn(K)
    dump = f.tree_dump(0)
    torch.cuda.synchronize()
    f.free()
    return i, d, dump


@pytest.mark.parametrize("prec", ["fp16", "fp32"])
def test_plan_replays_equal_each_alone(prec):
    from paper_1812_11689_amd import rpf
    sizes = [900, 3000, 150, 5000, 64, 2200, 700]
    dims = [16, 16, 8, 16, 8, 40, 16]
    T, n0, K = 3, 32, 7
    print(f"[plan] {prec} sizes={sizes} dims={dims}", flush=True)
    plan = rpf.Plan(sizes, dims, T, n0, K, dist_prec=prec, max_part_points=4000)
    assert len(plan.parts) >= 4  # d 16 is cut into several parts
    for rep, seed in enumerate([1000, 1000, 2000, 1000]):
        xs, Rs = _inputs(seed, sizes, dims, T, n0)
        plan.set_inputs(xs, Rs)
        if rep == 2:
            plan.tune()  # re-records the graph
        plan.launch()
        plan.check()
        torch.cuda.synchronize()
        for i in range(len(sizes)):
            gi, gd = plan.result(i)
            ai, ad, dump = _alone(xs[i], Rs[i], T, n0, K, prec)
            assert torch.equal(gi, ai) and torch.equal(gd, ad), f"replay {rep} data set {i}"
        # eager work of the program between replays
        torch.cuda.synchronize()
    plan.close()


def test_plan_reports_nonfinite_input():
    from paper_1812_11689_amd import rpf
    sizes, dims, T, n0 = [500, 800], [8, 8], 2, 30
    print("[plan] non-finite input", flush=True)
    plan = rpf.Plan(sizes, dims, T, n0, 5)
    xs, Rs = _inputs(3000, sizes, dims, T, n0)
    xs[1][123, 4] = np.nan
    plan.set_inputs(xs, Rs)
    plan.launch()
    with pytest.raises(rpf.RpfError) as e:
        plan.check()
    assert e.value.status == rpf.RPF_EINVAL
    xs[1][123, 4] = 0.5  # the same plan with finite data afterwards
    plan.set_inputs(xs, Rs)
    plan.launch()
    plan.check()
    ai, ad, _ = _alone(xs[1], Rs[1], T, n0, 5, "fp32")
    gi, gd = plan.result(1)
    assert torch.equal(gi, ai) and torch.equal(gd, ad)
    plan.close()
