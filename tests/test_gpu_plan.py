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


def test_plan_on_the_grid_equals_each_alone():
    # data sets on the 1/255 grid with int8 tiles: the recorded graph quantises each part,
    # grows its trees from the int8 rows and runs the int8 tiles; every replay gives each data
    # set the trees and neighbours of a forest grown over it alone
    from paper_1812_11689_amd import rpf
    sizes = [2500, 900, 4000, 1800]
    dims = [40, 40, 64, 24]
    T, n0, K = 3, 100, 6
    print(f"[plan] u8grid sizes={sizes} dims={dims}", flush=True)
    xs = [W.sparse_quantized(4100 + i, n, d) for i, (n, d) in enumerate(zip(sizes, dims))]
    Rs = [W.directions(4150 + i, T, heap_count(n, n0), 1, d) for i, (n, d) in enumerate(zip(sizes, dims))]
    plan = rpf.Plan(sizes, dims, T, n0, K, dist_prec="u8grid", max_part_points=4000)
    plan.set_inputs(xs, Rs)
    for rep in range(2):
        plan.launch()
        plan.check()
        torch.cuda.synchronize()
        for i in range(len(sizes)):
            gi, gd = plan.result(i)
            ai, ad, _ = _alone(xs[i], Rs[i], T, n0, K, "u8grid")
            assert torch.equal(gi, ai) and torch.equal(gd, ad), f"replay {rep} data set {i}"
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


@pytest.mark.parametrize("n,d,n0,K,prec", [(6000, 24, 60, 8, "fp16"),     # leaves <= 64: NB 2
                                          (7800, 32, 250, 12, "bf16x3"),  # leaves of 244: NB 8
                                          (7800, 32, 250, 12, "fp32")])
def test_every_tuned_choice_gives_the_same_result(n, d, n0, K, prec, tmp_path):
    # each Phase II tile shape, bucket size and build schedule the tuner can pick, entered
    # through the tuning table, must give the forest grown alone, bit for bit
    import json
    import math
    from paper_1812_11689_amd import rpf
    T = 6
    xs, Rs = _inputs(4000 + d, [n], [d], T, n0)
    ai, ad, _ = _alone(xs[0], Rs[0], T, n0, K, prec)
    L = rpf.depth(n, n0)
    key = dict(d=d, max_leaf=-(-n // (1 << L)), prec=rpf.PREC[prec], K=K, T=T, n_log2=int(math.floor(math.log2(n))))
    mask = 7 if key["max_leaf"] > 128 else 3
    seen = set()
    try:
        for shape in range(mask + 1):
            for S in (0, 4):
                print(f"[tuned choice] {prec} n={n} shape={shape} S={S}", flush=True)
                rpf.tune_clear()
                path = tmp_path / f"t{shape}_{S}.jsonl"
                path.write_text(json.dumps(dict(key, first_trees=3, tile_shape=shape, bucket_size=S,
                                                subtrees=shape & 1)) + "\n")
                assert rpf.tune_load(str(path)) == 1
                plan = rpf.Plan([n], [d], T, n0, K, dist_prec=prec)
                ch = plan.choices()[0]
                assert ch["tile_shape"] == shape and ch["first_trees"] == 3 and ch["subtrees"] == (shape & 1)
                if S:
                    assert ch["bucket_size"] == S
                seen.add((ch["tile_shape"], ch["bucket_size"]))
                plan.set_inputs(xs, Rs)
                plan.launch()
                plan.check()
                gi, gd = plan.result(0)
                assert torch.equal(gi, ai) and torch.equal(gd, ad), (shape, S)
                plan.close()
    finally:
        rpf.tune_clear()
    assert len(seen) == 2 * (mask + 1)


def test_tuner_records_its_choices(tmp_path):
    from paper_1812_11689_amd import rpf
    sizes, dims, T, n0, K = [3000, 5000], [16, 16], 5, 40, 9
    rpf.tune_clear()
    try:
        plan = rpf.Plan(sizes, dims, T, n0, K, dist_prec="fp16")
        xs, Rs = _inputs(5000, sizes, dims, T, n0)
        plan.set_inputs(xs, Rs)
        plan.tune()
        ch = plan.choices()
        plan.launch()
        plan.check()
        for i in range(len(sizes)):
            gi, gd = plan.result(i)
            ai, ad, _ = _alone(xs[i], Rs[i], T, n0, K, "fp16")
            assert torch.equal(gi, ai) and torch.equal(gd, ad)
        plan.close()
        path = tmp_path / "tuned.jsonl"
        rpf.tune_save(str(path))
        assert len(path.read_text().splitlines()) == 1  # one part
        rpf.tune_clear()
        assert rpf.tune_load(str(path)) == 1
        again = rpf.Plan(sizes, dims, T, n0, K, dist_prec="fp16")  # takes the saved choices
        assert again.choices() == ch
        again.close()
    finally:
        rpf.tune_clear()
