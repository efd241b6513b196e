"""The accuracy workload of Sec. 5 (missing rate and K-th distance as the forest grows) on
two Table-1-shaped stand-ins: the measures never increase with T over nested forests, the
K-th distance never falls below the exact one, and one point of a curve equals the oracle's
own forest, search, brute force and missing rate on the same directions."""

import numpy as np
import pytest

import oracle
from paper_1812_11689_amd import accuracy
from paper_1812_11689_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_sweep_curves_monotone_and_match_oracle():
    ds = [t for t in accuracy.TABLE1 if t[0] in ("wdbc", "image_segmentation")]
    print("[accuracy] reduced sweep on", [t[0] for t in ds], flush=True)
    out = accuracy.run(runs=2, trees=(10, 20, 40), datasets=ds, ntry_sweep=(1, 3))
    for name, entry in out["datasets"].items():
        for key in ("K5_leaf20", "K10_leaf30"):
            m = entry[key]["missing_rate"]
            e = entry[key]["kth_distance_excess"]
            print(f"    {name} {key}: {m} {e}", flush=True)
            assert all(a >= b - 1e-12 for a, b in zip(m, m[1:])), (name, key, m)
            assert all(a >= b - 1e-9 for a, b in zip(e, e[1:])), (name, key, e)
            assert min(e) >= -1e-7
    # the first point of wdbc's K 5 curve, run 0 and run 1, through the oracle alone
    name, d, n, n_try = next(t for t in ds if t[0] == "wdbc")
    x = accuracy.stand_in(name, d, n)
    ti, _ = oracle.bruteforce(x, x, 5, np.arange(n))
    L = oracle.depth(n, 20)
    vals = []
    for r in range(2):
        R = W.directions(W.SEED_BASE + 950 + 7919 * r, 40, (1 << L) - 1, n_try, d)
        f = oracle.build_forest(x, R, 10, 20, n_try)
        gi, _ = oracle.all_knn(f, 5)
        vals.append(oracle.missing_rate(gi, ti))
    assert abs(np.mean(vals) - out["datasets"]["wdbc"]["K5_leaf20"]["missing_rate"][0]) < 1e-6
