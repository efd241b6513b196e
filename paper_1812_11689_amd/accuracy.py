"""The accuracy workload of Sec. 5 (Figs. 2 and 3): the average missing rate m_K and the
average K-th neighbour distance of the all-points kNN search as the forest grows.

Protocol (Sec. 5, accuracy experiments): trees T in {10, 20, 40, 60, 80, 100}; K = 5 with
leaves of at most 20 points and K = 10 with leaves of at most 30; nTry per data set as the
paper lists it; results averaged over independent runs (independent direction streams).  A
second sweep varies nTry with T on the Musk-shaped set (K = 5).

The data sets of Table 1 are not available here: each is replaced by a seeded synthetic
Gaussian mixture of the same size and dimension (anisotropic clusters), so the curves are
the method's behaviour on data of those shapes, not the paper's figures.  The two sets wider
than the library's 4096 columns (Arcene, Olivetti) are left out.

Everything runs on the device through the library: forests by rpf_build, the search by
rpf_all_knn, the exact neighbours by rpf_exact_knn, the measures by `metrics`.
"""

from __future__ import annotations

import numpy as np

from . import metrics
from . import workloads as W

# Table 1 shapes (features, instances) and the paper's nTry for each data set
TABLE1 = [
    ("image_segmentation", 19, 2100, 3),
    ("parkinsons_telemonitoring", 20, 5815, 3),
    ("wdbc", 30, 569, 1),
    ("sensorless_drive", 49, 58509, 10),
    ("musk", 166, 6598, 10),
    ("ct_slice_localization", 386, 53500, 5),
    ("smartphone_activity", 561, 7767, 20),
]
TREES = (10, 20, 40, 60, 80, 100)
SETTINGS = ((5, 20), (10, 30))  # (K, leaf size)


def stand_in(name: str, d: int, n: int, seed: int = W.SEED_BASE + 900) -> np.ndarray:
    """A seeded anisotropic Gaussian mixture of n points in d dimensions (12 clusters)."""
    key = sum(ord(c) for c in name)
    return W.gaussian_mixture(seed + key, n, d, 12, anisotropic=True)


def _curve(rpf, torch, X, x_np, trees, K, n0, n_try, runs, seed, truth_i, truth_d, prec):
    n, d = x_np.shape
    L = rpf.depth(n, n0)
    H = (1 << L) - 1
    miss = np.zeros((runs, len(trees)))
    dk = np.zeros((runs, len(trees)))
    for r in range(runs):
        # one direction stream per run; forests of fewer trees are prefixes of the largest
        R = W.directions(seed + 7919 * r, max(trees), H, n_try, d)
        Rd = torch.from_numpy(R).cuda()
        for j, T in enumerate(trees):
            f = rpf.build(X, T, n0, Rd[:T].contiguous(), n_try=n_try, dist_prec=prec)
            gi, gd = f.all_knn(K)
            f.free()
            miss[r, j] = metrics.missing_rate(gi.cpu().numpy(), truth_i)
            dk[r, j] = metrics.kth_distance_excess(gd.cpu().numpy(), truth_d)
    return miss.mean(0), dk.mean(0)


def run(runs: int = 5, trees=TREES, datasets=TABLE1, prec: str = "fp32", ntry_sweep=(1, 3, 10, 20),
        progress=None) -> dict:
    """The two sweeps; returns a dict of curves (missing rate and K-th distance excess per T,
    averaged over `runs`), and for each curve the fitted decay rate of log(m_K) over T."""
    import torch
    from . import rpf

    out = {"trees": list(trees), "runs": runs, "tile_prec": prec, "data": "synthetic stand-ins of Table 1 shapes",
           "datasets": {}, "ntry_sweep": None}
    for name, d, n, n_try in datasets:
        x = stand_in(name, d, n)
        X = torch.from_numpy(x).cuda()
        entry = {"d": d, "n": n, "n_try": n_try}
        for K, n0 in SETTINGS:
            ti, td = rpf.exact_knn(X, X, K, torch.arange(n, device="cuda", dtype=torch.int64))
            truth_i, truth_d = ti.cpu().numpy(), td.cpu().numpy()
            m, e = _curve(rpf, torch, X, x, trees, K, n0, n_try, runs, W.SEED_BASE + 950, truth_i, truth_d, prec)
            entry[f"K{K}_leaf{n0}"] = {"missing_rate": [round(float(v), 6) for v in m],
                                       "kth_distance_excess": [round(float(v), 6) for v in e],
                                       "log_missing_rate_slope_per_tree": _slope(trees, m)}
            if progress:
                progress(f"{name} K={K}: missing {m[0]:.4f} -> {m[-1]:.4f}")
        out["datasets"][name] = entry
    if ntry_sweep:
        name, d, n, _ = next(t for t in datasets if t[0] == "musk") if any(t[0] == "musk" for t in datasets) \
            else datasets[0]
        x = stand_in(name, d, n)
        X = torch.from_numpy(x).cuda()
        K, n0 = SETTINGS[0]
        ti, td = rpf.exact_knn(X, X, K, torch.arange(n, device="cuda", dtype=torch.int64))
        sweep = {}
        for nt in ntry_sweep:
            m, e = _curve(rpf, torch, X, x, trees, K, n0, nt, runs, W.SEED_BASE + 990, ti.cpu().numpy(),
                          td.cpu().numpy(), prec)
            sweep[str(nt)] = {"missing_rate": [round(float(v), 6) for v in m],
                              "kth_distance_excess": [round(float(v), 6) for v in e]}
            if progress:
                progress(f"{name} nTry={nt}: missing {m[0]:.4f} -> {m[-1]:.4f}")
        out["ntry_sweep"] = {"dataset": name, "K": K, "leaf_size": n0, "curves": sweep}
    return out


def _slope(trees, m):
    """Least-squares slope of log(m_K) against T over the points with m_K > 0 (the decay rate
    the theory predicts to be negative), or None with fewer than two such points."""
    t = np.asarray(trees, float)
    v = np.asarray(m, float)
    ok = v > 0
    if ok.sum() < 2:
        return None
    return round(float(np.polyfit(t[ok], np.log(v[ok]), 1)[0]), 5)
