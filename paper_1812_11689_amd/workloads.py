"""Seeded synthetic inputs for the rpForests kNN path: data sets, query streams and the
random split directions of the forest.

This module draws random numbers and nothing else. It holds none of the method's
arithmetic: tree shapes, projections, splits and distances live in the HIP library and,
independently, in the CPU oracle. Both are fed the arrays produced here.

Random directions (Alg. 1 draws one per split node, Alg. 2 draws nTry of them) are
passed to both sides as an input array R[t][h-1][try][:] (heap id h, root h = 1), drawn
per tree from its own stream keyed by (seed, t).  A forest of T trees is therefore the
T-prefix of any larger forest drawn with the same seed.

Every generator uses numpy's PCG64 bit generator seeded through SeedSequence, so that a
(seed, shape) pair always yields the same array on any machine with this numpy version.
"""

from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 11689000  # data seeds are SEED_BASE + c, directions + 100, queries + 200


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def directions(seed: int, n_trees: int, n_heap: int, n_try: int, d: int,
               first_tree: int = 0) -> np.ndarray:
    """Random split directions, float32 [n_trees][n_heap][n_try][d].

    Each row is a standard normal vector divided by its (float64) Euclidean norm and then
    rounded to float32, i.e. a direction drawn uniformly from the unit sphere (the paper
    samples split hyperplanes from the unit sphere).  Tree t uses stream (seed, t).
    `n_heap` is the number of heap slots 2^L - 1 of the tree shape; it may be 0.
    """
    out = np.empty((n_trees, n_heap, n_try, d), dtype=np.float32)
    for k in range(n_trees):
        g = _rng(seed, first_tree + k).standard_normal((n_heap, n_try, d))
        nrm = np.sqrt(np.einsum("hjd,hjd->hj", g, g))[..., None]
        out[k] = (g / nrm).astype(np.float32)
    return out


def axis_directions(n_trees: int, n_heap: int, n_try: int, d: int, seed: int = 0) -> np.ndarray:
    """Coordinate-axis directions e_j with j drawn per (tree, node, try): the kd-tree case."""
    rng = _rng(seed, 7)
    axes = rng.integers(0, d, size=(n_trees, n_heap, n_try))
    out = np.zeros((n_trees, n_heap, n_try, d), dtype=np.float32)
    np.put_along_axis(out, axes[..., None], 1.0, axis=-1)
    return out


def gaussian_mixture(seed: int, n: int, d: int, n_clusters: int, mean_sd: float = 5.0,
                     anisotropic: bool = False, return_labels: bool = False):
    """Mixture of Gaussians, float32 [n][d].

    Cluster means ~ N(0, mean_sd^2 I); labels uniform.  Isotropic clusters have identity
    covariance.  Anisotropic clusters have covariance Q diag(lambda) Q^T with lambda_j
    log-uniform in [0.01, 1] and Q a Haar-random orthogonal matrix (QR of a Gaussian
    matrix with the signs of R's diagonal folded into Q).
    """
    rng = _rng(seed, 0)
    means = rng.standard_normal((n_clusters, d)) * mean_sd
    labels = rng.integers(0, n_clusters, size=n)
    x = np.empty((n, d), dtype=np.float32)
    order = np.argsort(labels, kind="stable")
    counts = np.bincount(labels, minlength=n_clusters)
    start = 0
    for c in range(n_clusters):
        idx = order[start:start + counts[c]]
        start += counts[c]
        z = _rng(seed, 1, c).standard_normal((len(idx), d))
        if anisotropic:
            crng = _rng(seed, 2, c)
            lam = np.exp(crng.uniform(np.log(0.01), 0.0, size=d))
            q, r = np.linalg.qr(crng.standard_normal((d, d)))
            q = q * np.sign(np.diag(r))[None, :]
            z = (z * np.sqrt(lam)[None, :]) @ q.T
        x[idx] = (means[c][None, :] + z).astype(np.float32)
    if return_labels:
        return x, labels
    return x


def sparse_quantized(seed: int, n: int, d: int, p_zero: float = 0.7) -> np.ndarray:
    """Entries are exactly 0 with probability p_zero, else float32(k)/float32(255) with
    k uniform on {1, ..., 255} (image-like data on a 1/255 grid)."""
    rng = _rng(seed, 0)
    out = np.empty((n, d), dtype=np.float32)
    step = 65536
    for s in range(0, n, step):
        e = min(n, s + step)
        k = rng.integers(1, 256, size=(e - s, d)).astype(np.float32)
        zero = rng.random((e - s, d)) < p_zero
        v = k / np.float32(255.0)
        v[zero] = 0.0
        out[s:e] = v
    return out


def mixture_queries(seed: int, x: np.ndarray, m: int, n_clusters: int, outlier_frac: float = 0.05,
                    mean_seed: int | None = None, mean_sd: float = 5.0) -> np.ndarray:
    """Queries for a served isotropic mixture: fresh draws from the same mixture (same means,
    regenerated from `mean_seed`), plus a fraction drawn uniformly in the bounding box of x."""
    d = x.shape[1]
    means = _rng(mean_seed, 0).standard_normal((n_clusters, d)) * mean_sd
    rng = _rng(seed, 0)
    lab = rng.integers(0, n_clusters, size=m)
    q = (means[lab] + rng.standard_normal((m, d))).astype(np.float32)
    n_out = int(round(outlier_frac * m))
    if n_out:
        lo, hi = x.min(axis=0), x.max(axis=0)
        pos = rng.choice(m, size=n_out, replace=False)
        q[pos] = rng.uniform(lo, hi, size=(n_out, d)).astype(np.float32)
    return q


@dataclass
class Workload:
    """One synthetic workload: data, (optional) queries and the forest parameters."""
    name: str
    x: np.ndarray
    n_trees: int
    leaf_size: int
    k: int
    n_try: int = 1
    dist_prec: str = "fp32"
    dir_seed: int = 0
    queries: np.ndarray | None = None
    meta: dict = field(default_factory=dict)


# The five workload shapes.  n, d, clusters, K, T and n0 follow the paper's data-set scale
# (Tables 1-2: n from hundreds to millions, d from 11 to about 10^4, T = 10..100 trees,
# small leaves) at sizes that exercise one MI355X.
CONFIGS = {
    1: dict(name="allknn_10k_d16_T4", n=10_000, d=16, clusters=10, k=10, T=4, n0=50, prec="fp32"),
    2: dict(name="allknn_1M_d128_T32", n=1_000_000, d=128, clusters=100, k=20, T=32, n0=256,
            prec="fp32", anisotropic=True),
    3: dict(name="allknn_1M_d784_T48_bf16", n=1_000_000, d=784, k=10, T=48, n0=512, prec="bf16"),
    4: dict(name="serve_4M_d96_T64_fp16", n=4_000_000, d=96, clusters=1000, k=10, T=64, n0=256,
            prec="fp16"),
}


def make_config(c: int, n: int | None = None) -> Workload:
    """Build workload c (optionally with fewer points, same recipe and seeds)."""
    cfg = CONFIGS[c]
    nn = cfg["n"] if n is None else n
    if c == 3:
        x = sparse_quantized(SEED_BASE + c, nn, cfg["d"])
    else:
        x = gaussian_mixture(SEED_BASE + c, nn, cfg["d"], cfg["clusters"],
                             anisotropic=cfg.get("anisotropic", False))
    return Workload(name=cfg["name"], x=x, n_trees=cfg["T"], leaf_size=cfg["n0"], k=cfg["k"],
                    dist_prec=cfg["prec"], dir_seed=SEED_BASE + 100 + c,
                    meta=dict(config=c, n=nn, d=cfg["d"]))


def batched_shapes(seed: int = SEED_BASE + 5, count: int = 512, n_lo: int = 2000, n_hi: int = 200_000,
                   dims=(8, 32, 64, 256)):
    """(n_i, d_i, clusters_i) of the uneven data sets: n log-uniform in [n_lo, n_hi], d from
    `dims`, 5..50 clusters."""
    rng = _rng(seed, 9)
    ns = np.round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count))).astype(np.int64)
    ds = rng.choice(np.asarray(dims), size=count)
    cs = rng.integers(5, 51, size=count)
    return [(int(ns[i]), int(ds[i]), int(cs[i])) for i in range(count)]


def batched_datasets(seed: int = SEED_BASE + 5, count: int = 512, n_lo: int = 2000,
                     n_hi: int = 200_000, dims=(8, 32, 64, 256), workers: int = 1):
    """Many uneven data sets (batched_shapes), each an isotropic unit-variance mixture with
    means ~ N(0, 25 I) from its own seed, so the result does not depend on `workers` (threads
    generating data sets side by side).  Returns a list of float32 arrays."""
    shapes = batched_shapes(seed, count, n_lo, n_hi, dims)

    def one(i):
        n, d, c = shapes[i]
        return gaussian_mixture(seed * 1000 + i, n, d, c)

    if workers <= 1:
        return [one(i) for i in range(count)]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(one, range(count)))


def serving_requests(seed: int, n_requests: int, rate_per_s: float, b_median: int = 64,
                     b_sigma: float = 1.5, b_max: int = 4096, ks=(1, 10, 100)):
    """Poisson arrivals at `rate_per_s`; batch sizes round(exp(N(ln b_median, b_sigma^2)))
    clipped to [1, b_max]; K uniform over `ks`.  Returns (arrival_s, sizes, ks)."""
    rng = _rng(seed, 3)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    sizes = np.clip(np.round(np.exp(rng.normal(np.log(b_median), b_sigma, size=n_requests))),
                    1, b_max).astype(np.int64)
    kk = rng.choice(np.asarray(ks), size=n_requests)
    return np.cumsum(gaps), sizes, kk
