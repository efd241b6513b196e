"""Shared helpers of the test suite: seeded problem instances fed identically to the
oracle and to the HIP library."""

import numpy as np

from paper_1812_11689_amd import workloads as W


def heap_count(n, n0):
    L = 0
    while -(-n // (1 << L)) > n0:
        L += 1
    return (1 << L) - 1


def problem(n, d, T, n0, n_try=1, seed=1, clusters=5, kind="mixture", dup_every=0):
    if kind == "mixture":
        x = W.gaussian_mixture(seed, n, d, clusters)
    elif kind == "aniso":
        x = W.gaussian_mixture(seed, n, d, clusters, anisotropic=True)
    elif kind == "quant":
        x = W.sparse_quantized(seed, n, d)
    elif kind == "wide":  # exponent spread of 2^+-40 and signed zeros
        rng = np.random.default_rng(seed)
        x = (rng.standard_normal((n, d)) * np.exp2(rng.integers(-40, 40, (n, d)))).astype(np.float32)
        x[rng.random((n, d)) < 0.05] = -0.0
    else:
        raise ValueError(kind)
    if dup_every:
        x[1::dup_every] = x[0]
    R = W.directions(seed + 1000, T, heap_count(n, n0), n_try, d)
    return x, R
