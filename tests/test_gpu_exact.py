"""GPU parity of the exact brute-force kNN (rpf_exact_knn, the ground truth of the accuracy
measures of Sec. 5.1) against the oracle's brute force: indices bit-exact (ties broken by
index under the binary64 ranking), distances within 1e-5 relative.  Cases: the register and
the streaming distance kernels (d <= 256 with d % 4 == 0, and otherwise), two query chunks,
K from 1 to 256, a left-out own point, padding when fewer than K candidates remain, mass
ties wider than the select's gather (3000 copies of one point), and wide exponents."""

import numpy as np
import pytest
import torch

import oracle
from tests.helpers import problem

pytestmark = pytest.mark.gpu

CASES = [
    # name, n, d, m, K, kind, dup_every, self
    ("mixture_d16_self", 5000, 16, 300, 10, "mixture", 0, True),
    ("scalar_d33_queries", 3000, 33, 200, 7, "mixture", 0, False),
    ("aniso_d128_self", 4000, 128, 500, 20, "aniso", 0, True),
    ("quant_d784_stream", 2000, 784, 100, 10, "quant", 0, True),
    ("two_chunks", 300_000, 16, 2000, 12, "mixture", 0, True),
    ("k256", 3000, 24, 64, 256, "mixture", 0, True),
    ("k1", 3000, 24, 64, 1, "mixture", 0, False),
    ("pad_k_above_n", 40, 3, 40, 60, "mixture", 0, True),
    ("duplicates", 6000, 8, 300, 8, "mixture", 5, True),
    ("mass_ties", 6000, 8, 200, 16, "mixture", 2, True),
    ("wide_exponents", 3000, 24, 150, 6, "wide", 0, True),
    ("d64_two_steps", 5000, 64, 200, 16, "mixture", 0, True),
    ("d256_eight_steps", 3000, 256, 130, 16, "aniso", 0, True),
    ("d8_one_step", 6000, 8, 300, 16, "mixture", 0, True),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_exact_knn_matches_oracle(case):
    from paper_1812_11689_amd import rpf
    name, n, d, m, K, kind, dup, use_self = case
    print(f"[exact] {name} n={n} d={d} m={m} K={K}", flush=True)
    x, _ = problem(n, d, 1, n, seed=len(name) + 400, kind=kind, dup_every=dup)
    rng = np.random.default_rng(len(name))
    if use_self:
        pts = np.sort(rng.choice(n, size=m, replace=False))
        if dup:
            pts[0] = 0  # a query on the repeated point
        q = x[pts]
        ri, rd = oracle.bruteforce(x, q, K, pts)
        sidx = torch.from_numpy(pts.astype(np.int64)).cuda()
    else:
        q, _ = problem(m, d, 1, m, seed=len(name) + 500, kind=kind)
        ri, rd = oracle.bruteforce(x, q, K)
        sidx = None
    gi, gd = rpf.exact_knn(torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda(), K, sidx)
    torch.cuda.synchronize()
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    np.testing.assert_array_equal(gi, ri)
    fin = np.isfinite(rd)
    assert np.array_equal(np.isfinite(gd), fin)
    np.testing.assert_allclose(gd[fin], rd[fin], rtol=1e-5, atol=0)
