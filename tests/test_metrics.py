"""Pins of the accuracy measures of Sec. 5.1 -- the average missing rate m_K and the mean
K-th neighbour distance d_K -- with hand-worked values, for the package's implementation
(used by the benchmark) and the oracle's (used by the tests).  CPU only."""

import numpy as np
import pytest

import oracle
from paper_1812_11689_amd import metrics

IMPLS = [("package", metrics.missing_counts, metrics.missing_rate),
         ("oracle", oracle.missing_counts, oracle.missing_rate)]


@pytest.mark.parametrize("name,counts,rate", IMPLS, ids=[i[0] for i in IMPLS])
def test_hand_worked_missing_rate(name, counts, rate):
    true = np.array([[0, 1, 2], [5, 6, 7], [9, 3, 4]])
    found = np.array([[2, 1, 0],     # all three found, other order: m = 0
                      [5, 8, -1],    # 6 and 7 missed (-1 padding matches nothing): m = 2
                      [4, 4, 9]])    # 3 missed, 4 twice counts once: m = 1
    assert list(counts(found, true)) == [0, 2, 1]
    assert rate(found, true) == pytest.approx(3 / 9)   # (0 + 2 + 1) / (n K), n = 3, K = 3
    # a found list longer than K: membership only
    assert list(counts(np.array([[7, 0, 3, 1]]), np.array([[0, 1]]))) == [0]
    # nothing found
    assert rate(np.full((2, 2), -1), np.array([[0, 1], [2, 3]])) == 1.0


@pytest.mark.parametrize("name,counts,rate", IMPLS, ids=[i[0] for i in IMPLS])
def test_duplicate_rows_count_by_index(name, counts, rate):
    # points 0 and 1 coincide; query point 2 at distance 1 from both, 4 from point 3.  The
    # true nearest neighbour by (distance, index) is 0: finding 1 instead is a miss by the
    # definition (neighbours are points, not distances) while the K-th distance is exact
    x = np.array([[0.0], [0.0], [1.0], [3.0]], np.float32)
    ti, td = oracle.bruteforce(x, x[2:3], 1, np.array([2]))
    assert ti.tolist() == [[0]] and td.tolist() == [[1.0]]
    found_i, found_d = np.array([[1]]), np.array([[1.0]])
    assert list(counts(found_i, ti)) == [1] and rate(found_i, ti) == 1.0
    assert metrics.kth_distance_excess(found_d, td) == 0.0


def test_kth_distance_measures():
    true_d = np.array([[1.0, 2.0], [0.5, 4.0]])
    found_d = np.array([[1.0, 3.0], [0.5, 4.0]])   # row 0 missed its 2nd neighbour
    assert metrics.mean_kth_distance(true_d) == 3.0    # (2 + 4) / 2
    assert metrics.mean_kth_distance(found_d) == 3.5   # (3 + 4) / 2
    assert metrics.kth_distance_excess(found_d, true_d) == pytest.approx(3.5 / 3.0 - 1.0)
    assert metrics.recall(np.array([[0, 9]]), np.array([[0, 1]])) == 0.5


def test_package_equals_oracle_on_random_lists():
    rng = np.random.default_rng(5)
    true = np.stack([rng.choice(1000, 10, replace=False) for _ in range(300)])
    found = np.where(rng.random((300, 10)) < 0.8, true, rng.integers(-1, 1000, (300, 10)))
    found = np.take_along_axis(found, rng.permuted(np.tile(np.arange(10), (300, 1)), axis=1), axis=1)
    assert np.array_equal(metrics.missing_counts(found, true), oracle.missing_counts(found, true))
    assert metrics.missing_rate(found, true) == oracle.missing_rate(found, true)
