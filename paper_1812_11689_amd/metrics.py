"""Accuracy measures of a kNN search (Sec. 5.1): the average missing rate and the average
k-th nearest neighbour distance.  Host logic on index and distance arrays, used by the
benchmark to report recall; none of the search's arithmetic lives here.

  m(i)   = number of the true K nearest neighbours of point i that the search missed
           (|TrueK(i) minus Found(i)|, as sets of point indices; -1 padding in Found
           matches nothing);
  m_K    = (1 / (n K)) sum_i m(i);            recall = 1 - m_K;
  d_K    = (1 / n) sum_i d_K(i), the mean distance to the K-th neighbour found; the search
           never finds a K-th distance below the true one (Sec. 5.1), so the ratio
           d_K(search) / d_K(exact) - 1 is >= 0.
"""

from __future__ import annotations

import numpy as np


def missing_counts(found_idx, true_idx) -> np.ndarray:
    """m(i) per row: entries of true_idx[i] (K distinct indices) absent from found_idx[i]."""
    found = np.asarray(found_idx, dtype=np.int64)
    true = np.asarray(true_idx, dtype=np.int64)
    if found.ndim != 2 or true.ndim != 2 or found.shape[0] != true.shape[0]:
        raise ValueError("found_idx and true_idx must be [n][*] arrays with the same rows")
    n, K = true.shape
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    # sort each found row, then look every true index up in its row
    fs = np.sort(found, axis=1)
    miss = np.empty(n, dtype=np.int64)
    for i in range(n):
        pos = np.searchsorted(fs[i], true[i])
        hit = (pos < fs.shape[1]) & (fs[i][np.minimum(pos, fs.shape[1] - 1)] == true[i])
        miss[i] = K - int(hit.sum())
    return miss


def missing_rate(found_idx, true_idx) -> float:
    """m_K = sum_i m(i) / (n K) (Sec. 5.1)."""
    true = np.asarray(true_idx)
    if true.size == 0:
        return 0.0
    return float(missing_counts(found_idx, true).sum()) / float(true.size)


def recall(found_idx, true_idx) -> float:
    """1 - m_K: the fraction of the true K nearest neighbours found."""
    return 1.0 - missing_rate(found_idx, true_idx)


def mean_kth_distance(dist) -> float:
    """d_K = mean over rows of the K-th (last) distance of each row (Sec. 5.1)."""
    d = np.asarray(dist, dtype=np.float64)
    return float(d[:, -1].mean()) if d.size else 0.0


def kth_distance_excess(found_dist, true_dist) -> float:
    """d_K(search) / d_K(exact) - 1 over the same rows (0 when nothing is missed)."""
    return mean_kth_distance(found_dist) / mean_kth_distance(true_dist) - 1.0
