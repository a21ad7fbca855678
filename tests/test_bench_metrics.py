"""Host-side metrics of bench.py: the adjusted Rand index of Section 7.2
(unclustered vertices as clusters of their own), pinned against a hand-worked
contingency table and scikit-learn's implementation."""

import numpy as np
import pytest

import bench


def test_ari_hand_worked():
    # C = {0,1,2} {3,4} ; G = {0,1} {2,3,4}; n = 5, C(5,2) = 10
    # n_ij: (C1,G1)=2, (C1,G2)=1, (C2,G2)=2 -> sum C(n_ij,2) = 1 + 0 + 1 = 2
    # rows 3, 2 -> 3 + 1 = 4; columns 2, 3 -> 1 + 3 = 4; expected 4*4/10 = 1.6
    # ARI = (2 - 1.6) / ((4 + 4)/2 - 1.6) = 0.4 / 2.4 = 1/6
    a = np.array([0, 0, 0, 3, 3])
    b = np.array([0, 0, 2, 2, 2])
    assert bench.adjusted_rand_index(a, b) == pytest.approx(1 / 6, abs=1e-15)
    assert bench.adjusted_rand_index(a, a) == 1.0
    # -1 entries are singletons: all unclustered on both sides is identical
    assert bench.adjusted_rand_index(np.full(4, -1), np.full(4, -1)) == 1.0


def test_ari_matches_sklearn():
    metrics = pytest.importorskip("sklearn.metrics")
    rng = np.random.default_rng(3)
    for n, k in [(50, 3), (400, 20), (2000, 200)]:
        a = rng.integers(-1, k, n)
        b = np.where(rng.random(n) < 0.7, a, rng.integers(-1, k, n))
        la, lb = bench._labels(a), bench._labels(b)
        assert bench.adjusted_rand_index(a, b) == pytest.approx(metrics.adjusted_rand_score(la, lb), abs=1e-12)
