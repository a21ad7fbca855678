"""Pins for the oracle's approximate similarities (Section 5; the degree
heuristic of Section 6.3): SimHash for cosine, k-partition MinHash for
Jaccard, with the random draws given as inputs.

* sketches worked by hand on tiny graphs;
* no edge approximated (degrees at most the threshold): the exact index;
* identical closed neighbourhoods give identical sketches, estimate 1;
* on a dense graph the estimates are unbiased: the mean angle (SimHash) and
  the mean Jaccard (MinHash) over the approximated edges match the exact ones.
"""

from __future__ import annotations

import math

import numpy as np
import pytest

import graphgen
import oracle


def test_simhash_sketch_hand_worked():
    # path 0 - 1 - 2, k = 4 directions with short dyadic coordinates (exact
    # sums). Dot products of N[v] with direction i, bit = (dot >= 0):
    #   N[0] = {0, 1}:    -2, 0, 1, 0        -> 0 1 1 1
    #   N[1] = {0, 1, 2}: -1, 1, -1, 0       -> 0 1 0 1
    #   N[2] = {1, 2}:    -2, 2, -3, -0.5    -> 0 1 0 0
    g = graphgen.from_edges(3, [(0, 1), (1, 2)])
    gauss = np.array([[1, -1, 2, 0.5], [-3, 1, -1, -0.5], [1, 1, -2, 0]], np.float64)
    bits = oracle.simhash_sketches(g, 4, gauss, [0, 1, 2])
    assert bits.tolist() == [[0, 1, 1, 1], [0, 1, 0, 1], [0, 1, 0, 0]]
    # weighted: w(0, 1) = w(1, 0) = 2 scales x = 1's term in N[0] and x = 0's in N[1]
    #   N[0]: 1 + 2(-3) = -5, -1 + 2 = 1, 2 - 2 = 0, 0.5 - 1 = -0.5   -> 0 1 1 0
    #   N[1]: 2(1) - 3 + 1 = 0, -2 + 1 + 1 = 0, 4 - 1 - 2 = 1, 1 - 0.5 = 0.5 -> 1 1 1 1
    w = np.array([2.0, 2.0, 1.0, 1.0])  # slots (0,1) (1,0) (1,2) (2,1)
    bits = oracle.simhash_sketches(g, 4, gauss, [0, 1], w)
    assert bits.tolist() == [[0, 1, 1, 0], [1, 1, 1, 1]]


def test_minhash_sketch_hand_worked():
    # n = 8, k = 4 bins of width 2: bin(x) = perm[x] // 2. Star 0-{1,2,3} and 4-5.
    #   N[0] = {0,1,2,3}: perm 5,2,7,0 -> bins 2,1,3,0 -> [0, 2, 5, 7]
    #   N[1] = {0,1}:     perm 5,2     -> [E, 2, 5, E]
    #   N[4] = {4,5}:     perm 3,6     -> [E, 3, E, 6]
    E = 0xFFFFFFFF
    g = graphgen.from_edges(8, [(0, 1), (0, 2), (0, 3), (4, 5)])
    perm = np.array([5, 2, 7, 0, 3, 6, 1, 4], np.uint32)
    sk = oracle.minhash_sketches(g, 4, perm, [0, 1, 4])
    assert sk.tolist() == [[0, 2, 5, 7], [E, 2, 5, E], [E, 3, E, 6]]


@pytest.mark.parametrize("kind,weighted", [(oracle.COSINE, False), (oracle.COSINE, True), (oracle.JACCARD, False)])
def test_below_threshold_is_exact(kind, weighted):
    g = graphgen.rmat(10, 8, seed=6)
    k = 64 * ((int(np.diff(g.off).max()) + 63) // 64)  # every degree <= k: nothing approximated
    gauss = graphgen.gaussians(g.n, k, 1) if kind == oracle.COSINE else None
    perm = graphgen.permutation(g.n, 1) if kind == oracle.JACCARD else None
    w = graphgen.edge_weights(g, 4) if weighted else None
    got = oracle.lsh_similarities(g, kind, k, gauss, perm, w)
    want = oracle.weighted_similarities(g, w) if weighted else oracle.similarities(g, kind)[1]
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_identical_neighbourhoods_estimate_one():
    n = 140  # K_n: every closed neighbourhood is V; degree 139 > 64 and 2*139 > 3*64
    g = graphgen.from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    s = oracle.lsh_similarities(g, oracle.COSINE, 64, gauss=graphgen.gaussians(n, 64, 3))
    assert np.all(s == 1.0)
    s = oracle.lsh_similarities(g, oracle.JACCARD, 64, perm=graphgen.permutation(n, 3))
    assert np.all(s == 1.0)


def planted_pair():
    """u = 0 and v = 1 adjacent; u also joined to 60 leaves A, v to 150
    leaves B, both to 100 leaves C. Only u and v are high degree, so only the
    edge {0, 1} is approximated. N[u] ∩ N[v] = {u, v} ∪ C (102), |N[u]| = 162,
    |N[v]| = 252, |N[u] ∪ N[v]| = 312."""
    A, B, C = range(2, 62), range(62, 212), range(212, 312)
    e = [(0, 1)] + [(0, x) for x in A] + [(1, x) for x in B] + [(0, x) for x in C] + [(1, x) for x in C]
    return graphgen.from_edges(312, e), 102 / math.sqrt(162 * 252), 102 / 312


def test_simhash_unbiased_angle():
    # P(a sketch bit differs) = theta / pi for each random direction, so over
    # independent draws the mean of h / k tends to theta / pi (Section 2.1.2).
    g, cos_exact, _ = planted_pair()
    k, seeds = 64, 200
    slot = int(g.off[0])  # (0, 1)
    fr = []
    for seed in range(seeds):
        s = oracle.lsh_similarities(g, oracle.COSINE, k, gauss=graphgen.gaussians(g.n, k, 1000 + seed))
        h = round(math.acos(min(1.0, s[slot])) * k / math.pi)
        assert s[slot] == math.cos(math.pi * h / k)  # the estimate is cos(pi h / k)
        fr.append(h / k)
        exact = oracle.similarities(g, oracle.COSINE)[1] if seed == 0 else exact
        rest = np.arange(g.nnz) != slot
        rest[g.off[1]] = False  # (1, 0) is the same edge
        assert np.array_equal(s[rest], exact[rest])
    theta = math.acos(cos_exact) / math.pi
    sd = math.sqrt(theta * (1 - theta) / k / seeds)
    assert abs(np.mean(fr) - theta) < 4 * sd


def test_minhash_unbiased_jaccard():
    # one-permutation hashing: matches / (k - jointly empty bins) is an
    # unbiased estimate of the Jaccard similarity over random permutations
    g, _, jac = planted_pair()
    k, seeds = 64, 200
    slot = int(g.off[0])
    est = [oracle.lsh_similarities(g, oracle.JACCARD, k, perm=graphgen.permutation(g.n, 2000 + s))[slot]
           for s in range(seeds)]
    sd = math.sqrt(jac * (1 - jac) / 40 / seeds)  # at least ~40 of the 64 bins are occupied here
    assert abs(np.mean(est) - jac) < 4 * sd
    assert all(0 <= x <= 1 for x in est)
