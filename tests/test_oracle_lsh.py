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


# --------------------------------------------------------------------------
# The per-edge entry point (the checker of sampled GPU parity on large
# graphs) against the full pass, and both against hand-worked estimates.


def two_stars(d: int):
    """u = 0 joined to 1..d-1 and to the leaves 2..d, v = 1 joined to 0 and to
    d+1..2d-1: deg(0) = deg(1) = d; N[0] = {0..d}, N[1] = {0, 1, d+1..2d-1};
    n = 2d. Only the edge {0, 1} joins two vertices of degree d."""
    e = [(0, 1)] + [(0, x) for x in range(2, d + 1)] + [(1, x) for x in range(d + 1, 2 * d)]
    return graphgen.from_edges(2 * d, e)


def test_simhash_approximated_edge_hand_worked():
    # k = 4 directions, d = 5 > k: {0, 1} is approximated, every other edge
    # (a leaf, degree 1) is exact. N[0] = {0..5}, N[1] = {0, 1, 6..9}.
    #   direction 0: all +1                      -> both dots 6        -> 1, 1
    #   direction 1: -1 on 2..5, +1/2 elsewhere  -> N[0]: 1 - 4 = -3    -> 0
    #                                               N[1]: 6 * 1/2 = 3   -> 1
    #   direction 2: all -1                      -> both -6            -> 0, 0
    #   direction 3: all 0                       -> both 0 (>= 0)      -> 1, 1
    # h = 1 differing bit: the estimate is cos(pi / 4).
    g = two_stars(5)
    gauss = np.zeros((10, 4))
    gauss[:, 0] = 1.0
    gauss[:, 1] = 0.5
    gauss[2:6, 1] = -1.0
    gauss[:, 2] = -1.0
    assert oracle.simhash_sketches(g, 4, gauss, [0, 1]).tolist() == [[1, 0, 0, 1], [1, 1, 0, 1]]
    want = math.cos(math.pi / 4)
    full = oracle.lsh_similarities(g, oracle.COSINE, 4, gauss=gauss)
    s01, s10 = int(g.off[0]), int(g.off[1])  # slots (0, 1) and (1, 0)
    assert full[s01] == want and full[s10] == want
    assert oracle.lsh_edge_similarities(g, oracle.COSINE, 4, [0, 1], [1, 0], gauss=gauss).tolist() == [want, want]
    # the leaf edges keep their exact cosine: c = 2, a = 6 and 2
    leaf = oracle.lsh_edge_similarities(g, oracle.COSINE, 4, [0], [2], gauss=gauss)[0]
    assert leaf == 2 / math.sqrt(12) and full[int(g.off[0]) + 1] == leaf
    # weighted, w(0, 1) = w(1, 0) = 2: direction 1 gives N[0]: 1/2 + 2/2 - 4 =
    # -2.5 -> 0 and N[1]: 2/2 + 1/2 + 2 = 3.5 -> 1; the other bits are unchanged
    w = np.ones(g.nnz)
    w[s01] = w[s10] = 2.0
    for kind in (oracle.COSINE, oracle.WEIGHTED_COSINE):
        fw = oracle.lsh_similarities(g, kind, 4, gauss=gauss, w=w)
        assert fw[s01] == want
        assert oracle.lsh_edge_similarities(g, kind, 4, [1], [0], gauss=gauss, w=w)[0] == want


def test_minhash_approximated_edge_hand_worked():
    # k = 4 bins, d = 7 > 3k/2 = 6: {0, 1} is approximated. n = 14, perm = the
    # identity, bin(x) = floor(4x / 14): x 0..3 -> 0, 4..6 -> 1, 7..10 -> 2,
    # 11..13 -> 3. N[0] = {0..7} -> [0, 4, 7, E]; N[1] = {0, 1, 8..13} ->
    # [0, E, 8, 11]. One match (bin 0), no bin empty in both: 1/4.
    E = 0xFFFFFFFF
    g = two_stars(7)
    perm = np.arange(14, dtype=np.uint32)
    assert oracle.minhash_sketches(g, 4, perm, [0, 1]).tolist() == [[0, 4, 7, E], [0, E, 8, 11]]
    full = oracle.lsh_similarities(g, oracle.JACCARD, 4, perm=perm)
    assert full[int(g.off[0])] == 0.25 and full[int(g.off[1])] == 0.25
    assert oracle.lsh_edge_similarities(g, oracle.JACCARD, 4, [0, 1], [1, 0], perm=perm).tolist() == [0.25, 0.25]
    # a leaf edge keeps the exact Jaccard: c = 2, a = 8 and 2 -> 2 / 8
    assert oracle.lsh_edge_similarities(g, oracle.JACCARD, 4, [0], [3], perm=perm)[0] == 0.25
    assert full[int(g.off[0]) + 2] == 0.25


LSH_CASES = [("simhash", oracle.COSINE, False), ("simhash_weighted", oracle.COSINE, True),
             ("simhash_weighted_kind", oracle.WEIGHTED_COSINE, True), ("minhash", oracle.JACCARD, False)]


@pytest.mark.parametrize("name,kind,weighted", LSH_CASES)
@pytest.mark.parametrize("gname", ["rmat10", "rmat11"])
def test_edge_function_equals_full_pass(name, kind, weighted, gname):
    # Every slot of graphs holding both approximated edges (two endpoints above
    # the threshold) and exact ones: the per-edge function must return the
    # full pass's value bit for bit.
    if gname == "rmat10":
        g, k = graphgen.rmat(10, 8, seed=6), 64
    else:
        g, k = graphgen.rmat(11, 16, seed=8), 128
    gauss = graphgen.gaussians(g.n, k, 31) if kind != oracle.JACCARD else None
    perm = graphgen.permutation(g.n, 31) if kind == oracle.JACCARD else None
    w = graphgen.edge_weights(g, 32) if weighted else None
    full = oracle.lsh_similarities(g, kind, k, gauss, perm, w, threads=4)
    rows = np.repeat(np.arange(g.n), np.diff(g.off))
    per_edge = oracle.lsh_edge_similarities(g, kind, k, rows, g.adj, gauss, perm, w)
    assert np.array_equal(full.view(np.uint64), per_edge.view(np.uint64))
    deg = np.diff(g.off)
    thr = (lambda d: 2 * d > 3 * k) if kind == oracle.JACCARD else (lambda d: d > k)
    approx = thr(deg[rows]) & thr(deg[g.adj])
    assert approx.any() and (~approx).any()  # both kinds of edges are covered
    # the exact edges equal the exact index of the same kind
    exact = (oracle.weighted_similarities(g, w) if weighted
             else oracle.similarities(g, oracle.JACCARD if kind == oracle.JACCARD else oracle.COSINE)[1])
    assert np.array_equal(full[~approx].view(np.uint64), exact[~approx].view(np.uint64))


def test_lsh_inputs_rejected():
    g = two_stars(5)
    gauss = np.zeros((10, 4))
    with pytest.raises(ValueError):
        oracle.lsh_similarities(g, 7, 4, gauss=gauss)  # unknown kind
    with pytest.raises(ValueError):
        oracle.lsh_similarities(g, oracle.WEIGHTED_COSINE, 4, gauss=gauss)  # no weights
    with pytest.raises(ValueError):
        oracle.lsh_edge_similarities(g, oracle.COSINE, 4, [0], [1], gauss=gauss[:9])  # short draws
    with pytest.raises(ValueError):
        oracle.lsh_similarities(g, oracle.JACCARD, 4)  # no permutation
    with pytest.raises(ValueError):
        oracle.lsh_similarities(g, oracle.JACCARD, 4, perm=np.full(10, 10, np.uint32))  # values >= n


def test_build_index_lsh_composes_the_orders():
    # the approximate index is Algorithm 2's orders over the LSH similarities
    g, k = graphgen.rmat(10, 8, seed=6), 64
    perm = graphgen.permutation(g.n, 9)
    ix = oracle.build_index_lsh(g, oracle.JACCARD, k, perm=perm)
    sim = oracle.lsh_similarities(g, oracle.JACCARD, k, perm=perm)
    assert np.array_equal(ix.sim.view(np.uint64), sim.view(np.uint64))
    no_ids, no_sim = oracle.neighbor_order(g, sim)
    assert np.array_equal(ix.no_ids, no_ids) and np.array_equal(ix.no_sim.view(np.uint64), no_sim.view(np.uint64))
    co_off, co_ids, co_thr = oracle.core_order(g, no_sim, ix.dmax)
    assert np.array_equal(ix.co_off, co_off) and np.array_equal(ix.co_ids, co_ids)
    for v in range(0, g.n, 97):
        a, b = int(g.off[v]), int(g.off[v + 1])
        ids, sims = oracle.neighbor_order_row(g.adj[a:b], sim[a:b])
        assert np.array_equal(ids, ix.no_ids[a:b])
