"""Pins for the oracle's weighted cosine (Section 3.1, the measure Algorithm 1
is written for): w(x, x) = 1, sums over closed neighbourhoods taken term by
term in ascending vertex id, similarity = dot / sqrt(S_u * S_v).

* a hand-worked fixture (tests/golden/weighted_hand.txt);
* reduction to the unweighted cosine with unit weights (pinned separately);
* closed forms on K2 and stars;
* a graph whose result depends on the summation order;
* brute force from the definition with dyadic weights (exact sums);
* the exact real value within the rounding bound, for full-mantissa weights.
"""

from __future__ import annotations

import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
getcontext().prec = 80


def weighted_graph(n, wedges):
    """(graph, weights per CSR slot) from (u, v, w) undirected edges."""
    g = graphgen.from_edges(n, [(u, v) for u, v, _ in wedges])
    wmap = {(min(u, v), max(u, v)): w for u, v, w in wedges}
    return g, slot_weights(g, wmap)


def slot_weights(g, wmap):
    w = np.zeros(g.nnz, np.float64)
    for u in range(g.n):
        for s in range(int(g.off[u]), int(g.off[u + 1])):
            v = int(g.adj[s])
            w[s] = wmap[(min(u, v), max(u, v))]
    return w


def closed(g, w, v):
    """N[v] as {x: w(v, x)} with w(v, v) = 1, written from the definition."""
    d = {int(g.adj[s]): float(w[s]) for s in range(int(g.off[v]), int(g.off[v + 1]))}
    d[v] = 1.0
    return d


def test_hand_worked():
    path = os.path.join(GOLDEN, "weighted_hand.txt")
    lines = [ln.split("#")[0].strip() for ln in open(path)]
    lines = [ln for ln in lines if ln]
    n = int(lines[0])
    wedges = [(int(a), int(b), float(c)) for a, b, c in (ln.split() for ln in lines[1:])]
    g, w = weighted_graph(n, wedges)
    sim = oracle.weighted_similarities(g, w)
    checks = 0
    for ln in open(path):
        if not ln.startswith("#!"):
            continue
        f = ln[2:].split()
        if f[0] == "sigma":
            u, v = int(f[1]), int(f[2])
            want = eval(f[3], {"sqrt": math.sqrt})
            assert oracle.weighted_edge_similarity(g, w, u, v) == want, ln
            for a, b in ((u, v), (v, u)):
                row = g.adj[g.off[a]:g.off[a + 1]]
                assert sim[g.off[a] + int(np.searchsorted(row, b))] == want, ln
        else:
            assert oracle.weighted_square_sum(g, w, int(f[1])) == float(f[2]), ln
        checks += 1
    assert checks == 8


@pytest.mark.parametrize("which", ["rmat10", "sbm", "tiny"])
def test_unit_weights_are_the_unweighted_cosine(which):
    if which == "rmat10":
        gs = [graphgen.rmat(10, 8, seed=5)]
    elif which == "sbm":
        gs = [graphgen.sbm(300, 6, 0.2, 0.01, seed=3)]
    else:
        gs = list(graphgen.tiny_graphs(5))
    for g in gs:
        ones = np.ones(g.nnz)
        _, cos = oracle.similarities(g, oracle.COSINE)
        assert np.array_equal(oracle.weighted_similarities(g, ones).view(np.uint64), cos.view(np.uint64))
        a = oracle.build_index_weighted(g, ones)
        b = oracle.build_index(g, oracle.COSINE)
        for f in ("no_ids", "no_sim", "co_off", "co_ids", "co_thr"):
            assert np.array_equal(getattr(a, f), getattr(b, f)), f


@pytest.mark.parametrize("x", [2.0, 0.5, 0.25, 3.0, 1.0])
def test_k2_closed_form(x):
    # N[0] = {0:1, 1:x}, N[1] = {0:x, 1:1}: dot 2x, S = 1 + x^2 on both sides
    g, w = weighted_graph(2, [(0, 1, x)])
    assert oracle.weighted_edge_similarity(g, w, 0, 1) == 2 * x / (1 + x * x)


def test_star_closed_form():
    # centre 0, leaves i with weights x_i: N[0] ∩ N[i] = {0, i}, dot = 2 x_i,
    # S_0 = 1 + sum x^2, S_i = 1 + x_i^2 (all short dyadics: exact)
    xs = [0.5, 1.0, 1.5, 2.0, 0.25]
    g, w = weighted_graph(6, [(0, i + 1, x) for i, x in enumerate(xs)])
    s0 = 1 + sum(x * x for x in xs)
    for i, x in enumerate(xs):
        assert oracle.weighted_edge_similarity(g, w, 0, i + 1) == 2 * x / math.sqrt(s0 * (1 + x * x))


def test_summation_order_is_ascending_id():
    # Edge {1, 2} with common neighbours 0 and 3. In ascending x the dot terms
    # are 1 (x=0), 2^-53 (x=1), 2^-53 (x=2), 2^-54 (x=3): each small term is
    # at most half an ulp of the running sum 1 and ties go to even, so the dot
    # is exactly 1; both square sums are exactly 2, and sigma = 1/2. Summed
    # in descending x the small terms first reach 2^-52 + 2^-54 and the dot
    # becomes 1 + 2^-52.
    e, h = 2.0 ** -53, 2.0 ** -27
    g, w = weighted_graph(4, [(0, 1, 1.0), (0, 2, 1.0), (1, 2, e), (1, 3, h), (2, 3, h)])
    assert oracle.weighted_square_sum(g, w, 1) == 2.0
    assert oracle.weighted_square_sum(g, w, 2) == 2.0
    assert oracle.weighted_edge_similarity(g, w, 1, 2) == 0.5
    terms = [1.0, e, e, h * h]
    desc = 0.0
    for t in reversed(terms):
        desc += t
    assert desc != 1.0  # the other order gives another result


def test_brute_force_dyadic():
    # Dyadic weights k/8: every product and sum is exact, so the definition
    # evaluated with fractions fixes the dot and the square sums exactly.
    for seed in range(12):
        g = graphgen.random_graph(9, 0.45, seed)
        if g.nnz == 0:
            continue
        wmap = {}
        for u in range(g.n):
            for s in range(int(g.off[u]), int(g.off[u + 1])):
                v = int(g.adj[s])
                wmap[(min(u, v), max(u, v))] = (1 + graphgen.draw(seed, min(u, v) * 16 + max(u, v)) % 16) / 8
        w = slot_weights(g, wmap)
        sim = oracle.weighted_similarities(g, w)
        for u in range(g.n):
            nu = closed(g, w, u)
            su = sum(Fraction(x) ** 2 for x in nu.values())
            for s in range(int(g.off[u]), int(g.off[u + 1])):
                v = int(g.adj[s])
                nv = closed(g, w, v)
                sv = sum(Fraction(x) ** 2 for x in nv.values())
                dot = sum(Fraction(nu[x]) * Fraction(nv[x]) for x in set(nu) & set(nv))
                assert float(dot) == dot and float(su) * float(sv) == su * sv
                assert sim[s] == float(dot) / math.sqrt(float(su * sv)), (seed, u, v)


def test_within_rounding_bound_of_the_real_value():
    # Full-mantissa positive weights: the FP64 result is within gamma_{k+4}
    # (relative, k = terms of the longest sum) of the exact real value.
    g = graphgen.rmat(9, 8, seed=11)
    w = graphgen.edge_weights(g, 5)
    sim = oracle.weighted_similarities(g, w)
    u_round = 2.0 ** -53
    rng = np.random.default_rng(0)
    for s in rng.choice(g.nnz, 300, replace=False).tolist():
        u = int(np.searchsorted(g.off, s, side="right") - 1)
        v = int(g.adj[s])
        nu, nv = closed(g, w, u), closed(g, w, v)
        dot = sum(Fraction(nu[x]) * Fraction(nv[x]) for x in set(nu) & set(nv))
        su = sum(Fraction(x) ** 2 for x in nu.values())
        sv = sum(Fraction(x) ** 2 for x in nv.values())
        exact = Decimal(dot.numerator) / Decimal(dot.denominator) / (
            Decimal((su * sv).numerator) / Decimal((su * sv).denominator)).sqrt()
        k = max(len(nu), len(nv)) + 4
        gamma = k * u_round / (1 - k * u_round)
        assert abs(Decimal(sim[s]) - exact) <= Decimal(gamma) * exact, (u, v)
        assert 0 < sim[s] <= 1.0 + 4 * u_round


def test_symmetric_slots_and_range():
    g = graphgen.sbm(400, 8, 0.15, 0.01, seed=9)
    w = graphgen.edge_weights(g, 3)
    sim = oracle.weighted_similarities(g, w, threads=4)
    for u in range(g.n):
        for s in range(int(g.off[u]), int(g.off[u + 1])):
            v = int(g.adj[s])
            row = g.adj[g.off[v]:g.off[v + 1]]
            assert sim[g.off[v] + int(np.searchsorted(row, u))] == sim[s]
    assert sim.min() > 0 and sim.max() <= 1.0


def test_weighted_edge_function_equals_full_pass():
    # the per-edge entry point (sampled checks on R-MAT-20) against the full
    # pass at every slot, with full-mantissa and asymmetric weights
    g = graphgen.rmat(10, 8, seed=12)
    w = graphgen.edge_weights(g, 5)
    w = w * np.where(np.arange(g.nnz) % 3 == 0, 0.75, 1.0)  # the two directions differ on some edges
    full = oracle.weighted_similarities(g, w, threads=4)
    rows = np.repeat(np.arange(g.n), np.diff(g.off))
    per_edge = oracle.weighted_edge_similarities(g, w, rows, g.adj.astype(np.int64))
    assert np.array_equal(full.view(np.uint64), per_edge.view(np.uint64))
