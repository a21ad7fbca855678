"""Pins for the CPU oracle against facts fixed outside it.

* hand-worked tiny graphs and closed forms (counts, both orders, queries);
* the paper's worked example and a graph consistent with its Figure 1-3
  captions;
* similarity values within the rounding bound of the exact real value;
* invariants (symmetry, range, twins, triangle identity, dense-matrix counts,
  order invariants);
* brute force: index queries equal a direct SCAN written from the definitions
  of Section 3.1, over every distinct (mu, eps) outcome.
"""

from __future__ import annotations

import json
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import brute_scan
import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
getcontext().prec = 60


def slot_of(g, u, v):
    row = g.adj[g.off[u]:g.off[u + 1]]
    k = int(np.searchsorted(row, v))
    assert row[k] == v
    return int(g.off[u]) + k


def exact_cosine(c, a, b):
    return Decimal(int(c)) / (Decimal(int(a)) * Decimal(int(b))).sqrt()


def within_ulps(x: float, exact: Decimal, ulps: float) -> bool:
    return abs(Decimal(x) - exact) <= Decimal(ulps) * Decimal(math.ulp(x))


# --------------------------------------------------------------------------
# Hand-worked graphs


HAND = json.load(open(os.path.join(GOLDEN, "tiny_hand.json")))["graphs"]


@pytest.mark.parametrize("name", sorted(HAND))
@pytest.mark.parametrize("kind", [oracle.COSINE, oracle.JACCARD])
def test_hand_counts_and_similarities(name, kind):
    h = HAND[name]
    g = graphgen.from_edges(h["n"], h["edges"])
    counts, sim = oracle.similarities(g, kind)
    deg = g.degrees()
    for key, c in h["c"].items():
        u, v = map(int, key.split("-"))
        for s in (slot_of(g, u, v), slot_of(g, v, u)):
            assert counts[s] == c
            a, b = deg[u] + 1, deg[v] + 1
            if kind == oracle.COSINE:
                assert within_ulps(sim[s], exact_cosine(c, a, b), 2)
            else:
                assert within_ulps(sim[s], Decimal(int(c)) / Decimal(int(a + b - c)), 0.5)
    for key, val in h.get("cos" if kind == oracle.COSINE else "jac", {}).items():
        u, v = map(int, key.split("-"))
        assert sim[slot_of(g, u, v)] == val


@pytest.mark.parametrize("name", sorted(HAND))
def test_hand_orders_and_queries(name):
    h = HAND[name]
    g = graphgen.from_edges(h["n"], h["edges"])
    ix = oracle.build_index(g, oracle.COSINE)
    for v, row in enumerate(h["no"]):
        assert ix.no_ids[ix.off[v]:ix.off[v + 1]].tolist() == row
    assert len(ix.co_off) == ix.dmax + 3
    for mu, seg in h["co"].items():
        mu = int(mu)
        assert ix.co_ids[ix.co_off[mu]:ix.co_off[mu + 1]].tolist() == seg
    for mu, eps, memb in h["queries"]:
        assert oracle.query(ix, mu, eps)[0].tolist() == memb, (mu, eps)


def load_edge_fixture(path):
    lines = [ln.split("#")[0].strip() for ln in open(path)]
    lines = [ln for ln in lines if ln]
    n = int(lines[0])
    edges = [tuple(map(int, ln.split())) for ln in lines[1:]]
    return graphgen.from_edges(n, edges)


def test_paper_worked_example_and_captions():
    g = load_edge_fixture(os.path.join(GOLDEN, "fig1_consistent.txt"))
    ix = oracle.build_index(g, oracle.COSINE)
    # Section 3.1: sigma(5,6) = |{5,6}| / (sqrt 3 sqrt 4) = 2/sqrt(12) ~ .58.
    c, s = oracle.edge_similarity(g, 5, 6)
    assert c == 2 and round(s, 2) == 0.58 and within_ulps(s, exact_cosine(2, 3, 4), 2)
    # Figure 2 caption: vertex 2 appears in NO[3] with similarity ~ .87.
    row = list(zip(ix.no_ids[ix.off[3]:ix.off[4]], ix.no_sim[ix.off[3]:ix.off[4]]))
    assert any(w == 2 and round(x, 2) == 0.87 for w, x in row)
    # Figure 3 caption: vertex 6's core threshold for mu = 2 is .75.
    seg = slice(ix.co_off[2], ix.co_off[3])
    thr6 = dict(zip(ix.co_ids[seg].tolist(), ix.co_thr[seg].tolist()))[6]
    assert thr6 == 0.75
    # Section 3.2: CO[3] holds exactly the nine vertices 1..9.
    assert sorted(ix.co_ids[ix.co_off[3]:ix.co_off[4]].tolist()) == list(range(1, 10))
    # Figure 1 caption at (mu, eps) = (3, .6): clusters {1,2,3,4} and
    # {6,7,8,11}; 5, 9, 10 unclustered; 11 is a border (clustered, not a core).
    memb, core = oracle.query(ix, 3, 0.6)
    clusters = {}
    for v, m in enumerate(memb.tolist()):
        if m >= 0:
            clusters.setdefault(m, set()).add(v)
    assert sorted(map(sorted, clusters.values())) == [[1, 2, 3, 4], [6, 7, 8, 11]]
    assert memb[5] == memb[9] == memb[10] == -1
    assert memb[11] >= 0 and core[11] == 0
    # The same caption: the unclustered 5 is a hub, 9 and 10 are outliers
    # (Section 2 definitions; Section 4.3 computes them).
    roles = oracle.roles(g, memb)
    assert roles[5] == oracle.ROLE_HUB and roles[9] == roles[10] == oracle.ROLE_OUTLIER
    assert all(roles[v] == oracle.ROLE_CLUSTERED for v in (1, 2, 3, 4, 6, 7, 8, 11))


def load_expectations(path):
    """The '#!' lines of a fixture: (mu, eps, memberships, roles)."""
    out = []
    for ln in open(path):
        if ln.startswith("#!"):
            left, right = ln[2:].split("|")
            f = left.split()
            out.append((int(f[0]), float(f[1]), [int(x) for x in f[2:]], [int(x) for x in right.split()]))
    return out


def test_hub_outlier_hand_worked():
    path = os.path.join(GOLDEN, "hub_outlier_hand.txt")
    g = load_edge_fixture(path)
    ix = oracle.build_index(g, oracle.COSINE)
    cases = load_expectations(path)
    assert len(cases) == 3
    for mu, eps, want_memb, want_roles in cases:
        memb, _ = oracle.query(ix, mu, eps)
        assert memb.tolist() == want_memb, (mu, eps)
        assert oracle.roles(g, memb).tolist() == want_roles, (mu, eps)


def test_roles_special_cases():
    # no clusters at all: every vertex is an outlier, isolated ones included
    g = graphgen.from_edges(5, [(0, 1), (1, 2)])
    assert oracle.roles(g, np.full(5, -1, np.int32)).tolist() == [2] * 5
    # a star whose leaves sit in three different clusters: the centre is a hub
    # whatever the labels' values; with two leaves in one cluster and the
    # third unclustered it is an outlier
    g = graphgen.from_edges(4, [(0, 1), (0, 2), (0, 3)])
    assert oracle.roles(g, np.array([-1, 7, 3, 9], np.int32)).tolist() == [1, 0, 0, 0]
    assert oracle.roles(g, np.array([-1, 7, 7, -1], np.int32)).tolist() == [2, 0, 0, 2]


# --------------------------------------------------------------------------
# Closed forms


@pytest.mark.parametrize("n", [2, 3, 5, 9])
def test_complete_graph(n):
    g = graphgen.from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    counts, sim = oracle.similarities(g)
    assert np.all(counts == n) and np.all(sim == 1.0)  # t = n - 2, all twins


@pytest.mark.parametrize("n", [4, 5, 8, 13])
def test_cycle_and_star(n):
    cyc = graphgen.from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    counts, sim = oracle.similarities(cyc)
    assert np.all(counts == 2)
    assert np.all(sim == sim[0]) and within_ulps(sim[0], exact_cosine(2, 3, 3), 2)
    star = graphgen.from_edges(n, [(0, i) for i in range(1, n)])
    counts, sim = oracle.similarities(star)
    assert np.all(counts == 2)
    assert within_ulps(sim[0], exact_cosine(2, n, 2), 2)
    counts, sim = oracle.similarities(star, oracle.JACCARD)
    assert np.all(sim == 2 / n)


def test_triangle_c3():
    g = graphgen.from_edges(3, [(0, 1), (1, 2), (0, 2)])
    counts, _ = oracle.similarities(g)
    assert np.all(counts - 2 == 1)


def test_empty_and_isolated():
    g = graphgen.from_edges(5, np.zeros((0, 2), np.int32))
    ix = oracle.build_index(g)
    assert ix.dmax == 0 and len(ix.co_off) == 3 and ix.co_off.tolist() == [0, 0, 0]
    assert oracle.query(ix, 2, 0.0)[0].tolist() == [-1] * 5
    g = graphgen.from_edges(6, [(1, 4)])
    ix = oracle.build_index(g)
    assert ix.co_ids.tolist() == [1, 4]
    assert oracle.query(ix, 2, 0.5)[0].tolist() == [-1, 1, -1, -1, 1, -1]


def test_query_rejects():
    g = graphgen.from_edges(3, [(0, 1)])
    ix = oracle.build_index(g)
    with pytest.raises(ValueError):
        oracle.query(ix, 1, 0.5)
    with pytest.raises(ValueError):
        oracle.query(ix, 2, float("nan"))
    assert oracle.query(ix, 100, 0.0)[0].tolist() == [-1, -1, -1]


def test_validate():
    good = graphgen.from_edges(4, [(0, 1), (1, 2)])
    assert oracle.validate(good) == -1
    bad = graphgen.Graph(3, np.array([0, 1, 1, 1]), np.array([1], np.int32))  # asymmetric
    assert oracle.validate(bad) == 0
    loop = graphgen.Graph(2, np.array([0, 1, 1]), np.array([0], np.int32))
    assert oracle.validate(loop) == 0
    unsorted = graphgen.Graph(3, np.array([0, 2, 3, 4]), np.array([2, 1, 0, 0], np.int32))
    assert oracle.validate(unsorted) == 0
    # a repeated id in a row (0 lists 1 twice; 1 lists 0 twice): not strictly ascending
    dup = graphgen.Graph(2, np.array([0, 2, 4]), np.array([1, 1, 0, 0], np.int32))
    assert oracle.validate(dup) == 0
    # repeated only in row 1: row 0 is fine, row 1 is the first bad one
    dup1 = graphgen.Graph(3, np.array([0, 1, 3, 4]), np.array([1, 0, 0, 1], np.int32))
    assert oracle.validate(dup1) == 1
    # ids past n - 1 and negative ids
    high = graphgen.Graph(3, np.array([0, 0, 1, 1]), np.array([3], np.int32))
    assert oracle.validate(high) == 1
    neg = graphgen.Graph(3, np.array([0, 0, 1, 1]), np.array([-1], np.int32))
    assert oracle.validate(neg) == 1
    # offsets that decrease (row 1 would be [2, 1))
    dec = graphgen.Graph(3, np.array([0, 2, 1, 2]), np.array([1, 2], np.int32))
    assert oracle.validate(dec) == 1


# --------------------------------------------------------------------------
# Invariants on larger graphs


def invariant_graphs():
    return [graphgen.rmat(10, 16, seed=3), graphgen.sbm(600, 6, 0.08, 0.004, seed=5),
            graphgen.random_graph(60, 0.3, seed=9)]


@pytest.mark.parametrize("gi", range(3))
@pytest.mark.parametrize("kind", [oracle.COSINE, oracle.JACCARD])
def test_similarity_invariants(gi, kind):
    g = invariant_graphs()[gi]
    counts, sim = oracle.similarities(g, kind)
    rows = np.repeat(np.arange(g.n), g.degrees())
    mirror = np.array([slot_of(g, int(v), int(u)) for u, v in zip(rows, g.adj)])
    assert np.array_equal(sim.view(np.uint64), sim[mirror].view(np.uint64))
    assert np.all(sim > 0) and np.all(sim <= 1)
    # sigma == 1 exactly iff the closed neighbourhoods are equal (twins).
    nb = brute_scan.closed_neighbourhoods(g)
    twins = np.array([nb[u] == nb[v] for u, v in zip(rows.tolist(), g.adj.tolist())])
    assert np.array_equal(sim == 1.0, twins)
    # Triangle identity: sum over slots of t = trace(A^3) = 6 * #triangles.
    A = sp.csr_matrix((np.ones(g.nnz, np.int64), g.adj, g.off), shape=(g.n, g.n))
    assert int((counts.astype(np.int64) - 2).sum()) == int((A @ A).multiply(A).sum())


def test_sbm2000_counts_by_dense_matrix_product():
    g = graphgen.sbm2000()
    counts, sim = oracle.similarities(g)
    A = np.zeros((g.n, g.n), np.float64)  # small integers: exact in float64
    rows = np.repeat(np.arange(g.n), g.degrees())
    A[rows, g.adj] = 1
    t = (A @ A)[rows, g.adj].astype(np.int64)
    assert np.array_equal(counts, t + 2)


@pytest.mark.parametrize("gi", range(3))
def test_order_invariants(gi):
    g = invariant_graphs()[gi]
    ix = oracle.build_index(g)
    deg = g.degrees()
    for v in range(g.n):
        a, b = ix.off[v], ix.off[v + 1]
        assert sorted(ix.no_ids[a:b].tolist()) == g.adj[a:b].tolist()
        keys = list(zip((-ix.no_sim[a:b]).tolist(), ix.no_ids[a:b].tolist()))
        assert keys == sorted(keys)
        assert all(ix.no_sim[a + k] == ix.sim[slot_of(g, v, int(w))] for k, w in enumerate(ix.no_ids[a:b]))
    assert ix.dmax == deg.max() and ix.co_off[-1] == g.nnz
    for mu in range(2, ix.dmax + 2):
        a, b = ix.co_off[mu], ix.co_off[mu + 1]
        ids = ix.co_ids[a:b]
        assert b - a == int((deg >= mu - 1).sum())
        assert sorted(ids.tolist()) == np.nonzero(deg >= mu - 1)[0].tolist()
        assert np.array_equal(ix.co_thr[a:b], ix.no_sim[ix.off[ids] + mu - 2])
        keys = list(zip((-ix.co_thr[a:b]).tolist(), ids.tolist()))
        assert keys == sorted(keys)
    # thr(v, mu) is non-increasing in mu, and CO[2]'s threshold is the best
    # neighbour similarity.
    for v in np.nonzero(deg > 0)[0]:
        row = ix.no_sim[ix.off[v]:ix.off[v + 1]]
        assert np.all(np.diff(row) <= 0) and row[0] == ix.sim[ix.off[v]:ix.off[v + 1]].max()


@pytest.mark.parametrize("gi", range(3))
def test_query_invariants(gi):
    g = invariant_graphs()[gi]
    ix = oracle.build_index(g)
    rows = np.repeat(np.arange(g.n), g.degrees())
    prev = {}
    for mu in (2, 3, 5, 9):
        for eps in (0.1, 0.3, 0.5, 0.7, 0.9):
            memb, core = oracle.query(ix, mu, eps)
            core = core.astype(bool)
            for (pm, pe), pc in prev.items():
                if pm <= mu and pe <= eps:
                    assert np.all(pc[core]), "cores must shrink as mu or eps grow"
            prev[(mu, eps)] = core
            simok = ix.sim >= eps
            cc = core[rows] & core[g.adj] & simok
            assert np.all(memb[rows[cc]] == memb[g.adj[cc]])
            A = sp.csr_matrix((np.ones(int(cc.sum())), (rows[cc], g.adj[cc])), shape=(g.n, g.n))
            _, comp = connected_components(A, directed=False)
            cidx = np.nonzero(core)[0]
            for c in np.unique(comp[cidx]):
                members = cidx[comp[cidx] == c]
                assert np.all(memb[members] == members.min())
            for v in np.nonzero(~core)[0]:
                a, b = g.off[v], g.off[v + 1]
                cand = [(-ix.sim[s], int(g.adj[s])) for s in range(a, b) if core[g.adj[s]] and ix.sim[s] >= eps]
                assert memb[v] == (memb[min(cand)[1]] if cand else -1)


# --------------------------------------------------------------------------
# Brute force: index query == direct SCAN for every distinct (mu, eps)


def check_against_direct_scan(g, kind):
    ix = oracle.build_index(g, kind)
    tables = brute_scan.sigma_table(g, kind)
    nb, sig = tables
    rows = np.repeat(np.arange(g.n), g.degrees())
    for s, (u, v) in enumerate(zip(rows.tolist(), g.adj.tolist())):
        assert ix.sim[s] == sig[(u, v)]
        assert ix.counts[s] == len(nb[u] & nb[v])
    for eps in brute_scan.eps_grid(sig.values()):
        for mu in range(2, ix.dmax + 3):
            m_o, c_o = oracle.query(ix, mu, eps)
            m_b, c_b = brute_scan.direct_scan(g, kind, mu, eps, tables)
            assert m_o.tolist() == m_b and c_o.tolist() == c_b, (mu, eps)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_direct_scan_exhaustive(n):
    for g in graphgen.tiny_graphs(n):
        for kind in (oracle.COSINE, oracle.JACCARD):
            check_against_direct_scan(g, kind)


@pytest.mark.parametrize("n", [6, 7])
def test_direct_scan_sampled_labelled(n):
    npairs = n * (n - 1) // 2
    for i in range(150):
        mask = graphgen.draw(100 + n, i) & ((1 << npairs) - 1)
        pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
        edges = [p for k, p in enumerate(pairs) if mask >> k & 1]
        g = graphgen.from_edges(n, edges or np.zeros((0, 2), np.int32))
        check_against_direct_scan(g, oracle.COSINE if i % 2 == 0 else oracle.JACCARD)


@pytest.mark.parametrize("n", [8, 10, 12])
@pytest.mark.parametrize("p", [0.2, 0.45, 0.7])
def test_direct_scan_random(n, p):
    for seed in range(8):
        g = graphgen.random_graph(n, p, seed=1000 * n + seed + int(100 * p))
        check_against_direct_scan(g, seed % 2)


def test_neighbor_order_row_pins():
    """One-row neighbour order: similarity descending, ties by lower id; the
    full pass is the per-row function applied to every row."""
    ids, sims = oracle.neighbor_order_row(np.array([5, 3, 9, 1]), np.array([0.5, 0.7, 0.5, 0.7]))
    assert ids.tolist() == [1, 3, 5, 9] and sims.tolist() == [0.7, 0.7, 0.5, 0.5]
    g = graphgen.random_graph(60, 0.2, seed=12)
    ix = oracle.build_index(g)
    for v in range(g.n):
        a, b = g.off[v], g.off[v + 1]
        ri, rs = oracle.neighbor_order_row(g.adj[a:b], ix.sim[a:b])
        assert np.array_equal(ri, ix.no_ids[a:b]) and np.array_equal(rs, ix.no_sim[a:b])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_query_props_match_oracle(seed):
    """The host-side query checker used at sizes beyond the oracle agrees with
    the oracle's query on small graphs, over a grid of (mu, eps)."""
    from query_props import expected_query

    g = graphgen.sbm(600, 6, 0.08, 0.004, seed=seed) if seed < 3 else graphgen.rmat(9, 8, seed=seed)
    ix = oracle.build_index(g)
    for mu in (2, 3, 5, 9):
        for eps in (0.1, 0.3, 0.5, 0.7):
            memb, core = oracle.query(ix, mu, eps)
            w, wc = expected_query(g.off, g.adj, ix.sim, ix.no_ids, ix.no_sim, mu, eps)
            assert np.array_equal(wc, core.astype(bool)), (mu, eps)
            assert np.array_equal(w, memb), (mu, eps)


# --------------------------------------------------------------------------
# Modularity (Section 7.2; unclustered vertices as singletons, Section 7.3.4)


def modularity_by_definition(g, memb):
    """The printed double sum over ordered vertex pairs, in exact rationals."""
    from fractions import Fraction

    n = g.n
    deg = np.diff(g.off)
    adj = [set(g.adj[g.off[v]:g.off[v + 1]].tolist()) for v in range(n)]
    cl = [int(m) if m >= 0 else -(v + 1) for v, m in enumerate(memb)]  # singletons get distinct labels
    two_m = int(g.nnz)
    total = Fraction(0)
    for u in range(n):
        for v in range(n):
            if cl[u] == cl[v]:
                total += Fraction(int(v in adj[u])) - Fraction(int(deg[u]) * int(deg[v]), two_m)
    return total / two_m


def test_modularity_closed_forms():
    # two disjoint triangles, one cluster each: 2 * (3/6 - (6/12)^2) = 1/2
    g = graphgen.from_edges(6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)])
    assert oracle.modularity(g, np.array([0, 0, 0, 3, 3, 3], np.int32))[0] == 0.5
    # a connected graph as one cluster: 1 - 1 = 0
    g = graphgen.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    assert oracle.modularity(g, np.zeros(4, np.int32))[0] == 0.0
    # every vertex on its own: -sum d^2 / (2m)^2 = -(1 + 4 + 4 + 1) / 36
    q, s_in, sd2 = oracle.modularity(g, np.full(4, -1, np.int32))
    assert (s_in, sd2) == (0, 10) and q == -10 / 36


@pytest.mark.parametrize("seed", range(6))
def test_modularity_matches_the_printed_sum(seed):
    from fractions import Fraction

    rng = np.random.default_rng(seed)
    g = graphgen.random_graph(9 + seed, 0.35, seed=seed + 40)
    if g.nnz == 0:
        return
    memb = rng.integers(-1, 3, g.n).astype(np.int32)
    memb = np.where(memb >= 0, memb * 2, -1).astype(np.int32)  # labels 0, 2, 4 or unclustered
    q, s_in, sd2 = oracle.modularity(g, memb)
    exact = modularity_by_definition(g, memb)
    assert (Fraction(s_in) - Fraction(sd2, g.nnz)) / g.nnz == exact
    assert abs(Fraction(q) - exact) <= Fraction(4 * 2 ** -52) * max(1, abs(exact))


# --------------------------------------------------------------------------
# The per-edge entry points (checkers of sampled parity on graphs too large
# for the full oracle pass) against the full pass, every slot.


@pytest.mark.parametrize("kind", [oracle.COSINE, oracle.JACCARD])
@pytest.mark.parametrize("gi", range(3))
def test_edge_similarities_equal_full_pass(gi, kind):
    g = invariant_graphs()[gi]
    counts, sim = oracle.similarities(g, kind, threads=4)
    rows = np.repeat(np.arange(g.n), g.degrees())
    c, s = oracle.edge_similarities(g, rows, g.adj.astype(np.int64), kind, threads=4)
    assert np.array_equal(c, counts)
    assert np.array_equal(s.view(np.uint64), sim.view(np.uint64))
    # the one-row order of a row's per-edge similarities is the full pass's row
    ix = oracle.build_index(g, kind)
    for v in range(0, g.n, max(1, g.n // 40)):
        a, b = int(g.off[v]), int(g.off[v + 1])
        ids, sims = oracle.neighbor_order_row(g.adj[a:b], s[a:b])
        assert np.array_equal(ids, ix.no_ids[a:b]) and np.array_equal(sims.view(np.uint64), ix.no_sim[a:b].view(np.uint64))
