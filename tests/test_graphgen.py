"""Input generators: determinism and CSR invariants (no method arithmetic)."""

import numpy as np
import pytest

import graphgen


def check_csr(g):
    assert g.off[0] == 0 and len(g.off) == g.n + 1
    assert np.all(np.diff(g.off) >= 0)
    assert g.nnz % 2 == 0
    if g.nnz == 0:
        return
    assert g.adj.min() >= 0 and g.adj.max() < g.n
    rows = np.repeat(np.arange(g.n), np.diff(g.off))
    assert not np.any(rows == g.adj), "self-loop"
    same_row = rows[1:] == rows[:-1]
    assert np.all(g.adj[1:][same_row] > g.adj[:-1][same_row]), "row not strictly ascending"
    fwd = rows.astype(np.int64) * g.n + g.adj
    bwd = g.adj.astype(np.int64) * g.n + rows
    assert np.array_equal(np.sort(fwd), np.sort(bwd)), "not symmetric"


@pytest.mark.parametrize("scale", [4, 8, 12])
def test_rmat_csr_and_determinism(scale):
    a = graphgen.rmat(scale, 16, seed=7)
    b = graphgen.rmat(scale, 16, seed=7)
    c = graphgen.rmat(scale, 16, seed=8)
    check_csr(a)
    assert np.array_equal(a.off, b.off) and np.array_equal(a.adj, b.adj)
    assert not (np.array_equal(a.off, c.off) and np.array_equal(a.adj, c.adj))
    # Skew: the first quadrant is the most likely, so vertex 0 has the top degree.
    d = a.degrees()
    assert d[0] == d.max()


def test_sbm_csr_and_expected_edges():
    g = graphgen.sbm2000()
    check_csr(g)
    # E|E| = 20*C(100,2)*0.1 + (C(2000,2) - 20*C(100,2))*0.002 = 9900 + 3800.
    mean, var = 9900 + 3800, 9900 * 0.9 + 3800 * 0.998
    assert abs(g.num_edges - mean) < 5 * var ** 0.5
    rows = np.repeat(np.arange(g.n), np.diff(g.off))
    within = (rows // 100) == (g.adj // 100)
    assert abs(within.sum() // 2 - 9900) < 5 * (9900 * 0.9) ** 0.5


def test_sbm_extremes():
    full = graphgen.sbm(30, 3, 1.0, 0.0, seed=1)
    check_csr(full)
    assert full.num_edges == 3 * 45
    empty = graphgen.sbm(30, 3, 0.0, 0.0, seed=1)
    assert empty.nnz == 0


def test_from_edges_cleans():
    g = graphgen.from_edges(5, [(0, 1), (1, 0), (2, 2), (3, 4), (4, 3), (0, 1)])
    check_csr(g)
    assert g.num_edges == 2


def test_batch_specs():
    specs = graphgen.batch_sbm_specs(256)
    assert len(specs) == 256
    for s in specs:
        assert 1000 <= s.n <= 200000 and 1 <= s.k <= 200 and 8 <= s.d <= 64
        assert 0 < s.p_in <= 1 and abs(s.p_out - 0.02 * s.p_in) < 1e-15
    assert specs == graphgen.batch_sbm_specs(256)


def test_degree_stats():
    g = graphgen.from_edges(4, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)])
    st = graphgen.degree_stats(g)
    assert st["dmax"] == 3 and st["edges"] == 5
    assert st["w_min"] == 2 + 2 + 3 + 2 + 2
    assert st["sum_deg2"] == 4 + 9 + 9 + 4


def test_owner_split():
    """The owner split partitions the edges and W_min; brute force on a small
    graph with a threshold that lands in the middle of the degree range."""
    g = graphgen.rmat(9, 8, seed=4)
    deg = np.diff(g.off)
    for small_max in (0, 3, 8, 10**6):
        sp = graphgen.owner_split(g, small_max)
        st = graphgen.degree_stats(g)
        assert sp["edges_small"] + sp["edges_big"] == g.num_edges
        assert sp["w_small"] + sp["w_big"] == st["w_min"]
        es = ws = 0
        for u in range(g.n):
            for v in g.adj[g.off[u]:g.off[u + 1]]:
                if v <= u:
                    continue
                owner = u if (deg[u], u) > (deg[v], v) else v
                if deg[owner] <= small_max:
                    es += 1
                    ws += min(deg[u], deg[v])
        assert (sp["edges_small"], sp["w_small"]) == (es, ws)


def test_edge_weights_symmetric_and_in_range():
    g = graphgen.rmat(10, 8, seed=6)
    w = graphgen.edge_weights(g, 9, 0.05, 1.0)
    assert w.shape == (g.nnz,) and w.min() >= 0.05 and w.max() < 1.0
    rows = np.repeat(np.arange(g.n), np.diff(g.off))
    # the weight of (u, v) equals that of (v, u): compare via a dict of pairs
    pair = {(int(u), int(v)): x for u, v, x in zip(rows, g.adj, w)}
    assert all(pair[(v, u)] == x for (u, v), x in pair.items())
    assert np.array_equal(w, graphgen.edge_weights(g, 9, 0.05, 1.0))  # seeded
    assert not np.array_equal(w, graphgen.edge_weights(g, 10, 0.05, 1.0))
    assert len(np.unique(w)) > 0.9 * g.num_edges  # full-mantissa draws, no repeats to speak of


def test_gaussians_moments_and_determinism():
    x = graphgen.gaussians(4000, 64, 3)
    assert x.shape == (4000, 64)
    assert abs(x.mean()) < 0.01 and abs(x.std() - 1.0) < 0.01
    # standard normal tails: about 4.55% beyond 2 sigma
    assert abs((np.abs(x) > 2).mean() - 0.0455) < 0.003
    assert np.array_equal(x, graphgen.gaussians(4000, 64, 3))
    assert np.array_equal(x[:10], graphgen.gaussians(10, 64, 3))  # coordinate c = x * k + i: prefixes agree


def test_permutation_is_a_permutation():
    for n in (1, 2, 17, 10000):
        p = graphgen.permutation(n, 5)
        assert p.dtype == np.uint32 and np.array_equal(np.sort(p), np.arange(n, dtype=np.uint32))
    p = graphgen.permutation(10000, 5)
    assert np.array_equal(p, graphgen.permutation(10000, 5))
    assert (p == np.arange(10000)).mean() < 0.01  # not close to the identity
