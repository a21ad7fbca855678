"""R-MAT scale 23 (edge factor 32, int64 offsets, hubs of degree > 1e5), cosine
and Jaccard, at full size. The oracle cannot build this index in test time,
so parity is checked on samples the oracle computes one by one (edge counts
and similarities, whole neighbour-order rows) and through properties that
hold at any size (core-order offsets from the degree distribution, core-order
segments against the definition, and every query output against the query's
definition evaluated on the host, tests/query_props.py)."""

from __future__ import annotations

import time

import numpy as np
import pytest
import graphgen
import oracle
import paper_2012_11188_amd as scan
from gpu_util import bits
from query_props import expected_query

pytestmark = pytest.mark.gpu

FLAGS = scan.SCAN_KEEP_SIMS | scan.SCAN_KEEP_COUNTS


def log(msg):
    print(msg, flush=True)


def export(ix):
    return {name: scan.scan_index_export(ix, code) for name, code in [
        ("sims", scan.ARR_SIMS), ("counts", scan.ARR_COUNTS), ("no_ids", scan.ARR_NO_IDS),
        ("no_sim", scan.ARR_NO_SIM), ("co_off", scan.ARR_CO_OFF), ("co_ids", scan.ARR_CO_IDS),
        ("co_thr", scan.ARR_CO_THR)]}


@pytest.fixture(scope="module")
def r23():
    import torch

    t = time.time()
    g = graphgen.rmat23()
    log(f"rmat23: n={g.n} nnz={g.nnz} generated in {time.time() - t:.1f}s")
    off = torch.from_numpy(g.off.astype(np.int64)).cuda()
    adj = torch.from_numpy(g.adj).cuda()
    out = {"g": g, "deg": np.diff(g.off).astype(np.int64), "dev": (off, adj), "ix": {}, "arr": {}}
    for kind in (scan.COSINE, scan.JACCARD):
        t = time.time()
        ix = scan.scan_build_index(off, adj, kind, FLAGS)
        torch.cuda.synchronize()
        log(f"kind {kind}: built in {time.time() - t:.2f}s")
        out["ix"][kind] = ix
        out["arr"][kind] = export(ix)
        log(f"kind {kind}: exported")
    return out


def row_of(off, slots):
    return np.searchsorted(off, slots, side="right") - 1


def test_r23_shape(r23):
    g, deg = r23["g"], r23["deg"]
    ix = r23["ix"][scan.COSINE]
    assert ix.info.n == g.n == 1 << 23 and ix.info.nnz == g.nnz
    assert ix.info.dmax == deg.max() > 100_000
    # CO[mu] holds every vertex of degree >= mu - 1, for mu = 2 .. dmax + 1
    for kind in (scan.COSINE, scan.JACCARD):
        co_off = r23["arr"][kind]["co_off"]
        dmax = int(deg.max())
        ge = np.cumsum(np.bincount(deg, minlength=dmax + 1)[::-1])[::-1]  # ge[k] = #(deg >= k)
        want = np.zeros(dmax + 3, np.int64)
        want[3:] = np.cumsum(ge[1:dmax + 1])
        assert np.array_equal(co_off, want)


@pytest.mark.parametrize("kind", [scan.COSINE, scan.JACCARD])
def test_r23_sampled_edges(r23, kind):
    g, deg, a = r23["g"], r23["deg"], r23["arr"][kind]
    rng = np.random.default_rng(23 + kind)
    hub = int(np.argmax(deg))
    slots = np.concatenate([rng.integers(0, g.nnz, 6000 if kind == scan.COSINE else 3000),
                            g.off[hub] + rng.choice(deg[hub], 1000, replace=False)])
    u = row_of(g.off, slots)
    v = g.adj[slots].astype(np.int64)
    t = time.time()
    cs, ss = oracle.edge_similarities(g, u, v, kind)
    log(f"oracle: {len(slots)} edges in {time.time() - t:.1f}s")
    assert np.array_equal(a["counts"][slots], cs)
    assert np.array_equal(bits(a["sims"][slots]), bits(ss))
    # the mirror slot of each sampled edge holds the same values
    mir = np.array([g.off[y] + np.searchsorted(g.adj[g.off[y]:g.off[y + 1]], x) for x, y in zip(u, v)])
    assert np.array_equal(g.adj[mir], u)
    assert np.array_equal(bits(a["sims"][mir]), bits(ss)) and np.array_equal(a["counts"][mir], cs)


@pytest.mark.parametrize("kind", [scan.COSINE, scan.JACCARD])
def test_r23_neighbor_order(r23, kind):
    g, deg, a = r23["g"], r23["deg"], r23["arr"][kind]
    rng = np.random.default_rng(230 + kind)
    small = np.flatnonzero((deg > 0) & (deg <= 400))
    rows = rng.choice(small, 60 if kind == scan.COSINE else 30, replace=False)
    t = time.time()
    for v in rows:
        b, e = g.off[v], g.off[v + 1]
        ids = g.adj[b:e]
        _, sims = oracle.edge_similarities(g, np.full(len(ids), v), ids.astype(np.int64), kind)
        wi, ws = oracle.neighbor_order_row(ids, sims)
        assert np.array_equal(a["no_ids"][b:e], wi), v
        assert np.array_equal(bits(a["no_sim"][b:e]), bits(ws)), v
    log(f"oracle rows: {time.time() - t:.1f}s")
    # hub rows (too long for the oracle's per-edge merges): a permutation of the
    # row whose sims are the (sampled-checked) slot sims, in (sim desc, id asc)
    for v in np.argsort(deg)[-5:]:
        b, e = g.off[v], g.off[v + 1]
        ni, ns = a["no_ids"][b:e], a["no_sim"][b:e]
        p = np.argsort(ni, kind="stable")
        assert np.array_equal(ni[p], g.adj[b:e])
        assert np.array_equal(bits(ns[p]), bits(a["sims"][b:e]))
        ok = (ns[:-1] > ns[1:]) | ((ns[:-1] == ns[1:]) & (ni[:-1] < ni[1:]))
        assert ok.all(), v


def test_r23_core_order(r23):
    g, deg = r23["g"], r23["deg"]
    dmax = int(deg.max())
    rng = np.random.default_rng(2323)
    mus = sorted({2, 3, 5, 16, 100, 1000, 10_000, 100_000, dmax, dmax + 1,
                  *rng.integers(2, 2000, 8).tolist()})
    for kind in (scan.COSINE, scan.JACCARD):
        a = r23["arr"][kind]
        for mu in mus:
            b, e = a["co_off"][mu], a["co_off"][mu + 1]
            ids, thr = a["co_ids"][b:e], a["co_thr"][b:e]
            assert np.array_equal(np.sort(ids), np.flatnonzero(deg >= mu - 1)), mu
            assert np.array_equal(bits(thr), bits(a["no_sim"][g.off[ids] + mu - 2])), mu
            ok = (thr[:-1] > thr[1:]) | ((thr[:-1] == thr[1:]) & (ids[:-1] < ids[1:]))
            assert ok.all(), mu


@pytest.mark.parametrize("mu,cores", [(2, 1_000_000), (5, 100_000), (16, 10_000), (3, 0)])
def test_r23_query(r23, mu, cores):
    """eps is the core threshold of the cores-th vertex of CO[mu], so the query
    has about that many cores (cores = 0: eps above every threshold)."""
    import torch

    g, deg = r23["g"], r23["deg"]
    a = r23["arr"][scan.COSINE]
    b = a["co_off"][mu]
    eps = float(a["co_thr"][b + cores]) if cores else 1.0 + 1e-9
    memb, core = scan.scan_query_ex(r23["ix"][scan.COSINE], mu, eps)
    torch.cuda.synchronize()
    memb, core = memb.cpu().numpy(), core.cpu().numpy()
    t = time.time()
    want, want_core = expected_query(g.off, g.adj, a["sims"], a["no_ids"], a["no_sim"], mu, eps)
    log(f"query ({mu}, {eps:.6f}): {int(want_core.sum())} cores, {len(np.unique(want[want >= 0]))} clusters, "
        f"host check {time.time() - t:.1f}s")
    assert np.array_equal(core.astype(bool), want_core)
    assert np.array_equal(memb, want)
