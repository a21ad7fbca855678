"""R-MAT scale 23 (edge factor 32, int64 offsets, hubs of degree > 1e5), cosine
and Jaccard, at full size. The oracle cannot build this index in test time,
so parity is checked on samples the oracle computes one by one (counts and
similarities of over 10^6 uniformly sampled CSR slots per kind plus slots of
the largest hub, and whole neighbour-order rows) and through properties that
hold at any size, over every row and every core-order segment:
  - each NO row is a permutation of its CSR row, its similarities are the
    slot similarities of the same neighbours, and it is sorted by (sim desc,
    id asc) (Algorithm 2);
  - CO[mu] holds exactly the vertices of degree >= mu - 1 with thresholds
    NO_SIM[off[v] + mu - 2], sorted by (thr desc, id asc), for every mu;
  - every query output equals the query's definition evaluated on the host
    (tests/query_props.py), for both kinds."""

from __future__ import annotations

import os
import time

import numpy as np
import pytest
import graphgen
import oracle
import paper_2012_11188_amd as scan
from gpu_util import bits
from query_props import expected_query

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

FLAGS = scan.SCAN_KEEP_SIMS | scan.SCAN_KEEP_COUNTS
THREADS = min(16, os.cpu_count() or 1)
SAMPLES = 1_000_000


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
    slots = np.unique(np.concatenate([rng.integers(0, g.nnz, SAMPLES + SAMPLES // 10),
                                      g.off[hub] + rng.choice(deg[hub], 2000, replace=False)]))
    assert len(slots) >= SAMPLES
    u = row_of(g.off, slots)
    v = g.adj[slots].astype(np.int64)
    t = time.time()
    cs, ss = oracle.edge_similarities(g, u, v, kind, threads=THREADS)
    log(f"oracle: {len(slots)} edges in {time.time() - t:.1f}s on {THREADS} threads")
    assert np.array_equal(a["counts"][slots], cs)
    assert np.array_equal(bits(a["sims"][slots]), bits(ss))
    # the mirror slot of each sampled edge holds the same values: positions of
    # (v, u) among the globally sorted (row, id) keys of the CSR
    key = (np.repeat(np.arange(g.n, dtype=np.int64), deg) << 23) | g.adj
    mir = np.searchsorted(key, (v << 23) | u)
    assert np.array_equal(key[mir], (v << 23) | u)
    del key
    assert np.array_equal(bits(a["sims"][mir]), bits(ss)) and np.array_equal(a["counts"][mir], cs)


@pytest.mark.parametrize("kind", [scan.COSINE, scan.JACCARD])
def test_r23_neighbor_order_rows_by_oracle(r23, kind):
    g, deg, a = r23["g"], r23["deg"], r23["arr"][kind]
    rng = np.random.default_rng(230 + kind)
    small = np.flatnonzero((deg > 0) & (deg <= 2000))
    rows = rng.choice(small, 400, replace=False)
    us = np.repeat(rows, deg[rows])
    vs = np.concatenate([g.adj[g.off[v]:g.off[v + 1]] for v in rows]).astype(np.int64)
    t = time.time()
    _, sims = oracle.edge_similarities(g, us, vs, kind, threads=THREADS)
    p = 0
    for v in rows:
        b, e = g.off[v], g.off[v + 1]
        wi, ws = oracle.neighbor_order_row(g.adj[b:e], sims[p:p + e - b])
        p += e - b
        assert np.array_equal(a["no_ids"][b:e], wi), v
        assert np.array_equal(bits(a["no_sim"][b:e]), bits(ws)), v
    log(f"oracle rows: {len(rows)} rows, {len(us)} edges, {time.time() - t:.1f}s")


@pytest.mark.parametrize("kind", [scan.COSINE, scan.JACCARD])
def test_r23_neighbor_order_every_row(r23, kind):
    """Every row: a permutation of the CSR row, with the slot similarities of
    the same neighbours, sorted by (sim desc, id asc)."""
    g, deg, a = r23["g"], r23["deg"], r23["arr"][kind]
    t = time.time()
    row = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    key_no = (row << 23) | a["no_ids"]
    p = np.argsort(key_no)
    key_adj = (row << 23) | g.adj
    del row
    assert np.array_equal(key_no[p], key_adj), "a neighbour-order row is not a permutation of its CSR row"
    del key_no, key_adj
    assert np.array_equal(bits(a["no_sim"][p]), bits(a["sims"])), "neighbour-order sims differ from slot sims"
    del p
    ns, ni = a["no_sim"], a["no_ids"]
    start = np.zeros(g.nnz, bool)
    start[g.off[:-1][deg > 0]] = True
    ok = (ns[:-1] > ns[1:]) | ((ns[:-1] == ns[1:]) & (ni[:-1] < ni[1:])) | start[1:]
    assert ok.all(), f"order broken in row {row_of(g.off, np.flatnonzero(~ok)[:1])}"
    log(f"NO every row, kind {kind}: {time.time() - t:.1f}s")


@pytest.mark.parametrize("kind", [scan.COSINE, scan.JACCARD])
def test_r23_core_order_every_segment(r23, kind):
    """Every mu: CO[mu] holds each vertex of degree >= mu - 1 once, with its
    threshold NO_SIM[off[v] + mu - 2], sorted by (thr desc, id asc)."""
    g, deg, a = r23["g"], r23["deg"], r23["arr"][kind]
    t = time.time()
    dmax = int(deg.max())
    co_off, ids, thr = a["co_off"], a["co_ids"], a["co_thr"]
    assert co_off[2] == 0 and co_off[dmax + 2] == g.nnz
    seg_len = np.diff(co_off[2:dmax + 3])
    mu = np.repeat(np.arange(2, dmax + 2, dtype=np.int64), seg_len)
    assert np.all(deg[ids] >= mu - 1), "a vertex of degree < mu - 1 in CO[mu]"
    pos = g.off[ids] + mu - 2
    assert np.array_equal(bits(thr), bits(a["no_sim"][pos])), "a threshold is not NO_SIM[off[v] + mu - 2]"
    del pos
    start = np.zeros(g.nnz, bool)
    start[co_off[2:dmax + 2][seg_len > 0]] = True
    ok = (thr[:-1] > thr[1:]) | ((thr[:-1] == thr[1:]) & (ids[:-1] < ids[1:])) | start[1:]
    assert ok.all(), f"order broken in CO[{int(mu[np.flatnonzero(~ok)[0]])}]"
    # strictly ordered segments hold no vertex twice; each vertex appears in
    # deg(v) segments, all with mu <= deg(v) + 1: exactly CO[2..deg(v)+1]
    assert np.array_equal(np.bincount(ids, minlength=g.n), deg)
    log(f"CO every segment, kind {kind}: {time.time() - t:.1f}s")


@pytest.mark.parametrize("kind", [scan.COSINE, scan.JACCARD])
@pytest.mark.parametrize("mu,cores", [(2, 1_000_000), (5, 100_000), (16, 10_000), (3, 0)])
def test_r23_query(r23, kind, mu, cores):
    """eps is the core threshold of the cores-th vertex of CO[mu], so the query
    has about that many cores (cores = 0: eps above every threshold)."""
    import torch

    g = r23["g"]
    a = r23["arr"][kind]
    b = a["co_off"][mu]
    eps = float(a["co_thr"][b + cores]) if cores else 1.0 + 1e-9
    memb, core = scan.scan_query_ex(r23["ix"][kind], mu, eps)
    torch.cuda.synchronize()
    memb, core = memb.cpu().numpy(), core.cpu().numpy()
    t = time.time()
    want, want_core = expected_query(g.off, g.adj, a["sims"], a["no_ids"], a["no_sim"], mu, eps)
    log(f"query kind {kind} ({mu}, {eps:.6f}): {int(want_core.sum())} cores, "
        f"{len(np.unique(want[want >= 0]))} clusters, host check {time.time() - t:.1f}s")
    assert np.array_equal(core.astype(bool), want_core)
    assert np.array_equal(memb, want)
