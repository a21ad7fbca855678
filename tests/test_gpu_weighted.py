"""Parity of the weighted-cosine build (Section 3.1) through the C ABI with
the oracle: similarity bits, both orders and queries, bit for bit."""

from __future__ import annotations

import ctypes

import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_11188_amd as scan
from gpu_util import bits, device_csr

pytestmark = pytest.mark.gpu
FLAGS = scan.SCAN_KEEP_SIMS


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    scan.load_library()
    yield
    torch.cuda.synchronize()


def hub_graph(leaves=5000, extra=20000, seed=7):
    """Vertex 0 joined to `leaves` others (three LDS tiles of its row) plus
    random edges among them: long owner rows next to short ones."""
    rng = np.random.default_rng(seed)
    e = [(0, i) for i in range(1, leaves + 1)]
    e += [tuple(x) for x in rng.integers(1, leaves + 1, size=(extra, 2)).tolist()]
    return graphgen.from_edges(leaves + 1, e)


def graphs():
    return [
        ("sbm600", graphgen.sbm(600, 6, 0.15, 0.01, seed=3)),
        ("rmat11", graphgen.rmat(11, 8, seed=12)),
        ("hub5000", hub_graph()),
    ]


def weighted_gpu(g, w, bits_=32, flags=FLAGS, on_device=True):
    import torch

    if on_device:
        off, adj = device_csr(g, bits_)
        return scan.scan_build_index_weighted(off, adj, torch.from_numpy(w).cuda(), flags)
    off = g.off.astype(np.int32 if bits_ == 32 else np.int64)
    return scan.scan_build_index_weighted(off, g.adj.astype(np.int32), w, flags)


def assert_weighted_equal(gix, oix):
    import torch

    torch.cuda.synchronize()
    assert gix.info.kind == scan.WEIGHTED_COSINE
    for name, code, want in (("sim", scan.ARR_SIMS, oix.sim), ("no_ids", scan.ARR_NO_IDS, oix.no_ids),
                             ("no_sim", scan.ARR_NO_SIM, oix.no_sim), ("co_off", scan.ARR_CO_OFF, oix.co_off),
                             ("co_ids", scan.ARR_CO_IDS, oix.co_ids), ("co_thr", scan.ARR_CO_THR, oix.co_thr)):
        got = scan.scan_index_export(gix, code)
        if got.dtype == np.float64:
            assert np.array_equal(bits(got), bits(want)), name
        else:
            assert np.array_equal(got, want), name


@pytest.mark.parametrize("gi", range(3))
def test_weighted_parity(gi):
    name, g = graphs()[gi]
    w = graphgen.edge_weights(g, 100 + gi)
    say("weighted parity", name, "n", g.n, "nnz", g.nnz)
    oix = oracle.build_index_weighted(g, w, threads=8)
    gix = weighted_gpu(g, w)
    assert_weighted_equal(gix, oix)
    for mu, eps in [(2, 0.3), (3, 0.5), (5, 0.2), (4, 0.7), (oix.dmax + 1, 0.01), (oix.dmax + 2, 0.0)]:
        memb, core = scan.scan_query_ex(gix, mu, eps)
        om, oc = oracle.query(oix, mu, eps)
        assert np.array_equal(memb.cpu().numpy(), om), (mu, eps)
        assert np.array_equal(core.cpu().numpy(), oc), (mu, eps)


def test_weighted_asymmetric_weights():
    # the two directions of an edge carry different weights: each side's own
    # weights enter the sums
    g = hub_graph(leaves=2500, extra=8000, seed=3)
    rng = np.random.default_rng(5)
    w = rng.uniform(0.01, 3.0, g.nnz)
    say("asymmetric weights nnz", g.nnz)
    assert_weighted_equal(weighted_gpu(g, w), oracle.build_index_weighted(g, w, threads=8))


def test_unit_weights_equal_the_cosine_index():
    import torch

    g = graphgen.rmat(12, 8, seed=2)
    say("unit weights rmat12 nnz", g.nnz)
    a = weighted_gpu(g, np.ones(g.nnz))
    off, adj = device_csr(g)
    b = scan.scan_build_index(off, adj, scan.COSINE, FLAGS)
    torch.cuda.synchronize()
    for code in (scan.ARR_SIMS, scan.ARR_NO_IDS, scan.ARR_NO_SIM, scan.ARR_CO_OFF, scan.ARR_CO_IDS, scan.ARR_CO_THR):
        x, y = scan.scan_index_export(a, code), scan.scan_index_export(b, code)
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), code


@pytest.mark.parametrize("bits_,on_device", [(64, True), (32, False), (64, False)])
def test_weighted_offsets_and_host_inputs(bits_, on_device):
    g = graphgen.sbm(700, 7, 0.12, 0.01, seed=8)
    w = graphgen.edge_weights(g, 44)
    say("weighted", bits_, "bit offsets, device", on_device)
    assert_weighted_equal(weighted_gpu(g, w, bits_, on_device=on_device), oracle.build_index_weighted(g, w))


@pytest.mark.parametrize("case", ["empty", "no_edges", "one_edge", "isolated", "path"])
def test_weighted_edge_cases(case):
    if case == "empty":
        g = graphgen.from_edges(0, np.zeros((0, 2), np.int32))
    elif case == "no_edges":
        g = graphgen.from_edges(5, np.zeros((0, 2), np.int32))
    elif case == "one_edge":
        g = graphgen.from_edges(2, [(0, 1)])
    elif case == "isolated":
        g = graphgen.from_edges(9, [(1, 4), (4, 7), (1, 7), (7, 8)])
    else:
        g = graphgen.from_edges(300, [(i, i + 1) for i in range(299)])
    w = graphgen.edge_weights(g, 3, 0.5, 2.0)
    say("weighted edge case", case)
    gix = weighted_gpu(g, w, on_device=g.n > 0)
    oix = oracle.build_index_weighted(g, w)
    if g.nnz:
        assert_weighted_equal(gix, oix)
    else:
        assert gix.info.n == g.n and gix.info.nnz == 0


def test_weighted_errors():
    import torch

    g = graphgen.sbm(100, 2, 0.2, 0.05, seed=1)
    off, adj = device_csr(g)
    w = torch.from_numpy(graphgen.edge_weights(g, 1)).cuda()
    with pytest.raises(scan.ScanError, match="EINVAL"):
        scan.scan_build_index_weighted(off, adj, w, scan.SCAN_KEEP_COUNTS)
    bad = w.clone()
    bad[7] = float("nan")
    with pytest.raises(scan.ScanError, match="EGRAPH"):
        scan.scan_build_index_weighted(off, adj, bad, scan.SCAN_VALIDATE)
    bad[7] = float("inf")
    with pytest.raises(scan.ScanError, match="EGRAPH"):
        scan.scan_build_index_weighted(off, adj, bad, scan.SCAN_VALIDATE)
    with pytest.raises(ValueError):
        scan.scan_build_index_weighted(off, adj, w[:-1])
    with pytest.raises(scan.ScanError, match="EINVAL"):  # the unweighted entry cannot build it
        scan.scan_build_index(off, adj, scan.WEIGHTED_COSINE)
    # a null weights pointer through the C ABI
    lib = scan.load_library()
    c, keep = scan._csr_struct(off, adj)
    out = ctypes.c_void_p()
    assert lib.scan_build_index_weighted(ctypes.byref(c), None, 0, None, ctypes.byref(out)) == -1
    assert not out.value


def test_weighted_rmat20_sampled():
    """R-MAT-20 (the benchmark's graph) with seeded weights: sampled edges
    against the oracle one by one, plus the orders' invariants."""
    import torch

    g = graphgen.rmat20()
    w = graphgen.edge_weights(g, 2020)
    say("weighted rmat20 nnz", g.nnz)
    off, adj = device_csr(g)
    gix = scan.scan_build_index_weighted(off, adj, torch.from_numpy(w).cuda(), FLAGS)
    torch.cuda.synchronize()
    sim = scan.scan_index_export(gix, scan.ARR_SIMS)
    deg = np.diff(g.off)
    rng = np.random.default_rng(20)
    slots = rng.choice(g.nnz, 1500, replace=False)
    hubs = np.argsort(deg)[-3:]
    slots = np.concatenate([slots] + [np.arange(g.off[h], g.off[h] + 40) for h in hubs])
    us = (np.searchsorted(g.off, slots, side="right") - 1).astype(np.int64)
    vs = g.adj[slots].astype(np.int64)
    want = oracle.weighted_edge_similarities(g, w, us, vs)
    assert np.array_equal(bits(sim[slots]), bits(want))
    # both slots of every edge hold the same value
    rows = np.repeat(np.arange(g.n), deg)
    mirror = np.empty(g.nnz, np.int64)
    key = rows.astype(np.int64) * g.n + g.adj
    order = np.argsort(g.adj.astype(np.int64) * g.n + rows, kind="stable")
    mirror[order] = np.arange(g.nnz)
    assert np.array_equal(key[mirror], g.adj.astype(np.int64) * g.n + rows)
    assert np.array_equal(bits(sim), bits(sim[mirror]))
    no_ids = scan.scan_index_export(gix, scan.ARR_NO_IDS)
    no_sim = scan.scan_index_export(gix, scan.ARR_NO_SIM)
    same = rows[1:] == rows[:-1]
    d = np.diff(no_sim)
    assert np.all(~same | (d < 0) | ((d == 0) & (np.diff(no_ids) > 0)))


def test_weighted_validated_build():
    # SCAN_VALIDATE on a valid graph with finite weights changes nothing
    g = graphgen.rmat(11, 8, seed=40)
    w = graphgen.edge_weights(g, 41)
    say("weighted validated build")
    assert_weighted_equal(weighted_gpu(g, w, flags=FLAGS | scan.SCAN_VALIDATE), oracle.build_index_weighted(g, w))
