"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Index arrays are compared bit for bit (counts, FP64 similarity bits, both
orders); queries compare memberships and core flags exactly. Inputs are
seeded synthetic graphs from graphgen."""

from __future__ import annotations

import json
import os

import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_11188_amd as scan
from gpu_util import assert_index_equal, assert_queries_equal, bits, export_all, gpu_build, query_grid

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    scan.load_library()
    yield
    torch.cuda.synchronize()


# --------------------------------------------------------------------------
# Device FP64 rounding


@pytest.mark.parametrize("kind", [scan.COSINE, scan.JACCARD])
def test_device_similarity_bits_match_host(kind):
    # every (c, a, b) with 2 <= c <= a <= b <= 160, plus random triples up to
    # the configs' maximum degrees
    a, b, c = [], [], []
    for x in range(2, 161):
        for y in range(x, 161):
            cs = np.arange(2, x + 1)
            c.append(cs)
            a.append(np.full(len(cs), x))
            b.append(np.full(len(cs), y))
    rng = np.random.default_rng(3)
    ra = rng.integers(2, 200_000, 1_000_000)
    rb = rng.integers(2, 200_000, 1_000_000)
    rc = 2 + (rng.random(1_000_000) * (np.minimum(ra, rb) - 1)).astype(np.int64)
    c = np.concatenate(c + [rc]).astype(np.int64)
    a = np.concatenate(a + [ra]).astype(np.int64)
    b = np.concatenate(b + [rb]).astype(np.int64)
    say("triples", len(c))
    dev = scan.scan_similarity_values(kind, c, a, b)
    if kind == scan.COSINE:
        host = c.astype(np.float64) / np.sqrt(a.astype(np.float64) * b.astype(np.float64))
    else:
        host = c.astype(np.float64) / (a + b - c).astype(np.float64)
    assert np.array_equal(bits(dev), bits(host))


# --------------------------------------------------------------------------
# Small graphs: full index + query grid


def hand_graphs():
    h = json.load(open(os.path.join(GOLDEN, "tiny_hand.json")))["graphs"]
    out = [graphgen.from_edges(v["n"], v["edges"]) for v in h.values()]
    lines = [ln.split("#")[0].strip() for ln in open(os.path.join(GOLDEN, "fig1_consistent.txt"))]
    lines = [ln for ln in lines if ln]
    out.append(graphgen.from_edges(int(lines[0]), [tuple(map(int, ln.split())) for ln in lines[1:]]))
    return out


def test_hand_graphs():
    for g in hand_graphs():
        for kind in (scan.COSINE, scan.JACCARD):
            say("hand graph", g.n, g.nnz, kind)
            gix = gpu_build(g, kind)
            oix = oracle.build_index(g, kind)
            assert_index_equal(gix, oix, g)
            assert_queries_equal(gix, oix, query_grid(oix.dmax, oix.sim))


@pytest.mark.parametrize("n,p", [(8, 0.5), (12, 0.3), (30, 0.2), (60, 0.5), (200, 0.05)])
def test_random_graphs(n, p):
    for seed in range(3):
        g = graphgen.random_graph(n, p, seed=seed + 17 * n)
        kind = seed % 2
        say("random", n, p, seed, g.nnz)
        gix = gpu_build(g, kind, bits=32 if seed % 2 else 64, on_device=seed != 2)
        oix = oracle.build_index(g, kind)
        assert_index_equal(gix, oix, g)
        assert_queries_equal(gix, oix, query_grid(oix.dmax, oix.sim)[::3])


@pytest.mark.parametrize("scale", [8, 11, 14])
@pytest.mark.parametrize("kind", [scan.COSINE, scan.JACCARD])
def test_rmat_small(scale, kind):
    g = graphgen.rmat(scale, 16, seed=scale)
    say("rmat", scale, g.nnz, kind)
    gix = gpu_build(g, kind, bits=32 if kind == 0 else 64)
    oix = oracle.build_index(g, kind, threads=8)
    assert_index_equal(gix, oix, g)
    assert_queries_equal(gix, oix, query_grid(oix.dmax, oix.sim)[::5])


def test_sbm2000_config():
    """2,000 vertices in 20 blocks, p_in 0.1, p_out 0.002, cosine; query
    (5, 0.6) and a sweep over mu in 2..16 and the 17-value eps grid."""
    g = graphgen.sbm2000()
    say("sbm2000", g.nnz)
    gix = gpu_build(g, scan.COSINE)
    oix = oracle.build_index(g, scan.COSINE)
    assert_index_equal(gix, oix, g)
    grid = [(mu, (10 + 5 * k) / 100.0) for mu in range(2, 17) for k in range(17)]
    assert_queries_equal(gix, oix, [(5, 0.6)] + grid)


def test_hub_rows_beyond_one_table_and_big_sorts():
    """Two hubs of degree > 8192 sharing most neighbours (rows split into
    id-range parts), rows > 4096 (merge-path sort passes) and CO segments >
    4096 entries."""
    n = 24000
    rng = np.random.default_rng(5)
    e = [(0, i) for i in range(2, n)] + [(1, i) for i in range(2, n) if i % 3]
    e += [(0, 1)]
    u = rng.integers(2, n, 60000)
    v = rng.integers(2, n, 60000)
    e += list(zip(u.tolist(), v.tolist()))
    g = graphgen.from_edges(n, e)
    say("hubs", g.n, g.nnz, int(g.degrees().max()))
    for kind in (scan.COSINE, scan.JACCARD):
        gix = gpu_build(g, kind)
        oix = oracle.build_index(g, kind, threads=8)
        assert_index_equal(gix, oix, g)
        assert_queries_equal(gix, oix, [(2, 0.1), (3, 0.05), (5, 0.02), (4, 0.3), (2, 0.9)])


def test_complete_and_twins():
    g = graphgen.from_edges(300, [(i, j) for i in range(300) for j in range(i + 1, 300)])
    gix = gpu_build(g)
    oix = oracle.build_index(g)
    assert_index_equal(gix, oix, g)
    assert np.all(export_all(gix)["sim"] == 1.0)
    assert_queries_equal(gix, oix, [(300, 1.0), (301, 1.0), (302, 0.0), (2, 1.0000000000000002)])


def test_empty_and_degenerate_graphs():
    import torch

    for g in [graphgen.from_edges(0, np.zeros((0, 2), np.int32)),
              graphgen.from_edges(7, np.zeros((0, 2), np.int32)),
              graphgen.from_edges(5, [(1, 3)])]:
        say("degenerate", g.n, g.nnz)
        for on_device in (True, False):
            gix = gpu_build(g, on_device=on_device)
            oix = oracle.build_index(g)
            assert gix.info.dmax == oix.dmax
            if g.nnz:
                assert_index_equal(gix, oix, g)
            assert np.array_equal(scan.scan_index_export(gix, scan.ARR_CO_OFF), oix.co_off)
            if g.n:
                for mu, eps in [(2, 0.5), (2, 1.0), (3, 0.0)]:
                    m, _ = scan.scan_query_ex(gix, mu, eps)
                    torch.cuda.synchronize()
                    assert np.array_equal(m.cpu().numpy(), oracle.query(oix, mu, eps)[0])


# --------------------------------------------------------------------------
# Errors, determinism, batch, host outputs, streams


def test_validation_errors():
    bad = {
        "unsorted": (np.array([0, 2, 3, 4]), np.array([2, 1, 0, 0])),
        "self_loop": (np.array([0, 1, 2]), np.array([0, 0])),
        "asymmetric": (np.array([0, 1, 1, 2]), np.array([1, 0])),
        "out_of_range": (np.array([0, 1, 2]), np.array([5, 0])),
        "duplicate": (np.array([0, 2, 3, 4]), np.array([1, 1, 0, 0])),
    }
    for name, (off, adj) in bad.items():
        say("validate", name)
        with pytest.raises(scan.ScanError) as ei:
            scan.scan_build_index(off.astype(np.int64), adj.astype(np.int32), scan.COSINE, scan.SCAN_VALIDATE)
        assert ei.value.status == scan.SCAN_EGRAPH, name
    g = graphgen.rmat(9, 16, seed=1)
    scan.scan_build_index(g.off, g.adj, scan.COSINE, scan.SCAN_VALIDATE)


def test_query_argument_errors():
    g = graphgen.rmat(8, 8, seed=2)
    ix = gpu_build(g)
    for mu, eps in [(1, 0.5), (0, 0.5), (-3, 0.2), (2, float("nan"))]:
        with pytest.raises(scan.ScanError) as ei:
            scan.scan_query(ix, mu, eps)
        assert ei.value.status == scan.SCAN_EINVAL
    with pytest.raises(scan.ScanError):
        scan.scan_query_batch(ix, [2, 1], [0.5, 0.5])
    with pytest.raises(scan.ScanError):
        scan.scan_index_export(gpu_build(g, flags=0), scan.ARR_SIMS)


def test_determinism_and_offset_widths():
    g = graphgen.rmat(13, 16, seed=4)
    a = export_all(gpu_build(g, bits=32))
    b = export_all(gpu_build(g, bits=64))
    c = export_all(gpu_build(g, bits=32, on_device=False))
    for k in a:
        assert np.array_equal(bits(a[k]) if a[k].dtype == np.float64 else a[k],
                              bits(b[k]) if b[k].dtype == np.float64 else b[k]), k
        assert np.array_equal(a[k], c[k]), k


def test_batch_equals_singles_and_host_output():
    import torch

    g = graphgen.rmat(12, 16, seed=9)
    ix = gpu_build(g)
    oix = oracle.build_index(g)
    mus = [2, 3, 5, 8, 16, 2, 5, 40, 3000]
    epss = [0.1, 0.3, 0.6, 0.5, 0.2, 0.9, 0.45, 0.3, 0.1]
    batch = scan.scan_query_batch(ix, mus, epss)
    host = scan.scan_query_batch(ix, mus, epss, out_on_device=False)
    torch.cuda.synchronize()
    batch = batch.cpu().numpy()
    for i, (mu, eps) in enumerate(zip(mus, epss)):
        single = scan.scan_query(ix, mu, eps)
        torch.cuda.synchronize()
        exp = oracle.query(oix, mu, eps)[0]
        assert np.array_equal(single.cpu().numpy(), exp)
        assert np.array_equal(batch[i], exp)
        assert np.array_equal(host[i], exp)
        hm, hc = scan.scan_query_ex(ix, mu, eps, out_on_device=False)
        assert np.array_equal(hm, exp) and np.array_equal(hc, oracle.query(oix, mu, eps)[1])


def test_queries_on_two_streams():
    import torch

    g = graphgen.rmat(12, 16, seed=10)
    ix = gpu_build(g)
    oix = oracle.build_index(g)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = []
    for i in range(6):
        s = s1 if i % 2 else s2
        mu, eps = 2 + i, 0.2 + 0.1 * i
        outs.append((mu, eps, scan.scan_query_ex(ix, mu, eps, stream=s)[0]))
    torch.cuda.synchronize()
    for mu, eps, m in outs:
        assert np.array_equal(m.cpu().numpy(), oracle.query(oix, mu, eps)[0])


def test_query_labels_repeatable():
    """Every core's label is its component's root after pointer jumping, on
    every run: the same queries, repeated, all equal the oracle. (A
    compressing find in the jumping step could overwrite a stored root with
    an ancestor read before it.)"""
    import torch

    g = graphgen.rmat(14, 16, seed=14)
    say("rmat", 14, g.nnz, "repeat")
    gix = gpu_build(g, scan.JACCARD, bits=64)
    oix = oracle.build_index(g, scan.JACCARD, threads=8)
    pairs = query_grid(oix.dmax, oix.sim)[:24]
    want = {p: oracle.query(oix, *p)[0] for p in pairs}
    for rep in range(6):
        for mu, eps in pairs:
            memb, _ = scan.scan_query_ex(gix, mu, eps)
            torch.cuda.synchronize()
            assert np.array_equal(memb.cpu().numpy(), want[(mu, eps)]), (rep, mu, eps)
