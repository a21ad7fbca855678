"""Intersection shapes: every scan_tune setting (small/large owner threshold,
chunk size, bitmap window, including windows far smaller than the id space so
that chunks sweep several windows) gives the oracle's index bit for bit; the
autotuner returns a setting that does too."""

from __future__ import annotations

import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_11188_amd as scan
from gpu_util import assert_index_equal, assert_queries_equal, device_csr

pytestmark = pytest.mark.gpu

FLAGS = scan.SCAN_KEEP_SIMS | scan.SCAN_KEEP_COUNTS

TUNES = [
    None,
    {"wbits": 10},                              # several windows per chunk (tabled ranges)
    {"wbits": 10, "flags": scan.SCAN_TUNE_SEARCH_WINDOWS},  # ... ranges searched per window
    {"wbits": 11, "spc": 1024},
    {"small_max": 1},                           # almost every owner takes the bitmap path
    {"small_max": 4096},                        # every owner up to degree 4096 takes the wave path
    {"spc": 1},                                 # one row slot per chunk
    {"small_max": 32, "spc": 128, "wbits": 12},
]


@pytest.fixture(scope="module")
def graphs():
    gs = [graphgen.rmat(13, 16, seed=3), graphgen.sbm(5000, 8, 0.03, 0.002, seed=4),
          graphgen.rmat(11, 32, seed=8)]
    return [(g, {k: oracle.build_index(g, k, threads=8) for k in (oracle.COSINE, oracle.JACCARD)}) for g in gs]


@pytest.mark.parametrize("ti", range(len(TUNES)))
def test_tune_invariance(graphs, ti):
    import torch

    tune = TUNES[ti]
    for gi, (g, oix) in enumerate(graphs):
        for kind in (scan.COSINE, scan.JACCARD):
            print("tune", tune, "graph", gi, "kind", kind, flush=True)
            ix = scan.scan_build_index(*device_csr(g, 64 if gi % 2 else 32), kind, FLAGS, tune=tune)
            torch.cuda.synchronize()
            assert_index_equal(ix, oix[kind], g)
            if kind == scan.COSINE:
                assert_queries_equal(ix, oix[kind], [(2, 0.4), (4, 0.6), (8, 0.3)])


def test_tune_batch_multiwindow(graphs):
    import torch

    gs = [g for g, _ in graphs]
    ixs = scan.scan_build_index_batch([device_csr(g) for g in gs], scan.COSINE, FLAGS, tune={"wbits": 10, "spc": 64})
    torch.cuda.synchronize()
    for (g, oix), ix in zip(graphs, ixs):
        assert_index_equal(ix, oix[scan.COSINE], g)


def test_tune_errors(graphs):
    g = graphs[0][0]
    for bad in ({"small_max": 5000}, {"spc": 2048}, {"wbits": 9}, {"wbits": 25}, {"small_max": -1}, {"flags": 2}):
        with pytest.raises(scan.ScanError) as ei:
            scan.scan_build_index(*device_csr(g), scan.COSINE, 0, tune=bad)
        assert ei.value.status == scan.SCAN_EINVAL, bad
    with pytest.raises(ValueError):
        scan.scan_build_index(*device_csr(g), scan.COSINE, 0, tune={"tile": 3})


def test_autotune(graphs):
    import torch

    g, oix = graphs[0]
    best = scan.scan_autotune([device_csr(g)], scan.COSINE, reps=1)
    print("autotune", best, flush=True)
    assert 1 <= best["small_max"] <= 4096 and 1 <= best["spc"] <= 1024 and 10 <= best["wbits"] <= 24
    assert best["ms"] > 0
    tune = {k: best[k] for k in ("small_max", "spc", "wbits")}
    ix = scan.scan_build_index(*device_csr(g), scan.COSINE, FLAGS, tune=tune)
    torch.cuda.synchronize()
    assert_index_equal(ix, oix[scan.COSINE], g)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tune_tiny_bitmap_owners(seed):
    """Graphs whose whole adjacency is shorter than one work item of the
    bitmap owners (the rows near the end of the adjacency are read through
    its padded tail copy), with every owner of degree >= 2 on that path."""
    import torch

    g = graphgen.random_graph(40 + 10 * seed, 0.2, seed=seed)
    assert g.nnz < 1024
    for kind in (scan.COSINE, scan.JACCARD):
        oix = oracle.build_index(g, kind, threads=1)
        ix = scan.scan_build_index(*device_csr(g), kind, FLAGS, tune={"small_max": 1, "spc": 4})
        torch.cuda.synchronize()
        assert_index_equal(ix, oix, g)


def test_window_table_long_rows():
    """Rows longer than the window table's streaming limit (2,048 ids), with
    ids over many bitmap windows: two hubs whose rows cross every window
    boundary, one whose ids skip most windows (empty ranges between and
    after), and a sparse background, at 10-bit windows (12 of them)."""
    import torch

    rng = np.random.default_rng(2012)
    n = 12_000
    edges = set()
    def add(u, v):
        if u != v:
            edges.add((min(u, v), max(u, v)))
    for h, m in ((0, 5000), (7000, 3000)):  # rows of 5,000 and 3,000 ids across all windows
        for v in rng.choice(n, size=m, replace=False):
            add(h, int(v))
    for v in np.concatenate([rng.choice(2048, size=1900, replace=False), rng.choice(1024, size=900, replace=False) + 9 * 1024]):
        add(11_999, int(v))  # ids in windows 0, 1 and 9 only
    for u, v in rng.integers(0, n, size=(40_000, 2)):
        add(int(u), int(v))
    g = graphgen.from_edges(n, sorted(edges))
    assert (np.diff(g.off) > 2048).sum() == 3
    for kind in (scan.COSINE, scan.JACCARD):
        oix = oracle.build_index(g, kind, threads=8)
        for tune in ({"wbits": 10, "spc": 256}, {"wbits": 10, "spc": 64, "small_max": 16}, {"wbits": 11}):
            print("kind", kind, "tune", tune, flush=True)
            ix = scan.scan_build_index(*device_csr(g, 64), kind, FLAGS, tune=tune)
            torch.cuda.synchronize()
            assert_index_equal(ix, oix, g)
