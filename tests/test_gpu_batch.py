"""Batched multi-graph build: every graph's index from one merged build equals
the oracle's index of that graph (bit for bit) and the single-graph build."""

from __future__ import annotations

import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_11188_amd as scan
from gpu_util import assert_index_equal, assert_queries_equal, bits, device_csr, export_all

pytestmark = pytest.mark.gpu


def mixed_graphs():
    return [
        graphgen.sbm(1500, 10, 0.08, 0.002, seed=1),
        graphgen.from_edges(0, np.zeros((0, 2), np.int32)),
        graphgen.rmat(10, 16, seed=5),
        graphgen.from_edges(6, np.zeros((0, 2), np.int32)),
        graphgen.random_graph(40, 0.3, seed=2),
        graphgen.sbm(3000, 4, 0.05, 0.001, seed=3),
        graphgen.from_edges(3, [(0, 1), (1, 2)]),
        graphgen.rmat(12, 8, seed=7),
    ]


def test_batch_matches_oracle_and_singles():
    import torch

    gs = mixed_graphs()
    args = []
    for i, g in enumerate(gs):
        bits_ = 32 if i % 2 else 64
        if i % 3 == 2:  # some host-resident
            args.append((g.off.astype(np.int32 if bits_ == 32 else np.int64), g.adj.astype(np.int32)))
        else:
            args.append(device_csr(g, bits_))
    flags = scan.SCAN_KEEP_SIMS | scan.SCAN_KEEP_COUNTS
    for kind in (scan.COSINE, scan.JACCARD):
        print("batch", len(gs), "kind", kind, flush=True)
        ixs = scan.scan_build_index_batch(args, kind, flags)
        torch.cuda.synchronize()
        assert len(ixs) == len(gs)
        for g, ix in zip(gs, ixs):
            oix = oracle.build_index(g, kind)
            assert ix.info.n == g.n and ix.info.nnz == g.nnz and ix.info.dmax == oix.dmax
            assert np.array_equal(scan.scan_index_export(ix, scan.ARR_OFFSETS), g.off.astype(np.int64))
            assert np.array_equal(scan.scan_index_export(ix, scan.ARR_CO_OFF), oix.co_off)
            if g.nnz:
                assert_index_equal(ix, oix, g)
                single = scan.scan_build_index(*device_csr(g), kind, flags)
                a, b = export_all(ix), export_all(single)
                for k in a:
                    assert np.array_equal(bits(a[k]) if a[k].dtype == np.float64 else a[k],
                                          bits(b[k]) if b[k].dtype == np.float64 else b[k]), k
            if g.n:
                assert_queries_equal(ix, oix, [(2, 0.3), (3, 0.5), (5, 0.2), (2, 0.9)])


def test_uneven_sbm_batch():
    import torch

    gs = graphgen.batch_sbm(24, seed=11, n_hi=20000.0)
    ixs = scan.scan_build_index_batch([device_csr(g) for g in gs], scan.COSINE, scan.SCAN_KEEP_SIMS | scan.SCAN_KEEP_COUNTS)
    torch.cuda.synchronize()
    for g, ix in zip(gs, ixs):
        print(g.name, g.nnz, flush=True)
        oix = oracle.build_index(g, oracle.COSINE, threads=8)
        assert_index_equal(ix, oix, g)
        assert_queries_equal(ix, oix, [(5, 0.6), (3, 0.3)])


def test_batch_errors_and_free_order():
    import torch

    g = graphgen.rmat(8, 8, seed=3)
    bad_off = np.array([0, 1, 1, 2], np.int64)  # 0->1 and 2->0 without their mirrors
    with pytest.raises(scan.ScanError) as ei:
        scan.scan_build_index_batch([device_csr(g), (bad_off, np.array([1, 0], np.int32))], scan.COSINE,
                                    scan.SCAN_VALIDATE)
    assert ei.value.status == scan.SCAN_EGRAPH
    ixs = scan.scan_build_index_batch([device_csr(g), device_csr(g)], scan.COSINE)
    torch.cuda.synchronize()
    first = scan.scan_index_export(ixs[1], scan.ARR_NO_IDS)
    ixs[0].free()  # views into the shared buffers stay valid
    assert np.array_equal(scan.scan_index_export(ixs[1], scan.ARR_NO_IDS), first)
    m = scan.scan_query(ixs[1], 2, 0.5)
    torch.cuda.synchronize()
    assert np.array_equal(m.cpu().numpy(), oracle.query(oracle.build_index(g), 2, 0.5)[0])


@pytest.mark.timeout(900)
def test_sbm256_full_config_every_graph():
    """The batched-build workload itself: 256 uneven SBM graphs (n log-uniform
    in [1e3, 2e5], 5-200 blocks, average degree 8-64, p_out / p_in = 0.02),
    built in one merged build; every graph's index equals the oracle's, bit for
    bit, and two queries per graph equal the oracle's."""
    import os
    import time
    from concurrent.futures import ThreadPoolExecutor

    import torch

    t = time.time()
    gs = graphgen.batch_sbm(256)
    print(f"256 graphs, sum nnz {sum(g.nnz for g in gs)}, generated in {time.time() - t:.1f}s", flush=True)
    dev = [device_csr(g, 64) for g in gs]
    t = time.time()
    ixs = scan.scan_build_index_batch(dev, scan.COSINE, scan.SCAN_KEEP_SIMS | scan.SCAN_KEEP_COUNTS)
    torch.cuda.synchronize()
    print(f"merged build {time.time() - t:.2f}s", flush=True)
    del dev
    threads = min(16, os.cpu_count() or 1)
    t = time.time()
    with ThreadPoolExecutor(threads) as ex:  # the oracle's C calls release the GIL
        futs = [ex.submit(oracle.build_index, g, oracle.COSINE, 1) for g in gs]
        for i, (g, ix, f) in enumerate(zip(gs, ixs, futs)):
            oix = f.result()
            assert_index_equal(ix, oix, g)
            assert_queries_equal(ix, oix, [(5, 0.6), (3, 0.3)])
            if i % 32 == 31:
                print(f"graphs 0..{i} equal ({time.time() - t:.1f}s)", flush=True)
