"""Builds return before the device has finished them (inside the call the
host waits only for the small read-backs that size the grids), builds on two
streams overlap on the device, and the indexes built that way equal, bit for
bit, the ones built one at a time (and the oracle's, on a graph it can
build)."""

from __future__ import annotations

import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_11188_amd as scan
from gpu_util import assert_index_equal, bits, device_csr, export_all

pytestmark = pytest.mark.gpu

FLAGS = scan.SCAN_KEEP_SIMS | scan.SCAN_KEEP_COUNTS


def arrays(ix):
    return {k: (bits(v) if v.dtype == np.float64 else v) for k, v in export_all(ix).items()}


def assert_same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_two_streams_return_early_overlap_and_match():
    import torch

    ga, gb = graphgen.rmat20(), graphgen.rmat(19, 16, seed=77)
    da, db = device_csr(ga, 64), device_csr(gb, 64)
    print(f"graphs: nnz {ga.nnz} and {gb.nnz}", flush=True)
    # one build at a time, each finished before the next starts
    ref_a = arrays(scan.scan_build_index(*da, scan.COSINE, FLAGS))
    ref_b = arrays(scan.scan_build_index(*db, scan.JACCARD, FLAGS))
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    # one untimed build per stream first: the caching allocator then holds
    # blocks for each stream, so the measured calls allocate nothing new
    for st, (d, kind) in ((sa, (da, scan.COSINE)), (sb, (db, scan.JACCARD))):
        with torch.cuda.stream(st):
            scan.scan_build_index(*d, kind, FLAGS).free()
    a_end = torch.cuda.Event(enable_timing=True)
    b_start = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(sa):
        ix_a = scan.scan_build_index(*da, scan.COSINE, FLAGS)
        busy = not sa.query()
        a_end.record()
    with torch.cuda.stream(sb):
        b_start.record()
        ix_b = scan.scan_build_index(*db, scan.JACCARD, FLAGS)
    torch.cuda.synchronize()
    lead = b_start.elapsed_time(a_end)
    print(f"second build started {lead:.3f} ms before the first ended", flush=True)
    assert busy, "the build call returned only after the device had finished"
    assert lead > 0, "the second build started only after the first had ended"
    assert_same(arrays(ix_a), ref_a)
    assert_same(arrays(ix_b), ref_b)


def test_free_before_finish_and_host_inputs():
    """Indexes freed while their build may still run, and host inputs
    overwritten right after the call, leave later builds exact."""
    import torch

    g = graphgen.rmat(14, 16, seed=5)
    oix = oracle.build_index(g, oracle.COSINE, threads=8)
    for rep in range(4):
        ix = scan.scan_build_index(*device_csr(g, 32 if rep % 2 else 64), scan.COSINE, FLAGS)
        ix.free()
    off, adj = g.off.astype(np.int64), g.adj.copy()
    ix = scan.scan_build_index(off, adj, scan.COSINE, FLAGS)
    off[:] = 0
    adj[:] = 0
    del off, adj
    torch.cuda.synchronize()
    assert_index_equal(ix, oix, g)


def test_batches_on_two_streams_with_profiling():
    """Merged builds (several graphs, tables uploaded on a helper stream, ids
    made local per graph) enqueued on two streams back to back, profiled,
    with the first batch's indexes freed before the device has finished:
    every index of the second batch equals the oracle's."""
    import torch

    gs = [graphgen.rmat(12, 16, seed=40 + i) for i in range(3)] + [graphgen.sbm(3000, 6, 0.04, 0.002, seed=7)]
    oix = [oracle.build_index(g, oracle.JACCARD, threads=8) for g in gs]
    dev = [device_csr(g, 64 if i % 2 else 32) for i, g in enumerate(gs)]
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    flags = FLAGS | scan.SCAN_PROFILE
    with torch.cuda.stream(sa):
        first = scan.scan_build_index_batch(dev[::-1], scan.JACCARD, flags, stream=sa)
    with torch.cuda.stream(sb):
        second = scan.scan_build_index_batch(dev, scan.JACCARD, flags, stream=sb)
    for ix in first:
        ix.free()
    torch.cuda.synchronize()
    for g, o, ix in zip(gs, oix, second):
        p = scan.scan_index_build_profile(ix)
        assert p["total_ms"] > 0
        assert_index_equal(ix, o, g)
