"""Continuous-batching server: every result equals the oracle's clustering for
its (mu, eps), whether it ran alone or inside a mixed batch, with and without
HIP graph replay, under concurrent submitters and queue back-pressure."""

from __future__ import annotations

import threading

import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_11188_amd as scan
from gpu_util import gpu_build

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served():
    g = graphgen.sbm(4000, 16, 0.06, 0.002, seed=41)
    ix = gpu_build(g)
    oix = oracle.build_index(g, oracle.COSINE, threads=8)
    return g, ix, oix


def mixed_requests(k, seed):
    rng = np.random.default_rng(seed)
    mus = rng.integers(2, 17, size=k)
    epss = rng.choice(np.round(np.arange(0.05, 1.0001, 0.05), 2), size=k)
    return [(int(m), float(e)) for m, e in zip(mus, epss)]


def expected(oix, reqs):
    cache = {}
    for r in reqs:
        if r not in cache:
            cache[r] = oracle.query(oix, *r)[0]
    return cache


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("slots,batch", [(1, 1), (16, 4), (32, 32)])
def test_server_results(served, use_graph, slots, batch):
    g, ix, oix = served
    reqs = mixed_requests(60, seed=slots * 7 + batch + int(use_graph))
    want = expected(oix, reqs)
    print("server", slots, batch, use_graph, flush=True)
    srv = scan.Server(ix, max_slots=slots, max_batch=batch, memory_budget=1 << 30, use_graph=use_graph)
    try:
        # alone: submit and wait one by one
        for r in reqs[:5]:
            dst = np.full(g.n, -7, np.int32)
            srv.wait(srv.submit(*r, dst))
            assert np.array_equal(dst, want[r]), r
        # in the mix: everything at once; results go to HBM, pinned host
        # memory (written by the device directly) or pageable host memory
        import torch

        def dst_for(i):
            if i % 3 == 1:
                return torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
            if i % 3 == 2:
                return torch.full((g.n,), -7, dtype=torch.int32).pin_memory().numpy()
            return np.full(g.n, -7, np.int32)

        dsts = [dst_for(i) for i in range(len(reqs))]
        lat = np.full(len(reqs), -1.0)
        torch.cuda.synchronize()
        tickets = [srv.submit_ex(*r, d, lat.ctypes.data + 8 * i) for i, (r, d) in enumerate(zip(reqs, dsts))]
        for t in tickets:
            srv.wait(t)
        for r, d in zip(reqs, dsts):
            got = d.cpu().numpy() if isinstance(d, torch.Tensor) else d
            assert np.array_equal(got, want[r]), r
        assert (lat > 0).all() and (lat < 60e3).all()
    finally:
        srv.close()


def test_server_concurrent_submitters_and_backpressure(served):
    g, ix, oix = served
    srv = scan.Server(ix, max_slots=8, max_batch=4, memory_budget=1 << 30, use_graph=True)
    errors = []
    busy = [0]

    def worker(seed):
        try:
            reqs = mixed_requests(40, seed)
            want = expected(oix, reqs)
            dsts = [np.empty(g.n, np.int32) for _ in reqs]
            tickets = []
            for r, d in zip(reqs, dsts):
                while True:
                    t = srv.try_submit(*r, d)
                    if t is not None:
                        break
                    busy[0] += 1
                    if tickets:
                        srv.wait(tickets[0])
                tickets.append(t)
            done = 0
            while done < len(tickets):  # poll until all complete
                done = sum(srv.poll(t) for t in tickets)
                if done < len(tickets):
                    srv.wait(tickets[-1])
            for r, d in zip(reqs, dsts):
                if not np.array_equal(d, want[r]):
                    errors.append(r)
        except Exception as e:  # noqa: BLE001
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(100 + i,)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    srv.close()
    assert not errors, errors[:5]


def test_server_budget_and_errors(served):
    g, ix, _ = served
    with pytest.raises(scan.ScanError) as ei:
        scan.Server(ix, max_slots=4, max_batch=2, memory_budget=1000)
    assert ei.value.status == scan.SCAN_ENOMEM
    with pytest.raises(scan.ScanError) as ei:
        scan.Server(ix, max_slots=0, max_batch=2)
    assert ei.value.status == scan.SCAN_EINVAL
    # a budget for 3 slots keeps 3 of the 64 requested
    srv = scan.Server(ix, max_slots=64, max_batch=64, memory_budget=3 * (9 * g.n + 64))
    try:
        with pytest.raises(scan.ScanError) as ei:
            srv.submit(1, 0.5, np.empty(g.n, np.int32))
        assert ei.value.status == scan.SCAN_EINVAL
        with pytest.raises(scan.ScanError):
            srv.submit(2, float("nan"), np.empty(g.n, np.int32))
        d = np.empty(g.n, np.int32)
        srv.wait(srv.submit(3, 0.4, d))
        assert np.array_equal(d, oracle.query(served[2], 3, 0.4)[0])
    finally:
        srv.close()


def test_server_drains_on_close(served):
    g, ix, oix = served
    srv = scan.Server(ix, max_slots=4, max_batch=2, use_graph=False)
    reqs = mixed_requests(30, seed=9)
    dsts = [np.full(g.n, -1, np.int32) for _ in reqs]
    for r, d in zip(reqs, dsts):
        srv.submit(*r, d)
    srv.close()  # returns after every queued request has been delivered
    want = expected(oix, reqs)
    for r, d in zip(reqs, dsts):
        assert np.array_equal(d, want[r]), r


def test_server_empty_graph():
    g = graphgen.from_edges(5, np.zeros((0, 2), np.int32))
    ix = gpu_build(g)
    srv = scan.Server(ix, max_slots=2, max_batch=2)
    try:
        d = np.full(5, 9, np.int32)
        srv.wait(srv.submit(2, 0.5, d))
        assert np.array_equal(d, oracle.query(oracle.build_index(g), 2, 0.5)[0])
    finally:
        srv.close()
