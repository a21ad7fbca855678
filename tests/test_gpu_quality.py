"""Modularity on the HIP path (Section 7.2, unclustered vertices as
singletons as in Section 7.3.4) and the paper's parameter sweep, through the C
ABI: device values equal the oracle's bit for bit (both accumulate the two
integer terms exactly and finish with the same two FP64 divisions)."""

from __future__ import annotations

import os

import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_11188_amd as scan
from gpu_util import gpu_build

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_edge_fixture(name):
    lines = [ln.split("#")[0].strip() for ln in open(os.path.join(GOLDEN, name))]
    lines = [ln for ln in lines if ln]
    return graphgen.from_edges(int(lines[0]), [tuple(map(int, ln.split())) for ln in lines[1:]])


def graphs():
    return {"hand": load_edge_fixture("hub_outlier_hand.txt"), "fig1": load_edge_fixture("fig1_consistent.txt"),
            "sbm2000": graphgen.sbm2000(), "rmat13": graphgen.rmat(13, 16, seed=5)}


@pytest.mark.parametrize("name", ["hand", "fig1", "sbm2000", "rmat13"])
def test_modularity_parity(name):
    import torch

    g = graphs()[name]
    gix = gpu_build(g)
    oix = oracle.build_index(g, oracle.COSINE, threads=8)
    grid = [(mu, (10 + 5 * k) / 100.0) for mu in (2, 3, 4, 6, 9) for k in range(0, 17, 3)]
    for mu, eps in grid:
        memb, _ = scan.scan_query_ex(gix, mu, eps)
        q = scan.scan_query_modularity(gix, memb)
        torch.cuda.synchronize()
        om, _ = oracle.query(oix, mu, eps)
        want = oracle.modularity(g, om)[0]
        assert np.float64(q).tobytes() == np.float64(want).tobytes(), (name, mu, eps, q, want)


def test_sweep_equals_single_queries():
    g = graphgen.sbm2000()
    gix = gpu_build(g)
    oix = oracle.build_index(g, oracle.COSINE, threads=8)
    grid = [p for p in scan.paper_sweep_grid(int(g.degrees().max())) if int(p[1] * 100) % 7 == 0]
    mus = np.array([m for m, _ in grid], np.int32)
    epss = np.array([e for _, e in grid])
    for batch in (1, 5, 32):
        q = scan.scan_sweep_modularity(gix, mus, epss, batch=batch)
        for i, (mu, eps) in enumerate(grid):
            om, _ = oracle.query(oix, int(mu), float(eps))
            want = oracle.modularity(g, om)[0]
            assert q[i].tobytes() == np.float64(want).tobytes(), (batch, mu, eps)
    best = int(np.argmax(q))
    assert q[best] > 0.0  # SBM-2000's planted blocks are found somewhere on the grid


def test_quality_errors():
    import torch

    g = load_edge_fixture("hub_outlier_hand.txt")
    gix = gpu_build(g)
    bad = torch.full((g.n,), g.n, dtype=torch.int32, device="cuda")  # label out of range
    with pytest.raises(scan.ScanError):
        scan.scan_query_modularity(gix, bad)
    with pytest.raises(scan.ScanError):
        scan.scan_sweep_modularity(gix, np.array([1], np.int32), np.array([0.5]))  # mu < 2
    with pytest.raises(scan.ScanError):
        scan.scan_sweep_modularity(gix, np.array([2], np.int32), np.array([0.5]), batch=0)
