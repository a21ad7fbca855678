"""Hubs and outliers (Section 4.3) on the HIP path, through the C ABI: the
roles computed on the device from a query's memberships equal the oracle's
roles of the oracle's memberships, exactly, over (mu, eps) grids on seeded
graphs (the hand-worked fixture, a graph consistent with the paper's Figure 1,
SBM-2000 and R-MAT graphs with hub rows longer than one wavefront step)."""

from __future__ import annotations

import os

import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_11188_amd as scan
from gpu_util import gpu_build, query_grid

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_edge_fixture(name):
    lines = [ln.split("#")[0].strip() for ln in open(os.path.join(GOLDEN, name))]
    lines = [ln for ln in lines if ln]
    return graphgen.from_edges(int(lines[0]), [tuple(map(int, ln.split())) for ln in lines[1:]])


def check_roles(g, pairs, kind=scan.COSINE):
    import torch

    gix = gpu_build(g, kind)
    oix = oracle.build_index(g, kind, threads=8)
    hubs = 0
    for mu, eps in pairs:
        memb, _ = scan.scan_query_ex(gix, mu, eps)
        roles = scan.scan_query_roles(gix, memb)
        torch.cuda.synchronize()
        om, _ = oracle.query(oix, mu, eps)
        want = oracle.roles(g, om)
        got = roles.cpu().numpy()
        assert np.array_equal(memb.cpu().numpy(), om), (mu, eps)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, f"(mu, eps) = ({mu}, {eps}): {bad.size} roles differ, first vertex {bad[0]}"
        hubs += int((want == oracle.ROLE_HUB).sum())
    return hubs


@pytest.mark.parametrize("name", ["hub_outlier_hand.txt", "fig1_consistent.txt"])
def test_roles_fixtures(name):
    g = load_edge_fixture(name)
    pairs = [(mu, eps) for mu in (2, 3, 4, 5) for eps in (0.3, 0.5, 0.6, 0.7, 0.9, 1.0)]
    assert check_roles(g, pairs) > 0  # both fixtures have a hub at some (mu, eps)


def test_roles_sbm2000():
    g = graphgen.sbm2000()
    pairs = [(mu, (10 + 5 * k) / 100.0) for mu in (2, 3, 5, 8) for k in range(0, 17, 2)]
    check_roles(g, pairs)


@pytest.mark.parametrize("kind", [scan.COSINE, scan.JACCARD])
def test_roles_rmat(kind):
    g = graphgen.rmat(13, 16, seed=5)
    assert g.degrees().max() > 64  # rows span several wavefront steps
    oix_sim = oracle.similarities(g, kind, threads=8)[1]
    pairs = query_grid(int(g.degrees().max()), oix_sim)[::3]
    assert check_roles(g, pairs, kind) > 0


def test_roles_errors():
    import torch

    g = load_edge_fixture("hub_outlier_hand.txt")
    gix = gpu_build(g)
    with pytest.raises(ValueError):
        scan.scan_query_roles(gix, torch.zeros(g.n, dtype=torch.int64, device="cuda"))
    with pytest.raises(scan.ScanError):
        scan._check(scan.load_library().scan_query_roles(gix._h, None, None, None))
