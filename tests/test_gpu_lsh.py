"""Parity of the approximate (LSH) build through the C ABI with the oracle:
with the same random draws as inputs, similarity bits, both orders and
queries agree exactly."""

from __future__ import annotations

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


def draws(g, kind, k, seed):
    if kind == scan.JACCARD:
        return None, graphgen.permutation(g.n, seed)
    return graphgen.gaussians(g.n, k, seed), None


def lsh_gpu(g, kind, k, gauss, perm, w=None, on_device=True, bits_=32):
    import torch

    if on_device:
        off, adj = device_csr(g, bits_)
        t = lambda a: None if a is None else torch.from_numpy(a).cuda()
        return scan.scan_build_index_lsh(off, adj, kind, k, t(gauss), t(perm), t(w), FLAGS)
    off = g.off.astype(np.int32 if bits_ == 32 else np.int64)
    return scan.scan_build_index_lsh(off, g.adj.astype(np.int32), kind, k, gauss, perm, w, FLAGS)


def assert_same(gix, oix):
    import torch

    torch.cuda.synchronize()
    for name, code, want in (("sim", scan.ARR_SIMS, oix.sim), ("no_ids", scan.ARR_NO_IDS, oix.no_ids),
                             ("no_sim", scan.ARR_NO_SIM, oix.no_sim), ("co_off", scan.ARR_CO_OFF, oix.co_off),
                             ("co_ids", scan.ARR_CO_IDS, oix.co_ids), ("co_thr", scan.ARR_CO_THR, oix.co_thr)):
        got = scan.scan_index_export(gix, code)
        if got.dtype == np.float64:
            assert np.array_equal(bits(got), bits(want)), name
        else:
            assert np.array_equal(got, want), name


CASES = [
    ("rmat12", scan.COSINE, 64),
    ("rmat12", scan.JACCARD, 64),
    ("rmat12", scan.WEIGHTED_COSINE, 64),
    ("dense", scan.COSINE, 192),
    ("dense", scan.JACCARD, 128),
    ("dense", scan.WEIGHTED_COSINE, 128),
]


def graph(name):
    if name == "rmat12":
        return graphgen.rmat(12, 16, seed=31)
    return graphgen.sbm(600, 2, 0.7, 0.3, seed=32)  # degrees ~300


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_lsh_parity(ci):
    name, kind, k = CASES[ci]
    g = graph(name)
    gauss, perm = draws(g, kind, k, 100 + ci)
    w = graphgen.edge_weights(g, 7) if kind == scan.WEIGHTED_COSINE else None
    okind = scan.JACCARD if kind == scan.JACCARD else scan.COSINE
    oix = oracle.build_index_lsh(g, okind, k, gauss, perm, w, threads=8)
    deg = np.diff(g.off)
    say("lsh parity", name, "kind", kind, "k", k, "high vertices", int((deg > k).sum()))
    gix = lsh_gpu(g, kind, k, gauss, perm, w)
    assert_same(gix, oix)
    for mu, eps in [(2, 0.3), (4, 0.5), (8, 0.6), (3, 0.9)]:
        memb, core = scan.scan_query_ex(gix, mu, eps)
        om, oc = oracle.query(oix, mu, eps)
        assert np.array_equal(memb.cpu().numpy(), om), (mu, eps)
        assert np.array_equal(core.cpu().numpy(), oc), (mu, eps)


@pytest.mark.parametrize("kind", [scan.COSINE, scan.JACCARD])
def test_lsh_host_inputs_and_int64(kind):
    g = graph("dense")
    k = 128
    gauss, perm = draws(g, kind, k, 5)
    oix = oracle.build_index_lsh(g, kind, k, gauss, perm, threads=8)
    say("lsh host inputs kind", kind)
    assert_same(lsh_gpu(g, kind, k, gauss, perm, on_device=False, bits_=64), oix)


def test_lsh_without_high_vertices_is_exact():
    import torch

    g = graphgen.sbm(500, 5, 0.1, 0.01, seed=2)  # degrees far below 64
    gauss, _ = draws(g, scan.COSINE, 64, 1)
    a = lsh_gpu(g, scan.COSINE, 64, gauss, None)
    off, adj = device_csr(g)
    b = scan.scan_build_index(off, adj, scan.COSINE, FLAGS)
    torch.cuda.synchronize()
    for code in (scan.ARR_SIMS, scan.ARR_NO_IDS, scan.ARR_CO_IDS, scan.ARR_CO_THR):
        assert np.array_equal(scan.scan_index_export(a, code).view(np.uint8),
                              scan.scan_index_export(b, code).view(np.uint8))


def _c_build_lsh(off, adj, kind, samples, gauss=None, perm=None, weights=None, flags=0):
    """scan_build_index_lsh called through the C ABI directly (no binding
    checks): returns the status."""
    import ctypes

    lib = scan.load_library()
    c, keep = scan._csr_struct(off, adj)
    ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
    spec = scan._Lsh(int(samples), 0, ptr(gauss), ptr(perm), ptr(weights))
    out = ctypes.c_void_p()
    st = lib.scan_build_index_lsh(ctypes.byref(c), int(kind), ctypes.byref(spec), int(flags), None, ctypes.byref(out))
    if st == scan.SCAN_OK:
        lib.scan_index_free(out)
    return st


def test_lsh_errors():
    import torch

    g = graph("dense")
    off, adj = device_csr(g)
    gauss = torch.from_numpy(graphgen.gaussians(g.n, 64, 1)).cuda()
    perm = torch.from_numpy(graphgen.permutation(g.n, 1)).cuda()
    w = torch.from_numpy(graphgen.edge_weights(g, 1)).cuda()
    for k in (0, 100, 8192):  # draws of the matching size: the library rejects k itself
        gk = torch.zeros(g.n * k, dtype=torch.float64, device="cuda")
        with pytest.raises(scan.ScanError, match="EINVAL"):
            scan.scan_build_index_lsh(off, adj, scan.COSINE, k, gauss=gk)
    # missing or misplaced draws and weights: the binding refuses them before
    # the library is called, and the library refuses them too
    for kind, kw in [(scan.COSINE, {"perm": perm}), (scan.JACCARD, {"gauss": gauss}),
                     (scan.JACCARD, {"perm": perm, "weights": w}), (scan.WEIGHTED_COSINE, {"gauss": gauss})]:
        with pytest.raises(ValueError):
            scan.scan_build_index_lsh(off, adj, kind, 64, **kw)
        assert _c_build_lsh(off, adj, kind, 64, **kw) == scan.SCAN_EINVAL
    with pytest.raises(scan.ScanError, match="EINVAL"):
        scan.scan_build_index_lsh(off, adj, scan.COSINE, 64, gauss=gauss, flags=scan.SCAN_KEEP_COUNTS)
    bad = perm.clone()
    bad[3] = g.n
    with pytest.raises(scan.ScanError, match="EINVAL"):
        scan.scan_build_index_lsh(off, adj, scan.JACCARD, 64, perm=bad)
    assert _c_build_lsh(off, adj, scan.COSINE, 64, gauss=gauss) == scan.SCAN_OK


@pytest.mark.parametrize("kind", [scan.COSINE, scan.JACCARD])
def test_lsh_rmat20_sampled(kind):
    """R-MAT-20 with k = 256: sampled approximated and exact edges against
    the oracle one by one, and the neighbour order's invariant."""
    import torch

    g = graphgen.rmat20()
    k = 256
    gauss, perm = draws(g, kind, k, 20)
    say("lsh rmat20 kind", kind)
    gix = lsh_gpu(g, kind, k, gauss, perm)
    torch.cuda.synchronize()
    sim = scan.scan_index_export(gix, scan.ARR_SIMS)
    deg = np.diff(g.off)
    rows = np.repeat(np.arange(g.n), deg)
    hi = (deg > k) if kind == scan.COSINE else (2 * deg > 3 * k)
    both = hi[rows] & hi[g.adj]
    rng = np.random.default_rng(3)
    pick = np.concatenate([rng.choice(np.flatnonzero(both), 400, replace=False),
                           rng.choice(np.flatnonzero(~both), 200, replace=False)])
    want = oracle.lsh_edge_similarities(g, kind, k, rows[pick], g.adj[pick], gauss, perm)
    assert np.array_equal(bits(sim[pick]), bits(want))
    no_ids = scan.scan_index_export(gix, scan.ARR_NO_IDS)
    no_sim = scan.scan_index_export(gix, scan.ARR_NO_SIM)
    same = rows[1:] == rows[:-1]
    d = np.diff(no_sim)
    assert np.all(~same | (d < 0) | ((d == 0) & (np.diff(no_ids) > 0)))


def test_lsh_weighted_host_inputs_int64_validated():
    # weighted SimHash with every input on the host, 64-bit offsets and the
    # CSR and weight checks switched on
    g = graph("dense")
    k = 128
    gauss, _ = draws(g, scan.COSINE, k, 77)
    w = graphgen.edge_weights(g, 78)
    oix = oracle.build_index_lsh(g, scan.COSINE, k, gauss, None, w, threads=8)
    say("weighted SimHash, host inputs, int64, validated")
    off = g.off.astype(np.int64)
    gix = scan.scan_build_index_lsh(off, g.adj.astype(np.int32), scan.WEIGHTED_COSINE, k, gauss, None, w,
                                    FLAGS | scan.SCAN_VALIDATE)
    assert_same(gix, oix)
