"""The allocation-free query entry point (scan_query_noalloc) against
scan_query_ex with device outputs, through the C ABI: two calls in a row on
one stream, the second on a smaller graph (so the shared scratch array holds
the first call's contents), then the first graph again; plus its size limit."""

import numpy as np
import pytest

import graphgen
import paper_2012_11188_amd as scan
from gpu_util import device_csr

pytestmark = pytest.mark.gpu


def _pair(ix, mu, eps):
    import torch

    ref_m, ref_c = scan.scan_query_ex(ix, mu, eps)
    m = torch.full((ix.n,), -7, dtype=torch.int32, device="cuda")
    c = torch.full((ix.n,), 9, dtype=torch.uint8, device="cuda")
    scan.scan_query_noalloc(ix, mu, eps, m, c)
    torch.cuda.synchronize()
    return ref_m.cpu().numpy(), ref_c.cpu().numpy(), m.cpu().numpy(), c.cpu().numpy()


def test_noalloc_matches_query_ex_on_shrinking_inputs():
    import torch

    big = graphgen.sbm(3000, 15, 0.12, 0.003, seed=41)
    small = graphgen.sbm(700, 7, 0.2, 0.01, seed=42)
    ib = scan.scan_build_index(*device_csr(big), scan.COSINE, 0)
    isml = scan.scan_build_index(*device_csr(small), scan.JACCARD, 0)
    torch.cuda.synchronize()
    seen_clusters = 0
    for ix, mu, eps in [(ib, 3, 0.3), (isml, 2, 0.25), (ib, 5, 0.2), (isml, 4, 0.15), (ib, 2, 1.01)]:
        rm, rc, m, c = _pair(ix, mu, eps)
        assert np.array_equal(m, rm), (ix.n, mu, eps)
        assert np.array_equal(c, rc), (ix.n, mu, eps)
        seen_clusters += int((rm >= 0).sum() > 0)
    assert seen_clusters >= 3  # the cases hold real clusters, not only -1


def test_noalloc_without_is_core_and_errors():
    import torch

    g = graphgen.sbm(500, 5, 0.2, 0.01, seed=43)
    ix = scan.scan_build_index(*device_csr(g), scan.COSINE, 0)
    m = torch.empty(g.n, dtype=torch.int32, device="cuda")
    scan.scan_query_noalloc(ix, 3, 0.3, m)
    ref, _ = scan.scan_query_ex(ix, 3, 0.3)
    torch.cuda.synchronize()
    assert np.array_equal(m.cpu().numpy(), ref.cpu().numpy())
    with pytest.raises(scan.ScanError):
        scan.scan_query_noalloc(ix, 1, 0.3, m)  # mu < 2
    # an index over more vertices than the scratch array holds is refused
    n = (1 << 23) + 1
    off = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    adj = torch.zeros(0, dtype=torch.int32, device="cuda")
    huge = scan.scan_build_index(off, adj, scan.COSINE, 0)
    mh = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(scan.ScanError, match="at most"):
        scan.scan_query_noalloc(huge, 2, 0.5, mh)
