"""Full-size parity: the R-MAT scale-20 cosine index (the benchmark workload,
int32 offsets, device-resident CSR, default kernel configuration) compared
bit for bit with the oracle's full build, plus queries."""

from __future__ import annotations

import os

import numpy as np
import pytest

import graphgen
import oracle
import paper_2012_11188_amd as scan
from gpu_util import assert_index_equal, gpu_build

pytestmark = pytest.mark.gpu


def test_rmat20_full_index_and_queries():
    import torch

    g = graphgen.rmat20()
    print("rmat20", g.n, g.nnz, flush=True)
    gix = gpu_build(g, scan.COSINE, bits=32, on_device=True)
    torch.cuda.synchronize()
    threads = min(16, os.cpu_count() or 1)
    oix = oracle.build_index(g, oracle.COSINE, threads=threads)
    print("oracle built", flush=True)
    assert_index_equal(gix, oix, g)
    for mu, eps in [(5, 0.6), (2, 0.3), (16, 0.1), (3, 0.9), (50, 0.2)]:
        memb, core = scan.scan_query_ex(gix, mu, eps)
        torch.cuda.synchronize()
        om, oc = oracle.query(oix, mu, eps)
        assert np.array_equal(memb.cpu().numpy(), om), (mu, eps)
        assert np.array_equal(core.cpu().numpy(), oc), (mu, eps)
