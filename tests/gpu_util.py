"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the oracle (inputs come from graphgen; expected values come from
the oracle or from properties, never from the GPU path)."""

from __future__ import annotations

import numpy as np

import oracle
import paper_2012_11188_amd as scan

ARRAYS = {
    "no_ids": scan.ARR_NO_IDS, "no_sim": scan.ARR_NO_SIM, "co_off": scan.ARR_CO_OFF,
    "co_ids": scan.ARR_CO_IDS, "co_thr": scan.ARR_CO_THR, "sim": scan.ARR_SIMS,
    "counts": scan.ARR_COUNTS,
}


def device_csr(g, bits=32):
    import torch

    off = torch.from_numpy(g.off.astype(np.int32 if bits == 32 else np.int64)).cuda()
    adj = torch.from_numpy(g.adj.astype(np.int32)).cuda()
    return off, adj


def gpu_build(g, kind=scan.COSINE, bits=32, on_device=True, flags=scan.SCAN_KEEP_SIMS | scan.SCAN_KEEP_COUNTS):
    if on_device:
        off, adj = device_csr(g, bits)
    else:
        off = g.off.astype(np.int32 if bits == 32 else np.int64)
        adj = g.adj.astype(np.int32)
    return scan.scan_build_index(off, adj, kind, flags)


def export_all(ix, keep=("sim", "counts")):
    out = {}
    for name, code in ARRAYS.items():
        if name in ("sim", "counts") and name not in keep:
            continue
        out[name] = scan.scan_index_export(ix, code)
    return out


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def assert_index_equal(gix, oix, g):
    """Bit-exact comparison of every index array."""
    assert gix.info.n == oix.n and gix.info.nnz == g.nnz and gix.info.dmax == oix.dmax
    arr = export_all(gix)
    assert np.array_equal(arr["counts"], oix.counts), "counts differ"
    assert np.array_equal(bits(arr["sim"]), bits(oix.sim)), "similarity bits differ"
    assert np.array_equal(arr["no_ids"], oix.no_ids), "neighbour order ids differ"
    assert np.array_equal(bits(arr["no_sim"]), bits(oix.no_sim)), "neighbour order sims differ"
    assert np.array_equal(arr["co_off"], oix.co_off), "core order offsets differ"
    assert np.array_equal(arr["co_ids"], oix.co_ids), "core order ids differ"
    assert np.array_equal(bits(arr["co_thr"]), bits(oix.co_thr)), "core thresholds differ"


def query_grid(dmax, sims):
    """(mu, eps) pairs covering every distinct outcome region of interest."""
    mus = sorted({2, 3, 4, 5, 8, max(2, dmax), dmax + 1, dmax + 2})
    vals = np.unique(sims) if len(sims) else np.array([0.5])
    pick = vals[np.linspace(0, len(vals) - 1, min(len(vals), 9)).astype(int)]
    epss = sorted(set(pick.tolist()) | {float(np.nextafter(x, 2)) for x in pick.tolist()}
                  | {0.0, -0.25, 0.6, 1.0, float(np.nextafter(1.0, 2))})
    return [(m, e) for m in mus for e in epss]


def assert_queries_equal(gix, oix, pairs):
    import torch

    for mu, eps in pairs:
        memb, core = scan.scan_query_ex(gix, mu, eps)
        torch.cuda.synchronize()
        om, oc = oracle.query(oix, mu, eps)
        assert np.array_equal(memb.cpu().numpy(), om), (mu, eps)
        assert np.array_equal(core.cpu().numpy(), oc), (mu, eps)
