"""The clustering a (mu, eps) query defines, evaluated from index arrays with
numpy/scipy (for sizes where the oracle's full build is too slow): cores by
the core test, clusters as connected components of cores joined by
eps-similar edges labelled by their smallest core, and every non-core with an
eps-similar core joining the cluster of the first such core in its neighbour
order (ties in the order already broken by id). Pinned against the oracle's
query on small graphs by the CPU tests."""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


def expected_query(off, adj, sims, no_ids, no_sim, mu: int, eps: float):
    """(memberships int32[n], core bool[n]); sims are per CSR slot."""
    n = len(off) - 1
    deg = np.diff(off).astype(np.int64)
    idx = np.where(deg >= mu - 1, off[:-1] + mu - 2, 0)
    core = (deg >= mu - 1) & (no_sim[idx] >= eps) if len(no_sim) else np.zeros(n, bool)
    srcs = np.repeat(np.arange(n, dtype=np.int32), deg)
    sel = sims >= eps
    sel &= core[adj]
    sel &= core[srcs]
    src, dst = srcs[sel], adj[sel]
    del srcs, sel
    A = sp.csr_matrix((np.ones(len(src), np.int8), (src, dst)), shape=(n, n))
    _, lab = connected_components(A, directed=False)
    cores = np.flatnonzero(core)
    want = np.full(n, -1, np.int64)
    if len(cores):
        uniq, first = np.unique(lab[cores], return_index=True)
        minid = np.zeros(lab.max() + 1, np.int64)
        minid[uniq] = cores[first]  # cores ascend: a label's first core is its smallest
        want[cores] = minid[lab[cores]]
        valid = (no_sim >= eps) & core[no_ids]
        pos = np.flatnonzero(valid)
        rows = np.searchsorted(off, pos, side="right") - 1
        ur, fi = np.unique(rows, return_index=True)
        nc = ~core[ur]
        want[ur[nc]] = want[no_ids[pos[fi[nc]]]]
    return want.astype(np.int32), core
