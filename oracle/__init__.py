"""CPU oracle for exact index-based SCAN — TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It shares no code with the GPU library.
The arithmetic lives in ``scan_oracle.cpp`` (plain C++17, no fast-math,
``-ffp-contract=off``); this module only marshals numpy arrays.

Parity status: each function below is pinned by the CPU tests named beside
it, against hand-worked graphs, closed forms, invariants or a brute-force
direct SCAN written separately from the definitions of Section 3.1; none is
"parity unpinned".

  validate                       test_oracle_pins: test_validate
  similarities, edge_similarity  test_oracle_pins: hand-worked, closed forms,
                                 trace(A^3), dense counts, brute force
  edge_similarities              test_oracle_pins:
                                 test_edge_similarities_equal_full_pass
  neighbor_order(_row), core_order, build_index
                                 test_oracle_pins: hand-worked orders and
                                 invariants; the one-row order equals the pass
  query                          test_oracle_pins: direct SCAN at every
                                 (mu, eps) breakpoint, hand-worked, Figure 1
  roles, modularity              test_oracle_pins: Figure 1, hand-worked
                                 fixture; closed forms, exact rational sums
  weighted_*                     test_oracle_weighted (the per-edge function:
                                 test_weighted_edge_function_equals_full_pass)
  simhash_/minhash_sketches      test_oracle_lsh: hand-worked sketches
  lsh_similarities               test_oracle_lsh: exact below the thresholds,
                                 twins, unbiasedness, hand-worked estimates
  lsh_edge_similarities          test_oracle_lsh: test_edge_function_equals_
                                 full_pass (every slot, SimHash, weighted
                                 SimHash, MinHash) and the hand-worked
                                 approximated edges
  build_index_lsh                test_oracle_lsh:
                                 test_build_index_lsh_composes_the_orders
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scan_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

COSINE = 0
JACCARD = 1
WEIGHTED_COSINE = 2


def build() -> str:
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-pthread", _SRC, "-o", _LIB_PATH + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.oracle_validate.argtypes = [i64, vp, vp, ctypes.POINTER(i64)]
    lib.oracle_validate.restype = ctypes.c_int
    lib.oracle_max_degree.argtypes = [i64, vp]
    lib.oracle_max_degree.restype = i64
    lib.oracle_similarities.argtypes = [i64, vp, vp, i32, i32, vp, vp]
    lib.oracle_similarities.restype = None
    lib.oracle_edge_similarity.argtypes = [vp, vp, i32, i64, i64, vp]
    lib.oracle_edge_similarity.restype = f64
    lib.oracle_edge_similarities.argtypes = [vp, vp, i32, i64, vp, vp, i32, vp, vp]
    lib.oracle_edge_similarities.restype = None
    lib.oracle_hardware_concurrency.argtypes = []
    lib.oracle_hardware_concurrency.restype = i32
    lib.oracle_neighbor_order.argtypes = [i64, vp, vp, vp, i32, vp, vp]
    lib.oracle_neighbor_order.restype = None
    lib.oracle_neighbor_order_row.argtypes = [i64, vp, vp, vp, vp]
    lib.oracle_neighbor_order_row.restype = None
    lib.oracle_core_order.argtypes = [i64, vp, vp, i64, i32, vp, vp, vp]
    lib.oracle_core_order.restype = None
    lib.oracle_query.argtypes = [i64, vp, vp, vp, vp, vp, vp, i64, i32, f64, vp, vp]
    lib.oracle_query.restype = ctypes.c_int
    lib.oracle_roles.argtypes = [i64, vp, vp, vp, vp]
    lib.oracle_roles.restype = None
    lib.oracle_modularity_terms.argtypes = [i64, vp, vp, vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.oracle_modularity_terms.restype = None
    lib.oracle_modularity_value.argtypes = [i64, i64, i64]
    lib.oracle_modularity_value.restype = f64
    lib.oracle_weighted_similarities.argtypes = [i64, vp, vp, vp, i32, vp]
    lib.oracle_weighted_similarities.restype = None
    lib.oracle_weighted_edge_similarity.argtypes = [vp, vp, vp, i64, i64]
    lib.oracle_weighted_edge_similarity.restype = f64
    lib.oracle_weighted_square_sum.argtypes = [vp, vp, vp, i64]
    lib.oracle_weighted_square_sum.restype = f64
    lib.oracle_simhash_sketches.argtypes = [vp, vp, vp, i64, vp, i64, vp, vp]
    lib.oracle_simhash_sketches.restype = None
    lib.oracle_minhash_sketches.argtypes = [i64, vp, vp, i64, vp, i64, vp, vp]
    lib.oracle_minhash_sketches.restype = None
    lib.oracle_lsh_similarities.argtypes = [i64, vp, vp, vp, i32, i64, vp, vp, i32, vp]
    lib.oracle_lsh_similarities.restype = None
    lib.oracle_lsh_edge_similarity.argtypes = [i64, vp, vp, vp, i32, i64, vp, vp, i64, i64]
    lib.oracle_lsh_edge_similarity.restype = f64
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data if a.size else None


def _csr(g):
    off = np.ascontiguousarray(g.off, dtype=np.int64)
    adj = np.ascontiguousarray(g.adj, dtype=np.int32)
    return off, adj


@dataclass
class OracleIndex:
    n: int
    off: np.ndarray      # int64[n+1]
    dmax: int
    kind: int
    counts: np.ndarray   # int32[nnz], c = |N[u] ∩ N[v]| per CSR slot
    sim: np.ndarray      # float64[nnz], per CSR slot
    no_ids: np.ndarray   # int32[nnz]
    no_sim: np.ndarray   # float64[nnz]
    co_off: np.ndarray   # int64[dmax+3], indexed by mu
    co_ids: np.ndarray   # int32[nnz]
    co_thr: np.ndarray   # float64[nnz]


def validate(g) -> int:
    """-1 if g is a valid simple undirected CSR, else the first bad row. Rows
    must lie inside adj and the last one must end at its end."""
    off, adj = _csr(g)
    if g.n > 0:
        past = np.nonzero(off[1:] > len(adj))[0]
        if len(past):
            return int(past[0])
        if int(off[-1]) != len(adj):
            return g.n - 1
    bad = ctypes.c_int64(-1)
    rc = _load().oracle_validate(g.n, _p(off), _p(adj), ctypes.byref(bad))
    return -1 if rc == 0 else int(bad.value)


def similarities(g, kind: int = COSINE, threads: int = 1):
    lib = _load()
    off, adj = _csr(g)
    nnz = int(off[-1])
    counts = np.zeros(nnz, np.int32)
    sim = np.zeros(nnz, np.float64)
    lib.oracle_similarities(g.n, _p(off), _p(adj), kind, threads, _p(counts), _p(sim))
    return counts, sim


def edge_similarity(g, u: int, v: int, kind: int = COSINE):
    """(c, sim) for one edge {u, v}."""
    off, adj = _csr(g)
    c = ctypes.c_int32()
    s = _load().oracle_edge_similarity(_p(off), _p(adj), kind, u, v, ctypes.byref(c))
    return int(c.value), float(s)


def hardware_concurrency() -> int:
    """std::thread::hardware_concurrency() of this host."""
    return int(_load().oracle_hardware_concurrency())


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or "unknown"."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def edge_similarities(g, us: np.ndarray, vs: np.ndarray, kind: int = COSINE, threads: int = 1):
    """(counts c, similarities) of the edges (us[i], vs[i]), each computed
    alone by oracle_edge_similarity, spread over `threads`."""
    off, adj = _csr(g)
    us = np.ascontiguousarray(us, dtype=np.int64)
    vs = np.ascontiguousarray(vs, dtype=np.int64)
    if us.shape != vs.shape:
        raise ValueError("us and vs differ in length")
    if len(us) and (min(us.min(), vs.min()) < 0 or max(us.max(), vs.max()) >= g.n):
        raise ValueError("edge endpoints must be vertices of g")
    cs = np.zeros(len(us), np.int32)
    ss = np.zeros(len(us), np.float64)
    _load().oracle_edge_similarities(_p(off), _p(adj), kind, len(us), _p(us), _p(vs), threads, _p(cs), _p(ss))
    return cs, ss


def neighbor_order(g, sim: np.ndarray, threads: int = 1):
    off, adj = _csr(g)
    nnz = int(off[-1])
    no_ids = np.zeros(nnz, np.int32)
    no_sim = np.zeros(nnz, np.float64)
    _load().oracle_neighbor_order(g.n, _p(off), _p(adj), _p(np.ascontiguousarray(sim)), threads,
                                  _p(no_ids), _p(no_sim))
    return no_ids, no_sim


def neighbor_order_row(ids: np.ndarray, sim: np.ndarray):
    """One row of the neighbour order: (ids, sims) sorted by sim desc, id asc."""
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    sim = np.ascontiguousarray(sim, dtype=np.float64)
    out_i = np.zeros(len(ids), np.int32)
    out_s = np.zeros(len(ids), np.float64)
    _load().oracle_neighbor_order_row(len(ids), _p(ids), _p(sim), _p(out_i), _p(out_s))
    return out_i, out_s


def core_order(g, no_sim: np.ndarray, dmax: int, threads: int = 1):
    off, _ = _csr(g)
    nnz = int(off[-1])
    co_off = np.zeros(dmax + 3, np.int64)
    co_ids = np.zeros(nnz, np.int32)
    co_thr = np.zeros(nnz, np.float64)
    _load().oracle_core_order(g.n, _p(off), _p(np.ascontiguousarray(no_sim)), dmax, threads,
                              _p(co_off), _p(co_ids), _p(co_thr))
    return co_off, co_ids, co_thr


def build_index(g, kind: int = COSINE, threads: int = 1) -> OracleIndex:
    off, _ = _csr(g)
    dmax = int(_load().oracle_max_degree(g.n, _p(off)))
    counts, sim = similarities(g, kind, threads)
    no_ids, no_sim = neighbor_order(g, sim, threads)
    co_off, co_ids, co_thr = core_order(g, no_sim, dmax, threads)
    return OracleIndex(g.n, off, dmax, kind, counts, sim, no_ids, no_sim, co_off, co_ids, co_thr)


def _weights(g, w) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    if w.shape != (g.nnz,):
        raise ValueError(f"weights must have nnz = {g.nnz} entries, got {w.shape}")
    return w


def weighted_similarities(g, w: np.ndarray, threads: int = 1) -> np.ndarray:
    """Section 3.1 weighted cosine of every edge, per CSR slot (w parallel to adj)."""
    off, adj = _csr(g)
    w = _weights(g, w)
    sim = np.zeros(g.nnz, np.float64)
    _load().oracle_weighted_similarities(g.n, _p(off), _p(adj), _p(w), threads, _p(sim))
    return sim


def weighted_edge_similarity(g, w: np.ndarray, u: int, v: int) -> float:
    off, adj = _csr(g)
    return float(_load().oracle_weighted_edge_similarity(_p(off), _p(adj), _p(_weights(g, w)), u, v))


def weighted_edge_similarities(g, w: np.ndarray, us: np.ndarray, vs: np.ndarray) -> np.ndarray:
    off, adj = _csr(g)
    w = _weights(g, w)
    lib = _load()
    po, pa, pw = _p(off), _p(adj), _p(w)
    return np.array([lib.oracle_weighted_edge_similarity(po, pa, pw, u, v)
                     for u, v in zip(us.tolist(), vs.tolist())], np.float64)


def weighted_square_sum(g, w: np.ndarray, v: int) -> float:
    """Sum of w(v, x)^2 over the closed neighbourhood of v (w(v, v) = 1)."""
    off, adj = _csr(g)
    return float(_load().oracle_weighted_square_sum(_p(off), _p(adj), _p(_weights(g, w)), v))


def build_index_weighted(g, w: np.ndarray, threads: int = 1) -> OracleIndex:
    """Algorithms 1 and 2 with the weighted cosine; counts are not defined
    for it (all zero here)."""
    off, _ = _csr(g)
    dmax = int(_load().oracle_max_degree(g.n, _p(off)))
    sim = weighted_similarities(g, w, threads)
    no_ids, no_sim = neighbor_order(g, sim, threads)
    co_off, co_ids, co_thr = core_order(g, no_sim, dmax, threads)
    return OracleIndex(g.n, off, dmax, WEIGHTED_COSINE, np.zeros(g.nnz, np.int32), sim, no_ids, no_sim,
                       co_off, co_ids, co_thr)


def simhash_sketches(g, k: int, gauss: np.ndarray, vs, w: np.ndarray | None = None) -> np.ndarray:
    """uint8[len(vs), k] SimHash bits (Section 2.1.2) of N[v] for v in vs."""
    off, adj = _csr(g)
    gauss = np.ascontiguousarray(gauss, dtype=np.float64).reshape(-1)
    assert gauss.size == g.n * k
    vs = np.ascontiguousarray(vs, dtype=np.int64)
    out = np.zeros((len(vs), k), np.uint8)
    ww = None if w is None else _weights(g, w)
    _load().oracle_simhash_sketches(_p(off), _p(adj), None if ww is None else _p(ww), k, _p(gauss), len(vs),
                                    _p(vs), _p(out))
    return out


def minhash_sketches(g, k: int, perm: np.ndarray, vs) -> np.ndarray:
    """uint32[len(vs), k] k-partition MinHash sketches of N[v] (empty bin = 2^32-1)."""
    off, adj = _csr(g)
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    vs = np.ascontiguousarray(vs, dtype=np.int64)
    out = np.zeros((len(vs), k), np.uint32)
    _load().oracle_minhash_sketches(g.n, _p(off), _p(adj), k, _p(perm), len(vs), _p(vs), _p(out))
    return out


def _lsh_inputs(g, kind: int, k: int, gauss, perm, w):
    """Checks and marshals the LSH draws: the cosine kinds (COSINE, and
    WEIGHTED_COSINE, which needs w) take SimHash directions gauss (n x k), JACCARD
    a permutation perm of 0..n-1; w has one weight per CSR slot. Returns
    (gauss flat or None, perm or None, w or None)."""
    if kind not in (COSINE, JACCARD, WEIGHTED_COSINE):
        raise ValueError(f"unknown similarity kind {kind}")
    if k < 1:
        raise ValueError("k must be >= 1")
    if kind == WEIGHTED_COSINE and w is None:
        raise ValueError("WEIGHTED_COSINE needs the edge weights w")
    if kind == JACCARD and w is not None:
        raise ValueError("weights go with the cosine kinds only")
    gp = pp = None
    if kind == JACCARD:
        if perm is None:
            raise ValueError("MinHash (JACCARD) needs the permutation perm")
        pp = np.ascontiguousarray(perm, dtype=np.uint32)
        if pp.shape != (g.n,) or (g.n and int(pp.max()) >= g.n):
            raise ValueError("perm must hold n values in [0, n)")
    else:
        if gauss is None:
            raise ValueError("SimHash (the cosine kinds) needs the Gaussian draws gauss")
        gp = np.ascontiguousarray(gauss, dtype=np.float64).reshape(-1)
        if gp.size != g.n * k:
            raise ValueError(f"gauss must hold n * k = {g.n * k} values")
    ww = None if w is None else _weights(g, w)
    return gp, pp, ww


def lsh_similarities(g, kind: int, k: int, gauss=None, perm=None, w=None, threads: int = 1) -> np.ndarray:
    """Per-slot approximate similarities (Section 5 + the Section 6.3 heuristic):
    the cosine kinds use SimHash with `gauss` (n x k), weighted when w is given
    (required for WEIGHTED_COSINE); JACCARD uses k-partition MinHash with
    `perm`."""
    gp, pp, ww = _lsh_inputs(g, kind, k, gauss, perm, w)
    off, adj = _csr(g)
    sim = np.zeros(g.nnz, np.float64)
    _load().oracle_lsh_similarities(g.n, _p(off), _p(adj), None if ww is None else _p(ww), kind, k,
                                    None if gp is None else _p(gp), None if pp is None else _p(pp), threads,
                                    _p(sim))
    return sim


def lsh_edge_similarities(g, kind: int, k: int, us, vs, gauss=None, perm=None, w=None) -> np.ndarray:
    """lsh_similarities at the given edges only (sampled checks on large
    graphs): each edge's sketches are recomputed from the draws."""
    gp, pp, ww = _lsh_inputs(g, kind, k, gauss, perm, w)
    off, adj = _csr(g)
    lib = _load()
    args = (g.n, _p(off), _p(adj), None if ww is None else _p(ww), kind, k, None if gp is None else _p(gp),
            None if pp is None else _p(pp))
    return np.array([lib.oracle_lsh_edge_similarity(*args, int(u), int(v)) for u, v in zip(us, vs)], np.float64)


def build_index_lsh(g, kind: int, k: int, gauss=None, perm=None, w=None, threads: int = 1) -> OracleIndex:
    """Approximate index: LSH similarities, then Algorithm 2's orders."""
    off, _ = _csr(g)
    dmax = int(_load().oracle_max_degree(g.n, _p(off)))
    sim = lsh_similarities(g, kind, k, gauss, perm, w, threads)
    no_ids, no_sim = neighbor_order(g, sim, threads)
    co_off, co_ids, co_thr = core_order(g, no_sim, dmax, threads)
    okind = WEIGHTED_COSINE if (kind == COSINE and w is not None) else kind
    return OracleIndex(g.n, off, dmax, okind, np.zeros(g.nnz, np.int32), sim, no_ids, no_sim, co_off, co_ids,
                       co_thr)


def query(ix: OracleIndex, mu: int, eps: float):
    """(memberships int32[n], is_core uint8[n]) for (mu, eps)."""
    memb = np.zeros(ix.n, np.int32)
    core = np.zeros(ix.n, np.uint8)
    rc = _load().oracle_query(ix.n, _p(ix.off), _p(ix.no_ids), _p(ix.no_sim), _p(ix.co_off),
                              _p(ix.co_ids), _p(ix.co_thr), ix.dmax, int(mu), float(eps),
                              _p(memb), _p(core))
    if rc != 0:
        raise ValueError(f"oracle_query rejected mu={mu} eps={eps}")
    return memb, core


ROLE_CLUSTERED, ROLE_HUB, ROLE_OUTLIER = 0, 1, 2


def roles(g, memberships: np.ndarray) -> np.ndarray:
    """Section 4.3: uint8[n], 0 in a cluster, 1 hub (unclustered, neighbours in
    >= 2 clusters), 2 outlier (unclustered, neighbours in at most one)."""
    off, adj = _csr(g)
    memb = np.ascontiguousarray(memberships, dtype=np.int32)
    out = np.zeros(g.n, np.uint8)
    _load().oracle_roles(g.n, _p(off), _p(adj), _p(memb), _p(out))
    return out


def modularity(g, memberships: np.ndarray):
    """Section 7.2 modularity with unclustered vertices as singletons
    (Section 7.3.4): (Q, s_in, sd2), see oracle_modularity_terms."""
    off, adj = _csr(g)
    memb = np.ascontiguousarray(memberships, dtype=np.int32)
    s_in, sd2 = ctypes.c_int64(), ctypes.c_int64()
    lib = _load()
    lib.oracle_modularity_terms(g.n, _p(off), _p(adj), _p(memb), ctypes.byref(s_in), ctypes.byref(sd2))
    return float(lib.oracle_modularity_value(s_in.value, sd2.value, g.nnz)), s_in.value, sd2.value
