"""Seeded synthetic graph inputs (R-MAT, stochastic block models, tiny graphs).

This package produces inputs only; it holds none of the clustering method's
arithmetic. Both the CPU oracle and the GPU library consume what it emits: a
simple undirected graph as CSR (``off`` int64[n+1], ``adj`` int32[nnz]) with
strictly ascending rows, no self-loops and both directions of every edge.

The random numbers come from a counter-based SplitMix64 stream (see
``graphgen.cpp``), so every graph is a pure function of its parameters and seed.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


class _CSR(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("off", ctypes.POINTER(ctypes.c_int64)),
        ("adj", ctypes.POINTER(ctypes.c_int32)),
    ]


def build() -> str:
    """Compile libgraphgen.so in place (host C++ with OpenMP)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _LIB_PATH + ".tmp"]
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
    P = ctypes.POINTER
    lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_uint64, P(_CSR)]
    lib.gg_rmat.restype = ctypes.c_int
    lib.gg_sbm.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                           ctypes.c_uint64, P(_CSR)]
    lib.gg_sbm.restype = ctypes.c_int
    lib.gg_from_pairs.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, P(_CSR)]
    lib.gg_from_pairs.restype = ctypes.c_int
    lib.gg_free.argtypes = [P(_CSR)]
    lib.gg_free.restype = None
    lib.gg_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.gg_draw.restype = ctypes.c_uint64
    lib.gg_unit.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.gg_unit.restype = ctypes.c_double
    lib.gg_gaussians.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p]
    lib.gg_gaussians.restype = None
    lib.gg_permutation.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p]
    lib.gg_permutation.restype = None
    lib.gg_edge_weights.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
    lib.gg_edge_weights.restype = None
    lib.gg_degree_stats.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p] + [P(ctypes.c_int64)] * 4
    lib.gg_degree_stats.restype = None
    lib.gg_owner_split.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    lib.gg_owner_split.restype = None
    _lib = lib
    return lib


@dataclass
class Graph:
    """Simple undirected graph in CSR form (both directions stored)."""

    n: int
    off: np.ndarray  # int64[n+1]
    adj: np.ndarray  # int32[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.off[-1]) if self.n >= 0 and len(self.off) else 0

    @property
    def num_edges(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.off)


def _take(csr: _CSR, name: str) -> Graph:
    lib = _load()
    n, nnz = int(csr.n), int(csr.nnz)
    off = np.ctypeslib.as_array(csr.off, shape=(n + 1,)).copy()
    adj = np.ctypeslib.as_array(csr.adj, shape=(max(nnz, 1),))[:nnz].copy() if nnz else np.zeros(0, np.int32)
    lib.gg_free(ctypes.byref(csr))
    return Graph(n, off, adj, name)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1) -> Graph:
    """R-MAT graph: 2**scale vertices, edge_factor * 2**scale sampled edges, then
    symmetrised, deduplicated and self-loop free."""
    lib = _load()
    csr = _CSR()
    samples = edge_factor << scale
    rc = lib.gg_rmat(scale, samples, a, b, c, seed, ctypes.byref(csr))
    if rc != 0:
        raise RuntimeError(f"gg_rmat failed ({rc})")
    return _take(csr, f"rmat{scale}_ef{edge_factor}_s{seed}")


def sbm(n: int, k: int, p_in: float, p_out: float, seed: int = 1) -> Graph:
    """Stochastic block model with k equal consecutive blocks."""
    lib = _load()
    csr = _CSR()
    rc = lib.gg_sbm(n, k, p_in, p_out, seed, ctypes.byref(csr))
    if rc != 0:
        raise RuntimeError(f"gg_sbm failed ({rc})")
    return _take(csr, f"sbm{n}_k{k}_s{seed}")


def from_edges(n: int, edges) -> Graph:
    """Simple undirected graph from an iterable of (u, v) pairs (either
    direction); self-loops and duplicates are dropped."""
    lib = _load()
    e = np.asarray(list(edges) if not isinstance(edges, np.ndarray) else edges, dtype=np.int32).reshape(-1, 2)
    pu = np.ascontiguousarray(e[:, 0])
    pv = np.ascontiguousarray(e[:, 1])
    csr = _CSR()
    rc = lib.gg_from_pairs(n, len(pu), pu.ctypes.data, pv.ctypes.data, ctypes.byref(csr))
    if rc != 0:
        raise RuntimeError(f"gg_from_pairs failed ({rc})")
    return _take(csr, f"edges{n}")


def draw(seed: int, ctr: int) -> int:
    return int(_load().gg_draw(seed, ctr))


def unit(seed: int, ctr: int) -> float:
    return float(_load().gg_unit(seed, ctr))


def edge_weights(g: Graph, seed: int, lo: float = 0.05, hi: float = 1.0) -> np.ndarray:
    """float64[nnz] edge weights parallel to g.adj, uniform in [lo, hi) with
    full 53-bit mantissas, equal for both directions of an edge."""
    lib = _load()
    off = np.ascontiguousarray(g.off, dtype=np.int64)
    adj = np.ascontiguousarray(g.adj, dtype=np.int32)
    w = np.zeros(g.nnz, np.float64)
    if g.nnz:
        lib.gg_edge_weights(g.n, off.ctypes.data, adj.ctypes.data, seed, lo, hi, w.ctypes.data)
    return w


def gaussians(n: int, k: int, seed: int) -> np.ndarray:
    """float64[n, k] standard normal draws (Box-Muller over the stream): the
    random hyperplanes of SimHash, one coordinate per vertex and sample."""
    out = np.zeros((n, k), np.float64)
    if n and k:
        _load().gg_gaussians(n, k, seed, out.ctypes.data)
    return out


def permutation(n: int, seed: int) -> np.ndarray:
    """uint32[n], a uniformly random permutation of 0..n-1 (Fisher-Yates)."""
    out = np.zeros(n, np.uint32)
    if n:
        _load().gg_permutation(n, seed, out.ctypes.data)
    return out


def degree_stats(g: Graph) -> dict:
    """n, nnz, |E|, Dmax, non-isolated vertices, W_min = sum over undirected
    edges of min(deg u, deg v), and sum of deg^2."""
    lib = _load()
    off = np.ascontiguousarray(g.off, dtype=np.int64)
    adj = np.ascontiguousarray(g.adj, dtype=np.int32)
    vals = [ctypes.c_int64() for _ in range(4)]
    lib.gg_degree_stats(g.n, off.ctypes.data, adj.ctypes.data if len(adj) else None,
                        *[ctypes.byref(v) for v in vals])
    dmax, noniso, wmin, s2 = (int(v.value) for v in vals)
    return {"n": g.n, "nnz": g.nnz, "edges": g.nnz // 2, "dmax": dmax, "non_isolated": noniso,
            "w_min": wmin, "sum_deg2": s2}


def owner_split(g: Graph, small_max: int) -> dict:
    """Edges and W_min split by owner class: an edge is owned by its endpoint
    larger in (degree, id), and owners of degree <= small_max are "small"."""
    off = np.ascontiguousarray(g.off, dtype=np.int64)
    adj = np.ascontiguousarray(g.adj, dtype=np.int32)
    out = np.zeros(4, np.int64)
    _load().gg_owner_split(g.n, off.ctypes.data, adj.ctypes.data if len(adj) else None, int(small_max),
                           out.ctypes.data)
    return {"edges_small": int(out[0]), "w_small": int(out[1]), "edges_big": int(out[2]), "w_big": int(out[3])}


# ---------------------------------------------------------------------------
# Workload recipes


def sbm2000(seed: int = 2000) -> Graph:
    """2,000 vertices in 20 blocks of 100, p_in = 0.1, p_out = 0.002."""
    g = sbm(2000, 20, 0.1, 0.002, seed)
    g.name = f"sbm2000_s{seed}"
    return g


def rmat20(seed: int = 20) -> Graph:
    g = rmat(20, 16, seed=seed)
    g.name = f"rmat20_s{seed}"
    return g


def rmat23(seed: int = 23) -> Graph:
    g = rmat(23, 32, seed=seed)
    g.name = f"rmat23_s{seed}"
    return g


@dataclass
class SbmSpec:
    n: int
    k: int
    d: float
    p_in: float
    p_out: float
    seed: int
    clamped: bool


def batch_sbm_specs(count: int = 256, seed: int = 256, n_lo: float = 1e3, n_hi: float = 2e5,
                    k_lo: int = 5, k_hi: int = 200, d_lo: float = 8.0, d_hi: float = 64.0,
                    ratio: float = 0.02) -> list[SbmSpec]:
    """Uneven SBM batch: n log-uniform in [n_lo, n_hi], k uniform in
    {k_lo..k_hi}, average degree d uniform in [d_lo, d_hi],
    p_in = d / ((s-1) + ratio*(n-s)) with s = n/k, p_out = ratio*p_in.
    k is clamped to floor(n/(ceil(d)+1)) when p_in would exceed 1."""
    specs = []
    for g in range(count):
        base = 4 * g
        n = int(round(math.exp(math.log(n_lo) + unit(seed, base) * (math.log(n_hi) - math.log(n_lo)))))
        k = k_lo + int(unit(seed, base + 1) * (k_hi - k_lo + 1))
        d = d_lo + unit(seed, base + 2) * (d_hi - d_lo)
        clamped = False
        kmax = max(1, n // (math.ceil(d) + 1))
        if k > kmax:
            k, clamped = kmax, True
        s = n / k
        p_in = d / ((s - 1) + ratio * (n - s))
        if p_in > 1.0:
            p_in, clamped = 1.0, True
        specs.append(SbmSpec(n, k, d, p_in, ratio * p_in, draw(seed, base + 3), clamped))
    return specs


def batch_sbm(count: int = 256, seed: int = 256, **kw) -> list[Graph]:
    out = []
    for i, sp in enumerate(batch_sbm_specs(count, seed, **kw)):
        g = sbm(sp.n, sp.k, sp.p_in, sp.p_out, sp.seed)
        g.name = f"bsbm{i}_n{sp.n}_k{sp.k}"
        out.append(g)
    return out


def tiny_graphs(n: int):
    """Every labelled simple graph on n vertices (2**(n(n-1)/2) of them)."""
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    for mask in range(1 << len(pairs)):
        yield from_edges(n, [p for b, p in enumerate(pairs) if mask >> b & 1] or np.zeros((0, 2), np.int32))


def random_graph(n: int, p: float, seed: int) -> Graph:
    """Erdos-Renyi G(n, p) from the counter-based stream (pair (i,j) uses
    counter i*n + j)."""
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if unit(seed, i * n + j) < p]
    return from_edges(n, edges or np.zeros((0, 2), np.int32))
