"""Direct SCAN from the definitions of Section 3.1, for tiny graphs.

Written independently of the oracle (pure Python sets, no index): similarity
over closed neighbourhoods, epsilon-neighbourhoods N_eps(v) over N[v] with
sigma(v, v) = 1, cores |N_eps(v)| >= mu, clusters by structural reachability
from cores, and border vertices resolved by the deterministic rule of Section
7.3.4 (most similar epsilon-similar core, ties to the lower id). Clusters are
labelled by their smallest core id; unclustered vertices get -1.
"""

from __future__ import annotations

import math


def closed_neighbourhoods(g):
    out = []
    for v in range(g.n):
        row = set(int(x) for x in g.adj[g.off[v]:g.off[v + 1]])
        row.add(v)
        out.append(row)
    return out


def sigma_table(g, kind: int):
    """{(u, v): sigma} for every ordered adjacent pair and for (v, v)."""
    nb = closed_neighbourhoods(g)
    sig = {}
    for u in range(g.n):
        for v in nb[u]:
            a, b = nb[u], nb[v]
            inter = len(a & b)
            if kind == 0:
                s = inter / math.sqrt(len(a) * len(b))
            else:
                s = inter / len(a | b)
            sig[(u, v)] = s
    return nb, sig


def direct_scan(g, kind: int, mu: int, eps: float, tables=None):
    nb, sig = tables if tables is not None else sigma_table(g, kind)
    n = g.n
    eps_nb = [{u for u in nb[v] if sig[(u, v)] >= eps} for v in range(n)]
    core = [len(eps_nb[v]) >= mu for v in range(n)]
    # Structural reachability: from a core, every epsilon-similar neighbour is
    # reached; the walk continues only through cores.
    label = [-1] * n
    for r in range(n):
        if not core[r] or label[r] != -1:
            continue
        comp, stack = {r}, [r]
        while stack:
            x = stack.pop()
            for y in eps_nb[x]:
                if core[y] and y not in comp:
                    comp.add(y)
                    stack.append(y)
        m = min(comp)
        for x in comp:
            label[x] = m
    memb = [-1] * n
    for v in range(n):
        if core[v]:
            memb[v] = label[v]
            continue
        best = None
        for u in nb[v]:
            if u != v and core[u] and v in eps_nb[u]:
                key = (-sig[(u, v)], u)
                if best is None or key < best[0]:
                    best = (key, u)
        if best is not None:
            memb[v] = label[best[1]]
    return memb, [int(c) for c in core]


def eps_grid(sig_values):
    """Finite set of eps values that covers every distinct outcome: the
    clustering is piecewise constant in eps with breakpoints at the similarity
    values, so each value, its successor, and the ends suffice."""
    vals = set(sig_values) | {0.0, 1.0}
    out = set()
    for s in vals:
        out.add(s)
        out.add(math.nextafter(s, math.inf))
    out.add(-0.5)
    return sorted(out)
