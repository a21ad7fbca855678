"""Benchmark of the exact SCAN index build and (mu, eps) queries on one MI355X.

Workloads (--workload):
  rmat20 (default)  cosine index build on R-MAT scale 20 (edge factor 16,
                    (a,b,c,d) = (.57,.19,.19,.05), symmetrised, deduplicated,
                    self-loops removed, int32 CSR), with intersection shapes
                    from the autotuner; then query latency one at a time vs
                    batched on the same index, closed loop and as open-loop
                    Poisson serving.
  rmat23            cosine and Jaccard builds on R-MAT scale 23, edge factor
                    32, int64 offsets (hubs of degree > 1e5).
  sbm256            batched build of 256 uneven stochastic-block-model graphs:
                    one merged build vs 256 per-graph builds.

One step = one full index build (degrees, ownership plan, intersection + FP64
similarity, neighbour order, core order) from a CSR resident in HBM to the
index resident in HBM. Prints ONE JSON line on stdout; progress goes to
stderr.

  python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload rmat20]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
METRIC = "index-build edges/s (R-MAT-20); query p50/p99 ms, batched vs one-at-a-time"
def counters_file(workload: str) -> str:
    """profiles/k_big_owner_<graph>_counters.txt for workload <graph>_..."""
    return os.path.join(ROOT, "profiles", f"k_big_owner_{workload.split('_')[0]}_counters.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2012_11188_amd", "csrc", "intersect.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def byte_model(st: dict, split: dict, s_off: int, deg=None, small_max: int = 256) -> dict:
    """Algorithmic bytes, fixed before measurement.

    Build, the survey's model (labelled "model" in the output): CSR read once,
    the min-side intersection work W_min charged 8 B per id (the shorter
    row's id, 4 B, and one 4 B probe of the longer row), similarities
    written once per slot, neighbour order read and written, core order read
    and written: s_off(n+1) + 56 nnz + 8 W_min.

    Build, memory model (what must cross the memory interface in this
    design): the same less the probe half, 4 W_min, since the longer row is
    probed in an LDS bitmap or hash table, on chip: s_off(n+1) + 56 nnz +
    4 W_min.

    Owner kernels, memory model: every lower neighbour's row streamed once per
    owned edge (4 B per id: 4 W), every owner slot staged once (its id, the
    neighbour's degree and offset: 16 B per slot of an owner of that class),
    both similarity slots of every owned edge written (16 B per edge). The
    survey's 8 W + 16 E is kept beside it."""
    n, nnz, wmin = st["n"], st["nnz"], st["w_min"]
    s_big = s_small = 0
    if deg is not None:
        s_big = int(deg[deg > small_max].sum())
        s_small = int(deg[deg <= small_max].sum())
    return {
        "build_model": s_off * (n + 1) + 56 * nnz + 8 * wmin,
        "build": s_off * (n + 1) + 56 * nnz + 4 * wmin,
        "floor": s_off * (n + 1) + 28 * nnz,
        "k_big_owner_model": 8 * split["w_big"] + 16 * split["edges_big"],
        "k_big_owner": 4 * split["w_big"] + 16 * s_big + 16 * split["edges_big"],
        "k_small_owner_model": 8 * split["w_small"] + 16 * split["edges_small"],
        "k_small_owner": 4 * split["w_small"] + 16 * s_small + 16 * split["edges_small"],
    }


def parse_tune(text: str):
    if not text or text == "auto":
        return None
    if text == "default":
        return {}
    out = {}
    for kv in text.split(","):
        k, v = kv.split("=")
        out[k.strip()] = int(v)
    return out


def tune_str(t: dict) -> str:
    return f"small_max={t['small_max']} spc={t['spc']} wbits={t['wbits']}"


def kernel_source_hash() -> str:
    """sha256 of the intersection kernels' source: intersect.hip up to its
    first host function."""
    src = open(KERNEL_SRC, encoding="utf-8").read()
    return hashlib.sha256(src[:src.index("IntersectPlan::~IntersectPlan")].encode()).hexdigest()


def counter_traffic(tune: dict, workload: str):
    """Measured HBM bytes per k_big_owner launch from the committed rocprofv3
    counter summary, if it was taken on this kernel source, workload and
    shape; else None and the reason."""
    path = counters_file(workload)
    if not os.path.exists(path):
        return None, "no counter summary"
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("device_source_sha256") != kernel_source_hash():
        return None, "kernel source changed since the counters were taken"
    if kv.get("workload") != workload or kv.get("config") != tune_str(tune):
        return None, f"counters taken on {kv.get('workload')} / {kv.get('config')}"
    fetch = float(kv["fetch_bytes_per_dispatch"])
    write = float(kv["write_bytes_per_dispatch"])
    return fetch + write, ("rocprofv3: read requests by size (32/64/128 B x TCC_EA0_RDREQ_{32B,64B,128B}) + "
                           "WRITE_SIZE; the size sum equals a 1 GiB copy and a 2 GiB reduction exactly")


def timed_builds(scan, torch, build, steps: int, warmup: int):
    """warmup untimed builds, then exactly `steps` builds back to back on the
    current stream; returns wall ms/step, device ms/step, per-step profiles
    and the last build's indexes."""
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        ixs = build()
        torch.cuda.synchronize()
        log(f"warmup {i}: {scan.scan_index_build_profile(ixs[0])}")
        del ixs
    profiles, keep = [], []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        keep.append(build())
        if len(keep) > 1:
            profiles.append(scan.scan_index_build_profile(keep.pop(0)[0]))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    profiles.append(scan.scan_index_build_profile(keep[-1][0]))
    return wall * 1e3 / steps, ev0.elapsed_time(ev1) / steps, profiles, keep[-1]


def med(profiles, key):
    return float(np.median([p[key] for p in profiles]))


PHASES = ("total_ms", "prepare_ms", "plan_ms", "intersect_ms", "intersect_small_ms", "intersect_big_ms",
          "no_sort_ms", "core_order_ms")


def autotune(scan, graphs, kind, tune_arg, reps=2):
    """Returns (tune dict, info). --tune auto runs the autotuner (untimed)."""
    t = parse_tune(tune_arg)
    if t is not None:
        full = {"small_max": t.get("small_max", 256), "spc": t.get("spc", 512), "wbits": t.get("wbits", 20)}
        return full, {"source": "given"}
    t0 = time.perf_counter()
    best = scan.scan_autotune(graphs, kind, reps=reps)
    info = {"source": "autotuner", "search_s": time.perf_counter() - t0, "through_intersect_ms": best["ms"]}
    log(f"autotune: {best} in {info['search_s']:.1f}s")
    return {k: best[k] for k in ("small_max", "spc", "wbits")}, info


def kernel_roofline(bm, phases, tune, workload):
    """Roofline of the dominant kernel, k_big_owner: achieved = its
    memory-model bytes per launch / its hipEvent duration; traffic = the
    measured bytes between L2 and memory per launch (rocprofv3 counters,
    calibrated); model_frac = the survey's 8 W + 16 E model, whose probe half
    is served from LDS (so it may exceed 1)."""
    big_ms = phases["intersect_big_ms"]
    sec = big_ms * 1e-3
    achieved = bm["k_big_owner"] / sec / 1e9
    traffic, why = counter_traffic(tune, workload)
    return {"bound": "hbm", "kernel": "k_big_owner", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": why,
            "traffic_frac": (traffic / sec / 1e9 / HBM_PEAK_GBS) if traffic else None,
            "bytes_per_launch": bm["k_big_owner"],
            "bytes_model": "4 B per streamed lower-row id + 16 B per owner slot + 16 B per owned edge",
            "launch_ms": big_ms,
            "model_bytes_per_launch": bm["k_big_owner_model"],
            "model_frac": bm["k_big_owner_model"] / sec / 1e9 / HBM_PEAK_GBS,
            "traffic_over_algorithmic": (traffic / bm["k_big_owner"]) if traffic else None}


def library_source_hash() -> str:
    """sha256 over every source file of the library (csrc/, sorted by name)."""
    d = os.path.join(ROOT, "paper_2012_11188_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()


def build_counter_traffic(workload: str, tune: dict):
    """Measured bytes between L2 and memory of one whole build (every kernel),
    from profiles/build_<graph>_counters.txt, if taken on this library source
    and shape; else None and the reason."""
    path = os.path.join(ROOT, "profiles", f"build_{workload.split('_')[0]}_counters.txt")
    if not os.path.exists(path):
        return None, "no counter summary"
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("library_source_sha256") != library_source_hash():
        return None, "library source changed since the counters were taken"
    if kv.get("workload") != workload or kv.get("config") != tune_str(tune):
        return None, f"counters taken on {kv.get('workload')} / {kv.get('config')}"
    return float(kv["fetch_bytes_per_build"]) + float(kv["write_bytes_per_build"]), "rocprofv3, every kernel of one build"


def build_roofline(bm, total_ms, workload=None, tune=None):
    sec = total_ms * 1e-3
    traffic, why = build_counter_traffic(workload, tune) if workload and tune else (None, "not taken")
    return {"bytes": bm["build"], "achieved": bm["build"] / sec / 1e9, "frac": bm["build"] / sec / 1e9 / HBM_PEAK_GBS,
            "bytes_model": "s_off(n+1) + 56 nnz + 4 W_min (intersection probes are on-chip)",
            "model_bytes": bm["build_model"], "model_frac": bm["build_model"] / sec / 1e9 / HBM_PEAK_GBS,
            "floor_bytes": bm["floor"], "floor_frac": bm["floor"] / sec / 1e9 / HBM_PEAK_GBS,
            "traffic": traffic, "traffic_source": why,
            "traffic_frac": (traffic / sec / 1e9 / HBM_PEAK_GBS) if traffic else None}


# ---------------------------------------------------------------------------
# Serving


def serve_ladder(scan, torch, ix, n, mode, max_slots, max_batch, queries, rates, dst_kind, seed=11):
    """Open-loop serving: `queries` requests with seeded Poisson arrivals at
    each offered rate, mu ~ U{2..16}, eps ~ U{0.10, 0.15, ..., 0.90}. Results
    go to a ring of device arrays or of pinned host arrays. Latency = result
    in place minus scheduled arrival, including time spent waiting to be
    admitted. Stops once the server no longer keeps up."""
    rng = np.random.default_rng(seed)
    mu = rng.integers(2, 17, queries).astype(np.int32)
    eps = np.array([(10 + 5 * k) / 100.0 for k in rng.integers(0, 17, queries)])
    if dst_kind == "device":
        ring = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(64)]
    else:
        ring = [torch.empty(n, dtype=torch.int32).pin_memory().numpy() for _ in range(64)]
    owner = [0] * len(ring)
    srv = scan.Server(ix, max_slots=max_slots, max_batch=max_batch, memory_budget=8 << 30, use_graph=True)
    out = []
    try:
        for i in range(100):  # warm-up
            srv.wait(srv.submit_ex(int(mu[i]), float(eps[i]), ring[i % len(ring)]))
        for rate in rates:
            arrive = np.cumsum(rng.exponential(1.0 / rate, queries))
            lat = np.zeros(queries)
            lag = np.zeros(queries)
            tickets = [0] * queries
            t0 = time.perf_counter()
            for i in range(queries):
                target = t0 + arrive[i]
                while time.perf_counter() < target:
                    pass
                r = i % len(ring)
                if owner[r]:
                    srv.wait(owner[r])
                while True:
                    t = srv.submit_ex(int(mu[i]), float(eps[i]), ring[r], lat.ctypes.data + 8 * i, block=False)
                    if t is not None:
                        break
                lag[i] = (time.perf_counter() - target) * 1e3
                tickets[i] = owner[r] = t
            for t in tickets:
                srv.wait(t)
            span = time.perf_counter() - t0
            owner = [0] * len(ring)
            total = lat + lag
            row = {"offered_qps": rate, "achieved_qps": queries / span,
                   "p50_ms": float(np.percentile(total, 50)), "p99_ms": float(np.percentile(total, 99))}
            out.append(row)
            log(f"serve {mode}/{dst_kind}: {row}")
            if row["achieved_qps"] < 0.95 * rate:
                break
    finally:
        srv.close()
    return {"max_slots": max_slots, "max_batch": max_batch, "ladder": out}


def sustainable(ladder, p99_budget=None):
    ok = [r for r in ladder if r["achieved_qps"] >= 0.95 * r["offered_qps"]
          and (p99_budget is None or r["p99_ms"] <= p99_budget)]
    return max(ok, key=lambda r: r["achieved_qps"]) if ok else None


def serving(scan, torch, ix, n, args):
    rates = [5000 * 1.5 ** k for k in range(9)]
    B = args.serve_batch
    res = {"queries_per_rate": args.serve_queries, "arrivals": "poisson (seeded, open loop)", "mu": "U{2..16}",
           "eps": "U{0.10,0.15,...,0.90}", "use_graph": True}
    for dst in ("device", "pinned_host"):
        # Host results cross PCIe (4n bytes each): smaller batches keep a batch's
        # copies short, so the tail latency stays low.
        b = B if dst == "device" else max(1, B // 4)
        one = serve_ladder(scan, torch, ix, n, "one_at_a_time", 1, 1, args.serve_queries, rates, dst)
        bat = serve_ladder(scan, torch, ix, n, "batched", 4 * b, b, args.serve_queries, rates, dst)
        top = sustainable(one["ladder"])
        budget = top["p99_ms"] if top else None
        best = sustainable(bat["ladder"], budget) if budget else None
        res[dst] = {"one_at_a_time": one, "batched": bat,
                    "p99_budget_ms": budget,
                    "one_at_a_time_max_qps": top["achieved_qps"] if top else 0.0,
                    "batched_max_qps_within_budget": best["achieved_qps"] if best else 0.0}
    return res


def query_bytes(scan, ix, mus, epss):
    """Per-query algorithmic bytes, B_q(mu, eps) = 4 K + 24 sum over the K
    cores u of (p_u + 1) + 8 n: the core ids, each core's eps-prefix of its
    neighbour order (ids, similarities and the neighbours' core tests) and the
    per-vertex state read and memberships written; p_u = the length of u's
    eps-prefix. Evaluated on the host from the exported index."""
    off = scan.scan_index_export(ix, scan.ARR_OFFSETS)
    no_sim = scan.scan_index_export(ix, scan.ARR_NO_SIM)
    co_off = scan.scan_index_export(ix, scan.ARR_CO_OFF)
    co_ids = scan.scan_index_export(ix, scan.ARR_CO_IDS)
    co_thr = scan.scan_index_export(ix, scan.ARR_CO_THR)
    n, dmax = ix.info.n, ix.info.dmax
    prefix = {}
    out = []
    for mu, eps in zip(mus, epss):
        mu, eps = int(mu), float(eps)
        if eps not in prefix:
            c = np.concatenate([[0], np.cumsum(no_sim >= eps)])
            prefix[eps] = c[off[1:]] - c[off[:-1]]
        K, z = 0, 0
        if mu <= dmax + 1:
            b, e = co_off[mu], co_off[mu + 1]
            K = int(np.searchsorted(-co_thr[b:e], -eps, side="right"))
            z = int((prefix[eps][co_ids[b:b + K]] + 1).sum())
        out.append(4 * K + 24 * z + 8 * n)
    return np.array(out, np.int64)


def closed_loop_queries(scan, torch, ix, n, queries, B):
    """mu ~ U{2..16}, eps ~ U{0.10, ..., 0.90}: synchronous one at a time vs
    scan_query_batch of B; each query's bytes B_q and the rate they imply at
    its one-at-a-time latency."""
    rng = np.random.default_rng(7)
    q_mu = rng.integers(2, 17, queries)
    q_eps = np.array([(10 + 5 * k) / 100.0 for k in rng.integers(0, 17, queries)])
    memb = torch.empty(n, dtype=torch.int32, device="cuda")
    for i in range(5):
        scan.scan_query(ix, int(q_mu[i]), float(q_eps[i]), memb)
    torch.cuda.synchronize()
    single = []
    for mu, eps in zip(q_mu, q_eps):
        t = time.perf_counter()
        scan.scan_query(ix, int(mu), float(eps), memb)
        torch.cuda.synchronize()
        single.append((time.perf_counter() - t) * 1e3)
    out = torch.empty((B, n), dtype=torch.int32, device="cuda")
    batched, tb0 = [], time.perf_counter()
    for i in range(0, queries, B):
        t = time.perf_counter()
        scan.scan_query_batch(ix, q_mu[i:i + B], q_eps[i:i + B], out[: len(q_mu[i:i + B])])
        torch.cuda.synchronize()
        batched += [(time.perf_counter() - t) * 1e3] * len(q_mu[i:i + B])
    tb = time.perf_counter() - tb0
    bq = query_bytes(scan, ix, q_mu, q_eps)
    rate = bq / (np.array(single) * 1e-3) / 1e9
    per_query = [{"mu": int(m), "eps": float(e), "bytes": int(b), "ms": float(t), "gbs": float(r)}
                 for m, e, b, t, r in zip(q_mu, q_eps, bq, single, rate)]
    return {"queries": queries, "batch": B,
            "bytes_model": "B_q = 4 K + 24 sum_cores (p_u + 1) + 8 n",
            "bytes_per_query": {"p50": float(np.percentile(bq, 50)), "min": int(bq.min()), "max": int(bq.max()),
                                "gbs_at_one_at_a_time_p50": float(np.percentile(rate, 50)),
                                "gbs_at_one_at_a_time_max": float(rate.max())},
            "per_query": per_query,
            "one_at_a_time": {"p50_ms": float(np.percentile(single, 50)), "p99_ms": float(np.percentile(single, 99)),
                              "qps": queries / (sum(single) / 1e3)},
            "batched": {"p50_ms": float(np.percentile(batched, 50)), "p99_ms": float(np.percentile(batched, 99)),
                        "qps": queries / tb}}


def roles_timing(scan, torch, ix, g, count=20):
    """Hubs and outliers (scan_query_roles) after seeded queries: device time
    per call (hipEvents) and its bytes, 8 B per neighbour of an unclustered
    vertex (neighbour id and its membership) + 5 B per vertex (membership read,
    role written); an upper bound, the scan of a hub stops early."""
    rng = np.random.default_rng(11)
    deg = np.diff(g.off)
    memb = torch.empty(g.n, dtype=torch.int32, device="cuda")
    roles = torch.empty(g.n, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    rows = []
    for _ in range(count):
        mu, eps = int(rng.integers(2, 17)), (10 + 5 * int(rng.integers(0, 17))) / 100.0
        scan.scan_query(ix, mu, eps, memb)
        scan.scan_query_roles(ix, memb, roles)  # warm
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        scan.scan_query_roles(ix, memb, roles)
        e1.record(stream)
        torch.cuda.synchronize()
        m = memb.cpu().numpy()
        r = roles.cpu().numpy()
        nbytes = 8 * int(deg[m < 0].sum()) + 5 * g.n
        rows.append((e0.elapsed_time(e1), nbytes, int((r == 1).sum()), int((r == 2).sum()), mu, eps))
    rows.sort()
    ms, nbytes, hubs, outl, mu, eps = rows[len(rows) // 2]
    return {"calls": count, "ms_p50": ms, "ms_max": rows[-1][0], "at_p50": {"mu": mu, "eps": eps, "hubs": hubs,
            "outliers": outl, "bytes_bound": nbytes, "gbs_bound": nbytes / (ms * 1e-3) / 1e9}}


def weighted_timing(scan, torch, graphgen, g, off, adj, st, steps):
    """Section 3.1's weighted cosine on the same graph, with seeded weights
    uniform in [0.05, 1) (equal for both directions of an edge): builds timed
    like the headline, the split between the square sums and the owner
    products (hipEvents), the owner kernel's algorithmic bytes and a sampled
    oracle rate. Owner kernel bytes: every lower row's ids and weights once
    per owned edge (12 B per id) and one 4 B tile probe per id (16 W_min),
    both similarity slots (16 B per edge) and the owner rows' ids and weights
    (12 B per slot)."""
    import oracle

    wh = graphgen.edge_weights(g, 2020)
    w = torch.from_numpy(wh).cuda()
    ms, dev_ms, profs, _ = timed_builds(
        scan, torch, lambda: [scan.scan_build_index_weighted(off, adj, w, scan.SCAN_PROFILE)], steps, 1)
    phases = {k: med(profs, k) for k in PHASES}
    owner_ms = phases["intersect_big_ms"]
    nbytes = 16 * st["w_min"] + 16 * g.num_edges + 12 * g.nnz
    k = 20_000
    rng = np.random.default_rng(7)
    slots = rng.integers(0, g.nnz, k)
    u = np.searchsorted(g.off, slots, side="right") - 1
    t = time.perf_counter()
    oracle.weighted_edge_similarities(g, wh, u, g.adj[slots].astype(np.int64))
    tc = time.perf_counter() - t
    return {"value": g.num_edges / (ms * 1e-3), "unit": "edges/s", "ms_per_step": ms, "device_ms_per_step": dev_ms,
            "phases_ms": phases, "weights": "uniform [0.05, 1), seed 2020, symmetric",
            "square_sums_ms": phases["intersect_small_ms"], "k_w_owner": {
                "bytes": nbytes, "launch_ms": owner_ms, "achieved_gbs": nbytes / max(owner_ms, 1e-6) / 1e6,
                "frac": nbytes / max(owner_ms, 1e-6) / 1e6 / HBM_PEAK_GBS},
            "cpu_baseline": {"value": k / tc, "unit": "edges/s", "cores": 1, "kind": "oracle",
                             "sample": f"weighted similarity of {k} uniformly sampled edges, one thread, {tc:.1f} s "
                                       f"(similarity phase only)"}}


def lsh_timing(scan, torch, graphgen, g, off, adj, exact_ms, steps, k=256):
    """Section 5's approximate index on the same graph with k = 256 samples:
    SimHash (cosine; seeded Gaussian draws, n x k) and k-partition MinHash
    (Jaccard; a seeded permutation), edges between two vertices of degree > k
    (> 3k/2 for Jaccard) approximated, the rest exact. Builds timed like the
    headline; the draws are resident before timing."""
    deg = np.diff(g.off)
    rows = np.repeat(np.arange(g.n), deg)
    out = {"samples": k}
    for name, kind in (("simhash_cosine", scan.COSINE), ("minhash_jaccard", scan.JACCARD)):
        if kind == scan.COSINE:
            gauss, perm = torch.from_numpy(graphgen.gaussians(g.n, k, 256)).cuda(), None
            hi = deg > k
        else:
            gauss, perm = None, torch.from_numpy(graphgen.permutation(g.n, 256)).cuda()
            hi = 2 * deg > 3 * k
        ms, dev_ms, profs, _ = timed_builds(
            scan, torch, lambda: [scan.scan_build_index_lsh(off, adj, kind, k, gauss, perm, None, scan.SCAN_PROFILE)],
            steps, 1)
        phases = {k_: med(profs, k_) for k_ in PHASES}
        slots = int((hi[rows] & hi[g.adj]).sum())
        entries = int((deg[hi] + 1).sum())  # sketched closed-neighbourhood entries
        # sketches: SimHash gathers k coordinates (8 B) per entry, MinHash one
        # permuted id (4 B) and the entry's id (4 B); estimates read two sketches
        # per approximated slot (k bits, or k 4-byte bins) and write 8 B
        sk_bytes = entries * (8 * k if kind == scan.COSINE else 8)
        est_bytes = slots * ((2 * k // 8 if kind == scan.COSINE else 8 * k) + 8)
        out[name] = {"value": g.num_edges / (ms * 1e-3), "unit": "edges/s", "ms_per_step": ms,
                     "device_ms_per_step": dev_ms, "phases_ms": phases,
                     "approximated_slots": slots, "sketched_vertices": int(hi.sum()),
                     "sketch_bytes": sk_bytes, "estimate_bytes": est_bytes,
                     "similarity_phase_gbs": (sk_bytes + est_bytes) / (phases["intersect_ms"] * 1e-3) / 1e9,
                     "over_exact_ms": ms - exact_ms}
        del gauss, perm
    return out


def sweep_timing(scan, torch, ix, dmax, batch=32):
    """Section 7.3.4's parameter selection on the index: the modularity of
    every (mu, eps) of the paper's grid Sigma (mu = 2, 4, ..., 2^18 by 99
    eps = .01 .. .99: 1,782 cells), as batched queries plus device modularity.
    Cells with mu > dmax + 1 have no cores: every vertex is a singleton."""
    grid = scan.paper_sweep_grid()
    mus = np.array([m for m, _ in grid], np.int32)
    epss = np.array([e for _, e in grid])
    scan.scan_sweep_modularity(ix, mus[:batch], epss[:batch], batch=batch)  # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    q = scan.scan_sweep_modularity(ix, mus, epss, batch=batch)
    wall = time.perf_counter() - t
    best = int(np.argmax(q))
    return {"queries": len(grid), "cells_mu_above_dmax_plus_1": int((mus > dmax + 1).sum()), "batch": batch,
            "wall_s": wall, "queries_per_s": len(grid) / wall,
            "best": {"mu": int(mus[best]), "eps": float(epss[best]), "modularity": float(q[best])}}


# ---------------------------------------------------------------------------
# Quality of approximate clusterings (Section 7.3.4)


def _labels(m):
    """Unclustered vertices (-1) as singletons: label n + v."""
    m = np.asarray(m, np.int64)
    return np.where(m >= 0, m, len(m) + np.arange(len(m)))


def adjusted_rand_index(a, b) -> float:
    """Section 7.2's adjusted Rand index of two clusterings (membership
    arrays, -1 = unclustered = a cluster of its own), from the contingency
    counts n_ij and their row and column sums, in exact integers up to the
    last division."""
    la, lb = _labels(a), _labels(b)
    n = len(la)
    if n < 2:
        return 1.0

    def pairs(cnt):
        cnt = cnt.astype(object)
        return int(sum(c * (c - 1) // 2 for c in cnt))

    _, ia = np.unique(la, return_inverse=True)
    _, ib = np.unique(lb, return_inverse=True)
    _, nij = np.unique(ia.astype(np.int64) * (ib.max() + 1) + ib, return_counts=True)
    sij, si, sj = pairs(nij), pairs(np.bincount(ia)), pairs(np.bincount(ib))
    total = n * (n - 1) // 2
    expected = si * sj / total
    top = 0.5 * (si + sj) - expected
    return 1.0 if top == 0 else (sij - expected) / top


def best_cell(scan, ix, grid, batch=32):
    mus = np.array([m for m, _ in grid], np.int32)
    epss = np.array([e for _, e in grid])
    q = scan.scan_sweep_modularity(ix, mus, epss, batch=batch)
    i = int(np.argmax(q))
    return int(mus[i]), float(epss[i]), float(q[i])


def approx_quality(scan, torch, graphgen, name, g, off, adj, k, seeds=5):
    """For SimHash (cosine) and MinHash (Jaccard) with k samples, over
    `seeds` draws: the best modularity over Sigma of the approximate index,
    and the ARI against the exact index's clustering at the exact index's
    best (mu, eps) of the approximate index's clustering at that same cell
    and at its own best cell (Section 7.3.4)."""
    grid = scan.paper_sweep_grid()
    deg = np.diff(g.off)
    out = {"graph": name, "samples": k, "seeds": seeds}
    for label, kind in (("simhash_cosine", scan.COSINE), ("minhash_jaccard", scan.JACCARD)):
        hi = deg > k if kind == scan.COSINE else 2 * deg > 3 * k
        exact = scan.scan_build_index(off, adj, kind, 0)
        mu, eps, q = best_cell(scan, exact, grid)
        ref = scan.scan_query(exact, mu, eps).cpu().numpy()
        rows = []
        for sd in range(seeds):
            if kind == scan.COSINE:
                gauss, perm = torch.from_numpy(graphgen.gaussians(g.n, k, 500 + sd)).cuda(), None
            else:
                gauss, perm = None, torch.from_numpy(graphgen.permutation(g.n, 500 + sd)).cuda()
            ax = scan.scan_build_index_lsh(off, adj, kind, k, gauss, perm, None, 0)
            amu, aeps, aq = best_cell(scan, ax, grid)
            am = scan.scan_query(ax, mu, eps).cpu().numpy()
            ab = scan.scan_query(ax, amu, aeps).cpu().numpy()
            rows.append({"seed": 500 + sd, "best_modularity": aq, "best": [amu, aeps],
                         "ari_at_exact_best": adjusted_rand_index(am, ref),
                         "ari_best_vs_exact_best": adjusted_rand_index(ab, ref)})
            del ax, gauss, perm
        out[label] = {"exact_best": {"mu": mu, "eps": eps, "modularity": q,
                                     "clusters": int(len(np.unique(ref[ref >= 0])))},
                      "sketched_vertices": int(hi.sum()),
                      "approx_best_modularity_mean": float(np.mean([r["best_modularity"] for r in rows])),
                      "ari_mean": float(np.mean([r["ari_at_exact_best"] for r in rows])),
                      "ari_best_vs_exact_best_mean": float(np.mean([r["ari_best_vs_exact_best"] for r in rows])),
                      "trials": rows}
        del exact
    return out


# ---------------------------------------------------------------------------
# Workloads


def record(value, steps, warmup, ms, dtype, config, **extra):
    rec = {"metric": METRIC, "value": value, "unit": "edges/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic", "config": config}
    rec.update(extra)
    return rec


def rmat_workload(args, scan, torch, graphgen):
    scale, ef = (20, 16) if args.workload == "rmat20" else (23, 32)
    s_off = 4 if scale == 20 else 8
    t0 = time.time()
    g = graphgen.rmat(scale, ef, seed=scale)
    st = graphgen.degree_stats(g)
    log(f"graph rmat{scale}: n={g.n} |E|={g.num_edges} nnz={g.nnz} dmax={st['dmax']} w_min={st['w_min']} "
        f"({time.time() - t0:.1f}s)")
    off = torch.from_numpy(g.off.astype(np.int32 if s_off == 4 else np.int64)).cuda()
    adj = torch.from_numpy(g.adj).cuda()
    torch.cuda.synchronize()
    kinds = [scan.COSINE] if scale == 20 else [scan.COSINE, scan.JACCARD]
    tune, tinfo = autotune(scan, [(off, adj)], scan.COSINE, args.tune, reps=2 if scale == 20 else 1)
    split = graphgen.owner_split(g, tune["small_max"])
    bm = byte_model(st, split, s_off, np.diff(g.off), tune["small_max"])
    results = {}
    for kind in kinds:
        ms, dev_ms, profs, ixs = timed_builds(
            scan, torch, lambda: [scan.scan_build_index(off, adj, kind, scan.SCAN_PROFILE, tune=tune)],
            args.steps, args.warmup)
        phases = {k: med(profs, k) for k in PHASES}
        log(f"kind {kind}: {ms:.2f} ms/step wall, device {dev_ms:.2f} ms/step, phases {phases}")
        results[kind] = (ms, dev_ms, phases, ixs[0])
    ms, dev_ms, phases, ix = results[scan.COSINE]
    value = g.num_edges / (ms * 1e-3)
    workload = f"rmat{scale}_cosine_index_build"
    config = {"workload": workload, "scale": scale, "edge_factor": ef, "abcd": [0.57, 0.19, 0.19, 0.05],
              "seed": scale, "n": g.n, "edges": g.num_edges, "nnz": g.nnz, "dmax": st["dmax"],
              "hubs_deg_gt_1e5": int((np.diff(g.off) > 100_000).sum()), "w_min": st["w_min"],
              "offsets": "int32" if s_off == 4 else "int64", "ids": "int32", "similarity": "cosine",
              "tune": tune}
    extra = {"phases_ms": phases, "device_ms_per_step": dev_ms,
             "tune": dict(tinfo, **tune), "owner_split": split,
             "roofline": kernel_roofline(bm, phases, tune, workload),
             "build_roofline": build_roofline(bm, phases["total_ms"], workload, tune),
             "k_small_owner": {"bytes": bm["k_small_owner"], "model_bytes": bm["k_small_owner_model"],
                               "launch_ms": phases["intersect_small_ms"],
                               "achieved_gbs": bm["k_small_owner"] / max(phases["intersect_small_ms"], 1e-6) / 1e6}}
    if scan.JACCARD in results:
        jms, jdev, jph, _ = results[scan.JACCARD]
        extra["jaccard"] = {"value": g.num_edges / (jms * 1e-3), "ms_per_step": jms, "device_ms_per_step": jdev,
                            "phases_ms": jph}
    if scale == 20 and not args.no_lsh:
        extra["lsh"] = lsh_timing(scan, torch, graphgen, g, off, adj, ms, args.steps)
        log(f"lsh: {extra['lsh']}")
        if not args.no_quality:
            qual = [approx_quality(scan, torch, graphgen, "rmat20", g, off, adj, 256)]
            # planted communities dense enough that every vertex is above
            # both degree thresholds at k = 64 (all edges approximated):
            # 20 blocks of 200, p_in = 0.6, p_out = 0.01 (degree about 157)
            s2 = graphgen.sbm(4000, 20, 0.6, 0.01, seed=4000)
            o2 = torch.from_numpy(s2.off.astype(np.int32)).cuda()
            a2 = torch.from_numpy(s2.adj).cuda()
            qual.append(approx_quality(scan, torch, graphgen, "sbm4000_dense", s2, o2, a2, 64))
            extra["approx_quality"] = qual
            log(f"approximate quality: {qual}")
    if scale == 20 and not args.no_weighted:
        extra["weighted"] = weighted_timing(scan, torch, graphgen, g, off, adj, st, args.steps)
        log(f"weighted: {extra['weighted']}")
    if scale == 20 and not args.no_queries:
        extra["query"] = closed_loop_queries(scan, torch, ix, g.n, args.queries, args.query_batch)
        log(f"queries: {extra['query']}")
        extra["roles"] = roles_timing(scan, torch, ix, g)
        log(f"roles: {extra['roles']}")
        extra["sweep"] = sweep_timing(scan, torch, ix, st["dmax"])
        log(f"sweep: {extra['sweep']}")
        if not args.no_serve:
            extra["serving"] = serving(scan, torch, ix, g.n, args)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = rmat_cpu_baseline(args, g, scale)
        log(f"cpu baseline: {cpu}")
    extra["cpu_baseline"] = cpu
    return record(value, args.steps, args.warmup, ms, "f64", config, **extra)


def host_info(oracle):
    return {"cpu_model": oracle.cpu_model(), "hardware_concurrency": oracle.hardware_concurrency(),
            "os_cpu_count": os.cpu_count()}


def rmat_cpu_baseline(args, g, scale):
    """The oracle on the host cores, untuned: one full cosine build on all
    cores (R-MAT-20; on R-MAT-23 the similarity of sampled edges, the full
    build being too slow), and the similarity of uniformly sampled edges on
    one thread and on all cores (each edge computed alone)."""
    import oracle

    info = host_info(oracle)
    threads = args.cpu_threads or info["hardware_concurrency"]
    rng = np.random.default_rng(5)
    k = 200_000 if scale == 20 else 100_000
    slots = rng.integers(0, g.nnz, k)
    u = np.searchsorted(g.off, slots, side="right") - 1
    v = g.adj[slots].astype(np.int64)
    t = time.perf_counter()
    oracle.edge_similarities(g, u, v, oracle.COSINE, threads=1)
    t1 = time.perf_counter() - t
    t = time.perf_counter()
    oracle.edge_similarities(g, u, v, oracle.COSINE, threads=threads)
    tn = time.perf_counter() - t
    sampled = {"one_thread": {"value": k / t1, "unit": "edges/s", "cores": 1, "seconds": t1},
               "all_cores": {"value": k / tn, "unit": "edges/s", "cores": threads, "seconds": tn},
               "sample": f"similarity of {k} uniformly sampled CSR slots of the same graph, each edge alone "
                         f"(the similarity phase only)"}
    if scale == 20:
        log(f"cpu baseline: oracle full build on {threads} threads ...")
        t = time.perf_counter()
        oracle.build_index(g, oracle.COSINE, threads=threads)
        tc = time.perf_counter() - t
        return dict({"value": g.num_edges / tc, "unit": "edges/s", "cores": threads, "kind": "oracle",
                     "sample": f"one full cosine index build of the same R-MAT-20 graph (similarities, "
                               f"neighbour order, core order) on {threads} threads, {tc:.1f} s",
                     "sampled_similarity": sampled}, **info)
    return dict({"value": sampled["all_cores"]["value"], "unit": "edges/s", "cores": threads, "kind": "oracle",
                 "sample": sampled["sample"] + f", on {threads} threads", "sampled_similarity": sampled}, **info)


def sbm_batch_workload(args, scan, torch, graphgen):
    t0 = time.time()
    gs = graphgen.batch_sbm(256)
    edges = sum(g.num_edges for g in gs)
    log(f"256 SBM graphs: sum n={sum(g.n for g in gs)} sum |E|={edges} ({time.time() - t0:.1f}s)")
    dev = [(torch.from_numpy(g.off.astype(np.int64)).cuda(), torch.from_numpy(g.adj).cuda()) for g in gs]
    torch.cuda.synchronize()
    tune, tinfo = autotune(scan, dev, scan.COSINE, args.tune, reps=1)
    ms, dev_ms, profs, _ = timed_builds(
        scan, torch, lambda: scan.scan_build_index_batch(dev, scan.COSINE, scan.SCAN_PROFILE, tune=tune),
        args.steps, args.warmup)
    phases = {k: med(profs, k) for k in PHASES}
    log(f"merged: {ms:.2f} ms/step, phases {phases}")
    # 256 separate builds on the same stream, same shapes
    for off, adj in dev[:4]:
        scan.scan_build_index(off, adj, scan.COSINE, 0, tune=tune)
    torch.cuda.synchronize()
    seq = []
    for _ in range(max(1, args.steps // 2)):
        t = time.perf_counter()
        ixs = [scan.scan_build_index(off, adj, scan.COSINE, 0, tune=tune) for off, adj in dev]
        torch.cuda.synchronize()
        seq.append((time.perf_counter() - t) * 1e3)
        del ixs
    seq_ms = float(np.median(seq))
    log(f"sequential: {seq_ms:.2f} ms per 256 builds")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        info = host_info(oracle)
        threads = args.cpu_threads or info["hardware_concurrency"]
        sample = gs[:32]
        t = time.perf_counter()
        for g in sample:
            oracle.build_index(g, oracle.COSINE, threads=threads)
        tc = time.perf_counter() - t
        t = time.perf_counter()
        for g in sample[:8]:
            oracle.build_index(g, oracle.COSINE, threads=1)
        t1 = time.perf_counter() - t
        cpu = dict({"value": sum(g.num_edges for g in sample) / tc, "unit": "edges/s", "cores": threads,
                    "kind": "oracle",
                    "sample": f"full cosine index builds of the first 32 of the 256 graphs on {threads} threads, "
                              f"{tc:.1f} s",
                    "one_thread": {"value": sum(g.num_edges for g in sample[:8]) / t1, "unit": "edges/s",
                                   "cores": 1, "sample": f"full builds of the first 8 graphs on one thread, "
                                                         f"{t1:.1f} s"}}, **info)
        log(f"cpu baseline: {cpu}")
    # memory-model bytes summed over the graphs (int64 offsets), and the
    # dominant kernel class of this workload: the small owners
    bm = {"build": 0, "build_model": 0, "floor": 0, "k_small_owner": 0, "k_small_owner_model": 0,
          "k_big_owner": 0, "k_big_owner_model": 0}
    for g in gs:
        b = byte_model(graphgen.degree_stats(g), graphgen.owner_split(g, tune["small_max"]), 8, np.diff(g.off),
                       tune["small_max"])
        for key in bm:
            bm[key] += b[key]
    sec = phases["intersect_small_ms"] * 1e-3
    small_roof = {"bound": "hbm", "kernel": "k_small_owner (both launches)",
                  "achieved": bm["k_small_owner"] / sec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": bm["k_small_owner"] / sec / 1e9 / HBM_PEAK_GBS, "traffic": None,
                  "traffic_source": "not taken for this workload", "bytes_per_launch": bm["k_small_owner"],
                  "bytes_model": "4 B per streamed lower-row id + 16 B per owner slot + 16 B per owned edge",
                  "launch_ms": phases["intersect_small_ms"], "model_bytes_per_launch": bm["k_small_owner_model"],
                  "model_frac": bm["k_small_owner_model"] / sec / 1e9 / HBM_PEAK_GBS}
    config = {"workload": "sbm256_batched_cosine_index_build", "graphs": 256, "seed": 256,
              "n_range": [1000, 200000], "blocks": [5, 200], "avg_degree": [8, 64], "p_out_over_p_in": 0.02,
              "sum_n": int(sum(g.n for g in gs)), "edges": int(edges), "offsets": "int64", "tune": tune}
    return record(edges / (ms * 1e-3), args.steps, args.warmup, ms, "f64", config,
                  phases_ms=phases, device_ms_per_step=dev_ms, tune=dict(tinfo, **tune),
                  roofline=small_roof, build_roofline=build_roofline(bm, phases["total_ms"]),
                  sequential={"ms_per_256_builds": seq_ms, "edges_per_s": edges / (seq_ms * 1e-3)},
                  speedup_vs_sequential=seq_ms / ms, cpu_baseline=cpu)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["rmat20", "rmat23", "sbm256"], default="rmat20")
    ap.add_argument("--tune", default="auto", help="auto | default | small_max=..,spc=..,wbits=..")
    ap.add_argument("--queries", type=int, default=200)
    ap.add_argument("--query-batch", type=int, default=25)
    ap.add_argument("--serve-queries", type=int, default=20000)
    ap.add_argument("--serve-batch", type=int, default=32)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-queries", action="store_true")
    ap.add_argument("--no-weighted", action="store_true", help="skip the weighted-cosine build timing")
    ap.add_argument("--no-lsh", action="store_true", help="skip the approximate (LSH) build timing")
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the approximate-vs-exact clustering quality (ARI, best modularity)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB (a known-size "
                         "reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the index build and queries run on a single MI355X); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import graphgen
    import paper_2012_11188_amd as scan

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # known-size references for the HBM byte counters: a copy (MiB read +
        # MiB written), a sum (MiB read) and a fill (MiB written) of int32
        src = torch.ones(args.copy_calibration << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        total = int(src.sum(dtype=torch.int64).item())
        dst.fill_(3)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB copied, summed ({total}) and filled")
        del src, dst
    if args.workload == "sbm256":
        rec = sbm_batch_workload(args, scan, torch, graphgen)
    else:
        rec = rmat_workload(args, scan, torch, graphgen)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
