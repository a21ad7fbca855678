"""Exact index-based SCAN on AMD MI355X — Python binding of libscan.so.

Argument marshalling only: every step of the index build and of the queries
runs in the HIP kernels of ``csrc/`` behind the C ABI of ``include/scan.h``.
PyTorch provides device memory and streams. If libscan.so is missing or no
GPU is visible, calls raise; there is no CPU fallback.

Method: Tseng, Dhulipala and Shun, "Parallel Index-Based Structural Graph
Clustering and Its Approximation" (SIGMOD 2021): similarities over closed
neighbourhoods (Section 3.1), the neighbour/core-order index (Section 3.2,
Algorithm 2) and (mu, eps) queries (Section 4.2, Algorithms 3-5; border rule
of Section 7.3.4).
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscan.so")

SCAN_OK, SCAN_EINVAL, SCAN_EGRAPH, SCAN_ENOMEM, SCAN_EDEVICE, SCAN_EBUSY = 0, -1, -2, -3, -4, -5
COSINE, JACCARD, WEIGHTED_COSINE = 0, 1, 2
SCAN_VALIDATE, SCAN_KEEP_SIMS, SCAN_KEEP_COUNTS, SCAN_PROFILE = 1, 2, 4, 8
SCAN_TUNE_SEARCH_WINDOWS = 1
(ARR_OFFSETS, ARR_NO_IDS, ARR_NO_SIM, ARR_CO_OFF, ARR_CO_IDS, ARR_CO_THR, ARR_SIMS,
 ARR_COUNTS) = range(8)
_ARR_DTYPE = {ARR_OFFSETS: np.int64, ARR_NO_IDS: np.int32, ARR_NO_SIM: np.float64,
              ARR_CO_OFF: np.int64, ARR_CO_IDS: np.int32, ARR_CO_THR: np.float64,
              ARR_SIMS: np.float64, ARR_COUNTS: np.int32}
_STATUS = {SCAN_EINVAL: "SCAN_EINVAL", SCAN_EGRAPH: "SCAN_EGRAPH", SCAN_ENOMEM: "SCAN_ENOMEM",
           SCAN_EDEVICE: "SCAN_EDEVICE", SCAN_EBUSY: "SCAN_EBUSY"}


class ScanError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("offset_bits", ctypes.c_int32),
                ("on_device", ctypes.c_int32), ("offsets", ctypes.c_void_p), ("adj", ctypes.c_void_p)]


class _Lsh(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int32), ("reserved", ctypes.c_int32), ("gauss", ctypes.c_void_p),
                ("perm", ctypes.c_void_p), ("weights", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("dmax", ctypes.c_int64),
                ("kind", ctypes.c_int32), ("flags", ctypes.c_int32), ("device_bytes", ctypes.c_int64)]


class _Profile(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double), ("prepare_ms", ctypes.c_double), ("plan_ms", ctypes.c_double),
                ("intersect_ms", ctypes.c_double), ("no_sort_ms", ctypes.c_double),
                ("core_order_ms", ctypes.c_double), ("intersect_small_ms", ctypes.c_double),
                ("intersect_big_ms", ctypes.c_double), ("intersect_launches", ctypes.c_int32),
                ("small_owners", ctypes.c_int32), ("big_chunks", ctypes.c_int32), ("window_bits", ctypes.c_int32)]


class _Tune(ctypes.Structure):
    _fields_ = [("small_max", ctypes.c_int32), ("spc", ctypes.c_int32), ("wbits", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("memory_budget", ctypes.c_int64), ("use_graph", ctypes.c_int32)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)

# Every symbol include/scan.h declares (checked by the CPU tests).
EXPORTS = [
    "scan_set_allocator", "scan_build_index", "scan_build_index_batch", "scan_build_index_weighted",
    "scan_build_index_lsh", "scan_query",
    "scan_query_ex", "scan_query_batch", "scan_index_get_info", "scan_index_export",
    "scan_index_device_ptr", "scan_index_free", "scan_server_create", "scan_server_submit",
    "scan_server_submit_ex", "scan_server_poll", "scan_server_wait", "scan_server_destroy", "scan_last_error",
    "scan_version", "scan_similarity_values", "scan_index_build_profile", "scan_build_index_ex",
    "scan_autotune", "scan_segmented_sort", "scan_query_roles", "scan_query_modularity",
    "scan_sweep_modularity", "scan_query_noalloc",
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libscan.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2012_11188_amd.build_lib`")
    # PyTorch ships its own HIP runtime under the same soname as the system
    # one. Loading torch first makes the library bind to that copy, so the
    # process has one HIP runtime; loading the library first would bring in a
    # second one, and the two do not share devices.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, i64, f64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_uint32, ctypes.c_uint64)
    P = ctypes.POINTER
    sig = {
        "scan_set_allocator": ([_ALLOC_FN, _RELEASE_FN, vp], i32),
        "scan_build_index": ([P(_Csr), i32, u32, vp, P(vp)], i32),
        "scan_build_index_batch": ([P(_Csr), i32, i32, u32, vp, P(vp)], i32),
        "scan_build_index_weighted": ([P(_Csr), vp, u32, vp, P(vp)], i32),
        "scan_build_index_lsh": ([P(_Csr), i32, P(_Lsh), u32, vp, P(vp)], i32),
        "scan_build_index_ex": ([P(_Csr), i32, i32, u32, P(_Tune), vp, P(vp)], i32),
        "scan_autotune": ([P(_Csr), i32, i32, i32, vp, P(_Tune), P(ctypes.c_float)], i32),
        "scan_segmented_sort": ([vp, i64, vp, vp, vp, vp], i32),
        "scan_query": ([vp, i32, f64, vp], i32),
        "scan_query_ex": ([vp, i32, f64, vp, vp, i32, vp], i32),
        "scan_query_batch": ([vp, i32, vp, vp, vp, i32, vp], i32),
        "scan_query_noalloc": ([vp, i32, f64, vp, vp, vp], i32),
        "scan_query_roles": ([vp, vp, vp, vp], i32),
        "scan_query_modularity": ([vp, vp, P(f64), vp], i32),
        "scan_sweep_modularity": ([vp, i32, vp, vp, i32, vp, vp], i32),
        "scan_index_get_info": ([vp, P(_Info)], i32),
        "scan_index_export": ([vp, i32, vp, i64], i32),
        "scan_index_device_ptr": ([vp, i32, P(vp), P(i64)], i32),
        "scan_index_free": ([vp], None),
        "scan_server_create": ([vp, P(_ServerOpts), P(vp)], i32),
        "scan_server_submit": ([vp, i32, f64, vp, P(u64)], i32),
        "scan_server_submit_ex": ([vp, i32, f64, vp, i32, vp, P(u64)], i32),
        "scan_server_poll": ([vp, u64, P(i32)], i32),
        "scan_server_wait": ([vp, u64], i32),
        "scan_server_destroy": ([vp], None),
        "scan_last_error": ([], ctypes.c_char_p),
        "scan_version": ([], ctypes.c_char_p),
        "scan_similarity_values": ([i32, i64, vp, vp, vp, vp], i32),
        "scan_index_build_profile": ([vp, P(_Profile)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(st: int):
    if st != SCAN_OK:
        raise ScanError(st, load_library().scan_last_error().decode())


# ---------------------------------------------------------------------------
# Device memory and streams from PyTorch.

_torch_hooks = None


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the SCAN library runs on the GPU only")
    return torch


def use_torch_allocator(enable: bool = True):
    """Routes the library's device allocations through PyTorch's caching
    allocator (stream ordered). Called on first use."""
    global _torch_hooks
    lib = load_library()
    if not enable:
        _check(lib.scan_set_allocator(_ALLOC_FN(), _RELEASE_FN(), None))
        _torch_hooks = None
        return
    torch = _torch()

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), int(stream or 0))
        except Exception:
            return None

    def _release(ptr, nbytes, stream, ctx):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass

    hooks = (_ALLOC_FN(_alloc), _RELEASE_FN(_release))
    _check(lib.scan_set_allocator(hooks[0], hooks[1], None))
    _torch_hooks = hooks


def _stream_handle(stream) -> int:
    torch = _torch()
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _hold_inputs(stream_handle: int, *objs) -> None:
    """A build returns before the device has read its device inputs. When it
    runs on a stream other than PyTorch's current one, the input tensors are
    marked as used there, so that the caching allocator does not hand their
    memory to the current stream while the build may still read it."""
    import torch

    if stream_handle == torch.cuda.current_stream().cuda_stream:
        return
    ext = None
    todo = list(objs)
    while todo:
        o = todo.pop()
        if isinstance(o, (tuple, list)):
            todo.extend(o)
        elif isinstance(o, torch.Tensor) and o.is_cuda and o.numel():
            if ext is None:
                ext = torch.cuda.ExternalStream(stream_handle)
            o.record_stream(ext)


def _ready():
    lib = load_library()
    _torch()
    if _torch_hooks is None:
        use_torch_allocator(True)
    return lib


# ---------------------------------------------------------------------------
# Index


@dataclass
class IndexInfo:
    n: int
    nnz: int
    dmax: int
    kind: int
    flags: int
    device_bytes: int


class Index:
    """A device-resident SCAN index (NO + CO). Freed with the object."""

    def __init__(self, handle: int, stream: int):
        self._h = ctypes.c_void_p(handle)
        self.stream = stream
        self.info = scan_index_get_info(self)

    @property
    def n(self):
        return self.info.n

    def free(self):
        if self._h is not None and self._h.value:
            load_library().scan_index_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _csr_struct(off, adj):
    """Builds a scan_csr from torch tensors (device) or numpy arrays (host).
    Returns (struct, keepalive)."""
    try:
        import torch
        is_tensor = isinstance(off, torch.Tensor)
    except ImportError:
        is_tensor = False
    if is_tensor:
        if off.dtype not in (torch.int32, torch.int64) or adj.dtype != torch.int32:
            raise TypeError("offsets must be int32/int64, adj int32")
        if not (off.is_cuda and adj.is_cuda):
            raise TypeError("torch tensors must be on the GPU (pass numpy arrays for host data)")
        off, adj = off.contiguous(), adj.contiguous()
        bits = 32 if off.dtype == torch.int32 else 64
        c = _Csr(off.numel() - 1, adj.numel(), bits, 1, off.data_ptr(), adj.data_ptr() if adj.numel() else None)
        return c, (off, adj)
    off = np.ascontiguousarray(off)
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    if off.dtype not in (np.int32, np.int64):
        off = off.astype(np.int64)
    bits = 32 if off.dtype == np.int32 else 64
    c = _Csr(len(off) - 1, len(adj), bits, 0, off.ctypes.data, adj.ctypes.data if len(adj) else None)
    return c, (off, adj)


def _tune_struct(tune):
    """dict (small_max / spc / wbits / flags; missing or 0 = default) -> scan_tune, or None."""
    if tune is None:
        return None
    unknown = set(tune) - {"small_max", "spc", "wbits", "flags"}
    if unknown:
        raise ValueError(f"unknown tune fields {sorted(unknown)}")
    return _Tune(int(tune.get("small_max", 0)), int(tune.get("spc", 0)), int(tune.get("wbits", 0)),
                 int(tune.get("flags", 0)))


def scan_build_index(off, adj, kind: int = COSINE, flags: int = 0, stream=None, tune=None) -> Index:
    """Builds the index (Algorithms 1 and 2) of the CSR graph (off, adj).
    tune: optional intersection shapes {"small_max", "spc", "wbits"}."""
    if tune is not None:
        return scan_build_index_batch([(off, adj)], kind, flags, stream, tune)[0]
    lib = _ready()
    c, keep = _csr_struct(off, adj)
    s = _stream_handle(stream)
    out = ctypes.c_void_p()
    _check(lib.scan_build_index(ctypes.byref(c), int(kind), int(flags), ctypes.c_void_p(s), ctypes.byref(out)))
    _hold_inputs(s, keep)
    del keep
    return Index(out.value, s)


def _numel(a) -> int:
    return int(a.numel()) if hasattr(a, "numel") else int(np.asarray(a).size)


def scan_build_index_weighted(off, adj, weights, flags: int = 0, stream=None) -> Index:
    """Builds the index under Section 3.1's weighted cosine; weights (float64,
    one per CSR slot, parallel to adj) live where the graph does: a GPU
    tensor with GPU tensors, a numpy array with numpy arrays. A weight count
    other than nnz raises ValueError before anything runs."""
    c, keep = _csr_struct(off, adj)
    if weights is None or _numel(weights) != c.nnz:
        raise ValueError(f"weights must have nnz = {c.nnz} entries")
    lib = _ready()
    if c.on_device:
        import torch
        if not (isinstance(weights, torch.Tensor) and weights.is_cuda and weights.dtype == torch.float64):
            raise TypeError("weights must be a float64 GPU tensor when the graph is on the GPU")
        weights = weights.contiguous()
        ptr = weights.data_ptr() if weights.numel() else None
    else:
        weights = np.ascontiguousarray(weights, dtype=np.float64)
        ptr = weights.ctypes.data if weights.size else None
    s = _stream_handle(stream)
    out = ctypes.c_void_p()
    _check(lib.scan_build_index_weighted(ctypes.byref(c), ctypes.c_void_p(ptr), int(flags), ctypes.c_void_p(s),
                                         ctypes.byref(out)))
    _hold_inputs(s, keep, weights)
    del keep, weights
    return Index(out.value, s)


def _side_ptr(a, on_device, dtype_np, dtype_name):
    """Pointer of an optional input living where the graph lives."""
    if a is None:
        return None, None
    if on_device:
        import torch
        if not (isinstance(a, torch.Tensor) and a.is_cuda and str(a.dtype) == "torch." + dtype_name):
            raise TypeError(f"{dtype_name} GPU tensor expected with a GPU graph")
        a = a.contiguous()
        return (a.data_ptr() if a.numel() else None), a
    a = np.ascontiguousarray(a, dtype=dtype_np)
    return (a.ctypes.data if a.size else None), a


def _check_lsh_inputs(n: int, nnz: int, kind: int, samples: int, gauss, perm, weights):
    """The draw and weight arrays must have exactly the sizes the kernels
    read: gauss n x samples (cosine kinds), perm n (Jaccard), weights nnz
    (weighted cosine). Raises ValueError otherwise, before any device work."""
    if kind in (COSINE, WEIGHTED_COSINE):
        if gauss is None or _numel(gauss) != n * int(samples):
            raise ValueError(f"SimHash needs gauss with n * samples = {n * int(samples)} values")
        if perm is not None:
            raise ValueError("perm goes with JACCARD only")
    elif kind == JACCARD:
        if perm is None or _numel(perm) != n:
            raise ValueError(f"MinHash needs perm with n = {n} values")
        if gauss is not None:
            raise ValueError("gauss goes with the cosine kinds only")
    else:
        raise ValueError(f"unknown similarity kind {kind}")
    if kind == WEIGHTED_COSINE:
        if weights is None or _numel(weights) != nnz:
            raise ValueError(f"WEIGHTED_COSINE needs weights with nnz = {nnz} values")
    elif weights is not None:
        raise ValueError("weights go with WEIGHTED_COSINE only")


def scan_build_index_lsh(off, adj, kind: int, samples: int, gauss=None, perm=None, weights=None, flags: int = 0,
                         stream=None) -> Index:
    """Approximate index (Section 5 with Section 6.3's heuristic): SimHash for
    COSINE / WEIGHTED_COSINE (gauss: n x samples float64 draws; weights for
    the weighted kind), k-partition MinHash for JACCARD (perm: uint32
    permutation of 0..n-1). Inputs live where the graph lives; arrays of any
    other size raise ValueError before anything runs."""
    c, keep = _csr_struct(off, adj)
    _check_lsh_inputs(int(c.n), int(c.nnz), int(kind), samples, gauss, perm, weights)
    lib = _ready()
    pg, kg = _side_ptr(gauss, c.on_device, np.float64, "float64")
    pp, kp = _side_ptr(perm, c.on_device, np.uint32, "uint32")
    pw, kw = _side_ptr(weights, c.on_device, np.float64, "float64")
    spec = _Lsh(int(samples), 0, pg, pp, pw)
    s = _stream_handle(stream)
    out = ctypes.c_void_p()
    _check(lib.scan_build_index_lsh(ctypes.byref(c), int(kind), ctypes.byref(spec), int(flags), ctypes.c_void_p(s),
                                    ctypes.byref(out)))
    _hold_inputs(s, keep, kg, kp, kw)
    del keep, kg, kp, kw
    return Index(out.value, s)


def _csr_array(graphs):
    structs, keep = [], []
    for off, adj in graphs:
        c, k = _csr_struct(off, adj)
        structs.append(c)
        keep.append(k)
    return (_Csr * len(structs))(*structs), keep


def scan_build_index_batch(graphs, kind: int = COSINE, flags: int = 0, stream=None, tune=None) -> list[Index]:
    """Builds one index per (off, adj) graph in merged launches."""
    lib = _ready()
    arr, keep = _csr_array(graphs)
    outs = (ctypes.c_void_p * len(arr))()
    s = _stream_handle(stream)
    t = _tune_struct(tune)
    if t is None:
        _check(lib.scan_build_index_batch(arr, len(arr), int(kind), int(flags), ctypes.c_void_p(s), outs))
    else:
        _check(lib.scan_build_index_ex(arr, len(arr), int(kind), int(flags), ctypes.byref(t), ctypes.c_void_p(s),
                                       outs))
    _hold_inputs(s, keep)
    del keep
    return [Index(outs[i], s) for i in range(len(arr))]


def scan_segmented_sort(seg_off: np.ndarray, keys: np.ndarray, ids: np.ndarray):
    """Diagnostic: per segment, (keys, ids) sorted by key desc, id asc."""
    lib = _ready()
    seg_off = np.ascontiguousarray(seg_off, dtype=np.int64)
    keys = np.ascontiguousarray(keys, dtype=np.float64)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    ko = np.empty_like(keys)
    io = np.empty_like(ids)
    _check(lib.scan_segmented_sort(seg_off.ctypes.data, len(seg_off) - 1, keys.ctypes.data, ids.ctypes.data,
                                   ko.ctypes.data, io.ctypes.data))
    return ko, io


def scan_autotune(graphs, kind: int = COSINE, reps: int = 2, stream=None) -> dict:
    """Sweeps the intersection shapes on the (off, adj) graphs (built merged)
    and returns {"small_max", "spc", "wbits", "ms"} of the fastest."""
    lib = _ready()
    arr, keep = _csr_array(graphs)
    best, ms = _Tune(), ctypes.c_float()
    _check(lib.scan_autotune(arr, len(arr), int(kind), int(reps), ctypes.c_void_p(_stream_handle(stream)),
                             ctypes.byref(best), ctypes.byref(ms)))
    del keep
    return {"small_max": best.small_max, "spc": best.spc, "wbits": best.wbits, "ms": ms.value}


def scan_index_get_info(ix: Index) -> IndexInfo:
    info = _Info()
    _check(load_library().scan_index_get_info(ix._h, ctypes.byref(info)))
    return IndexInfo(info.n, info.nnz, info.dmax, info.kind, info.flags, info.device_bytes)


def _array_count(ix: Index, what: int) -> int:
    i = ix.info
    return {ARR_OFFSETS: i.n + 1, ARR_CO_OFF: i.dmax + 3}.get(what, i.nnz)


def scan_index_export(ix: Index, what: int) -> np.ndarray:
    """Copies one index array to host memory."""
    out = np.empty(_array_count(ix, what), dtype=_ARR_DTYPE[what])
    _check(load_library().scan_index_export(ix._h, int(what), out.ctypes.data if out.size else None, out.nbytes))
    return out


def scan_index_build_profile(ix: Index) -> dict:
    """Per-phase device milliseconds of a build made with SCAN_PROFILE."""
    p = _Profile()
    _check(load_library().scan_index_build_profile(ix._h, ctypes.byref(p)))
    return {name: getattr(p, name) for name, _ in _Profile._fields_}


def scan_index_device_ptr(ix: Index, what: int):
    p, b = ctypes.c_void_p(), ctypes.c_int64()
    _check(load_library().scan_index_device_ptr(ix._h, int(what), ctypes.byref(p), ctypes.byref(b)))
    return p.value, b.value


def scan_query(ix: Index, mu: int, eps: float, memberships=None):
    """(mu, eps) query on the index's stream; returns int32[n] on the GPU."""
    torch = _torch()
    lib = _ready()
    if memberships is None:
        memberships = torch.empty(ix.n, dtype=torch.int32, device="cuda")
    _check(lib.scan_query(ix._h, int(mu), float(eps), ctypes.c_void_p(memberships.data_ptr() if ix.n else 0)))
    return memberships


def scan_query_ex(ix: Index, mu: int, eps: float, memberships=None, is_core=None, stream=None,
                  out_on_device: bool = True):
    """(mu, eps) query on `stream`; returns (memberships, is_core)."""
    torch = _torch()
    lib = _ready()
    s = _stream_handle(stream)
    if out_on_device:
        if memberships is None:
            memberships = torch.empty(ix.n, dtype=torch.int32, device="cuda")
        if is_core is None:
            is_core = torch.empty(ix.n, dtype=torch.uint8, device="cuda")
        mp, cp = memberships.data_ptr(), is_core.data_ptr()
    else:
        if memberships is None:
            memberships = np.empty(ix.n, np.int32)
        if is_core is None:
            is_core = np.empty(ix.n, np.uint8)
        mp, cp = memberships.ctypes.data, is_core.ctypes.data
    _check(lib.scan_query_ex(ix._h, int(mu), float(eps), ctypes.c_void_p(mp if ix.n else 0),
                             ctypes.c_void_p(cp if ix.n else 0), int(out_on_device), ctypes.c_void_p(s)))
    return memberships, is_core


def scan_query_noalloc(ix: Index, mu: int, eps: float, memberships, is_core=None, stream=None):
    """(mu, eps) query into device tensors (int32[n] memberships, optional
    uint8[n] is_core) with the library's fixed scratch workspace: no device
    allocation in the call. Asynchronous on `stream`."""
    torch = _torch()
    lib = _ready()
    n = ix.n
    if not (isinstance(memberships, torch.Tensor) and memberships.is_cuda and memberships.dtype == torch.int32
            and memberships.numel() == n and memberships.is_contiguous()):
        raise ValueError("memberships must be a contiguous device int32 tensor of n entries")
    if is_core is not None and not (isinstance(is_core, torch.Tensor) and is_core.is_cuda
                                    and is_core.dtype == torch.uint8 and is_core.numel() == n
                                    and is_core.is_contiguous()):
        raise ValueError("is_core must be a contiguous device uint8 tensor of n entries")
    cp = is_core.data_ptr() if (is_core is not None and n) else 0
    _check(lib.scan_query_noalloc(ix._h, int(mu), float(eps), ctypes.c_void_p(memberships.data_ptr() if n else 0),
                                  ctypes.c_void_p(cp), ctypes.c_void_p(_stream_handle(stream))))
    return memberships, is_core


ROLE_CLUSTERED, ROLE_HUB, ROLE_OUTLIER = 0, 1, 2


def scan_query_roles(ix: Index, memberships, roles=None, stream=None):
    """Hub / outlier roles (Section 4.3) of a query's memberships (a device
    int32 tensor of n); returns a device uint8 tensor: ROLE_CLUSTERED,
    ROLE_HUB or ROLE_OUTLIER per vertex. Asynchronous on `stream`."""
    torch = _torch()
    lib = _ready()
    if memberships.device.type != "cuda" or memberships.dtype != torch.int32 or memberships.numel() != ix.n:
        raise ValueError("memberships must be a device int32 tensor of n entries")
    if roles is None:
        roles = torch.empty(ix.n, dtype=torch.uint8, device=memberships.device)
    s = _stream_handle(stream)
    _check(lib.scan_query_roles(ix._h, ctypes.c_void_p(memberships.data_ptr() if ix.n else 0),
                                ctypes.c_void_p(roles.data_ptr() if ix.n else 0), ctypes.c_void_p(s)))
    return roles


def scan_query_modularity(ix: Index, memberships, stream=None) -> float:
    """Section 7.2 modularity of a clustering (a device int32 tensor of n
    memberships; unclustered vertices are singletons). Synchronous."""
    torch = _torch()
    lib = _ready()
    if memberships.device.type != "cuda" or memberships.dtype != torch.int32 or memberships.numel() != ix.n:
        raise ValueError("memberships must be a device int32 tensor of n entries")
    q = ctypes.c_double()
    _check(lib.scan_query_modularity(ix._h, ctypes.c_void_p(memberships.data_ptr() if ix.n else 0),
                                     ctypes.byref(q), ctypes.c_void_p(_stream_handle(stream))))
    return q.value


def paper_sweep_grid(dmax: int | None = None):
    """The parameter set of Section 7.3.4: mu in {2, 4, ..., 2^18} x eps in
    {.01, ..., .99} (eps built as k / 100.0); mu above dmax + 1 is dropped
    when dmax is given (no cores there)."""
    mus = [1 << k for k in range(1, 19)]
    if dmax is not None:
        mus = [m for m in mus if m <= dmax + 1]
    return [(m, k / 100.0) for m in mus for k in range(1, 100)]


def scan_sweep_modularity(ix: Index, mus, epss, batch: int = 32, stream=None) -> np.ndarray:
    """Modularity of the clustering of every (mus[i], epss[i]), run as batched
    queries (Section 7.3.4's parameter selection). Synchronous."""
    mus = np.ascontiguousarray(mus, dtype=np.int32)
    epss = np.ascontiguousarray(epss, dtype=np.float64)
    if mus.shape != epss.shape or mus.ndim != 1:
        raise ValueError("mus and epss must be 1-d of one length")
    q = np.zeros(len(mus), np.float64)
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data if a.size else 0)  # noqa: E731
    _check(_ready().scan_sweep_modularity(ix._h, len(mus), ptr(mus), ptr(epss), int(batch), ptr(q),
                                          ctypes.c_void_p(_stream_handle(stream))))
    return q


def scan_query_batch(ix: Index, mus, epss, out=None, stream=None, out_on_device: bool = True):
    """Batched queries; returns int32[count, n] (GPU tensor or numpy)."""
    torch = _torch()
    lib = _ready()
    mu = np.ascontiguousarray(mus, dtype=np.int32)
    eps = np.ascontiguousarray(epss, dtype=np.float64)
    if mu.shape != eps.shape:
        raise ValueError("mu and eps differ in length")
    count = len(mu)
    s = _stream_handle(stream)
    if out is None:
        out = (torch.empty((count, ix.n), dtype=torch.int32, device="cuda") if out_on_device
               else np.empty((count, ix.n), np.int32))
    ptr = out.data_ptr() if out_on_device else out.ctypes.data
    _check(lib.scan_query_batch(ix._h, count, mu.ctypes.data, eps.ctypes.data,
                                ctypes.c_void_p(ptr if ix.n and count else 0), int(out_on_device), ctypes.c_void_p(s)))
    return out


def scan_similarity_values(kind: int, c, a_u, a_v) -> np.ndarray:
    """Device similarity function on host triples (diagnostic)."""
    lib = _ready()
    c = np.ascontiguousarray(c, dtype=np.int64)
    a = np.ascontiguousarray(a_u, dtype=np.int64)
    b = np.ascontiguousarray(a_v, dtype=np.int64)
    out = np.empty(len(c), np.float64)
    _check(lib.scan_similarity_values(int(kind), len(c), c.ctypes.data, a.ctypes.data, b.ctypes.data,
                                      out.ctypes.data))
    return out


def version() -> str:
    return load_library().scan_version().decode()


# ---------------------------------------------------------------------------
# Server


class Server:
    """Continuous-batching query server over one resident index."""

    def __init__(self, ix: Index, max_slots: int = 16, max_batch: int = 16,
                 memory_budget: int = 1 << 30, use_graph: bool = True):
        lib = _ready()
        self.ix = ix
        opts = _ServerOpts(max_slots, max_batch, memory_budget, int(use_graph))
        h = ctypes.c_void_p()
        _check(lib.scan_server_create(ix._h, ctypes.byref(opts), ctypes.byref(h)))
        self._h = h

    def _dst(self, dst: np.ndarray) -> int:
        n = self.ix.info.n
        if not (isinstance(dst, np.ndarray) and dst.dtype == np.int32 and dst.shape == (n,)
                and dst.flags.c_contiguous and dst.flags.writeable):
            raise ValueError(f"dst must be a writeable contiguous int32 array of shape ({n},)")
        return dst.ctypes.data

    def submit(self, mu: int, eps: float, dst: np.ndarray) -> int:
        """Queues (mu, eps); dst (int32[n], kept alive by the caller) receives the
        memberships. Raises ScanError(SCAN_EBUSY) when the queue is full."""
        t = ctypes.c_uint64()
        _check(load_library().scan_server_submit(self._h, int(mu), float(eps), self._dst(dst), ctypes.byref(t)))
        return t.value

    def submit_ex(self, mu: int, eps: float, dst, latency_ms: int = 0, block: bool = True):
        """Queues (mu, eps) with dst either a host int32[n] array or a device
        int32 tensor of n elements (written in place by the kernels).
        latency_ms is the address of a host float64 (0: none) that receives the
        request's latency. With block=False returns None when the queue is full."""
        if not isinstance(dst, np.ndarray):
            torch = _torch()
            if not (isinstance(dst, torch.Tensor) and dst.is_cuda and dst.dtype == torch.int32
                    and dst.numel() == self.ix.info.n and dst.is_contiguous()):
                raise ValueError("device dst must be a contiguous int32 CUDA tensor of n elements")
            ptr, on_dev = dst.data_ptr(), 1
        else:
            ptr, on_dev = self._dst(dst), 0
        t = ctypes.c_uint64()
        st = load_library().scan_server_submit_ex(self._h, int(mu), float(eps), ptr, on_dev, latency_ms or None,
                                                  ctypes.byref(t))
        if st == SCAN_EBUSY and not block:
            return None
        _check(st)
        return t.value

    def try_submit(self, mu: int, eps: float, dst: np.ndarray):
        """Like submit, but returns None when the queue is full."""
        t = ctypes.c_uint64()
        st = load_library().scan_server_submit(self._h, int(mu), float(eps), self._dst(dst), ctypes.byref(t))
        if st == SCAN_EBUSY:
            return None
        _check(st)
        return t.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int32()
        _check(load_library().scan_server_poll(self._h, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int):
        _check(load_library().scan_server_wait(self._h, ticket))

    def close(self):
        if self._h is not None and self._h.value:
            load_library().scan_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
