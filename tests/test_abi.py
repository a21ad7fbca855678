"""C ABI: the library loads, exports every symbol include/scan.h declares, and
rejects bad arguments before any device work (no GPU needed)."""

import ctypes
import os
import re
import subprocess

import pytest

import paper_2012_11188_amd as scan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "scan.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scan_[a-z_]+)\s*\(", text)))


def test_header_parses_and_binding_lists_it():
    names = header_functions()
    assert "scan_build_index" in names and "scan_query" in names and "scan_query_batch" in names
    assert sorted(scan.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = scan.load_library()
    for name in header_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", scan.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (scan_\w+)", out))
    assert set(header_functions()) <= exported


def test_header_compiles_as_c():
    src = '#include "scan.h"\nint main(void){scan_csr g; (void)g; return 0;}\n'
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        "-x", "c", "-", "-o", "/dev/null"], input=src, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_version_and_error_string():
    lib = scan.load_library()
    assert b"gfx950" in lib.scan_version()
    assert isinstance(lib.scan_last_error(), bytes)


def _csr(n, nnz, bits=32, offsets=1, adj=1):
    return scan._Csr(n, nnz, bits, 1, ctypes.c_void_p(offsets), ctypes.c_void_p(adj))


@pytest.mark.parametrize("csr,kind,flags,needle", [
    (None, 0, 0, b"null graph"),
    (_csr(-1, 0), 0, 0, b"negative"),
    (_csr(4, 3), 0, 0, b"odd nnz"),
    (_csr(4, 4, bits=16), 0, 0, b"offset_bits"),
    (_csr(4, 4, offsets=0), 0, 0, b"null offsets"),
    (_csr(4, 4, adj=0), 0, 0, b"null adj"),
    (_csr(1 << 31, 4, bits=64), 0, 0, b"int32 vertex ids"),
    (_csr(4, 4), 7, 0, b"unknown similarity kind"),
    (_csr(4, 4), 0, 1 << 9, b"unknown build flags"),
])
def test_build_rejects_bad_arguments(csr, kind, flags, needle):
    lib = scan.load_library()
    out = ctypes.c_void_p(1)
    st = lib.scan_build_index(ctypes.byref(csr) if csr is not None else None, kind, flags, None, ctypes.byref(out))
    assert st == scan.SCAN_EINVAL
    assert out.value is None
    assert needle in lib.scan_last_error()


def test_query_and_misc_reject_bad_arguments():
    lib = scan.load_library()
    assert lib.scan_query(None, 2, 0.5, None) == scan.SCAN_EINVAL
    assert lib.scan_query_ex(None, 2, 0.5, None, None, 1, None) == scan.SCAN_EINVAL
    assert lib.scan_query_batch(None, 1, None, None, None, 1, None) == scan.SCAN_EINVAL
    assert lib.scan_index_get_info(None, None) == scan.SCAN_EINVAL
    assert lib.scan_index_export(None, 0, None, 0) == scan.SCAN_EINVAL
    assert lib.scan_server_create(None, None, None) == scan.SCAN_EINVAL
    assert lib.scan_set_allocator(scan._ALLOC_FN(lambda *a: None), scan._RELEASE_FN(), None) == scan.SCAN_EINVAL
    assert lib.scan_similarity_values(5, 1, None, None, None, None) == scan.SCAN_EINVAL
    assert lib.scan_similarity_values(0, -1, None, None, None, None) == scan.SCAN_EINVAL
    lib.scan_index_free(None)
    lib.scan_server_destroy(None)


def test_product_path_has_no_cpu_fallback():
    src = open(scan.__file__).read()
    assert "oracle" not in src.replace("no CPU fallback", "")
    for f in os.listdir(os.path.join(ROOT, "paper_2012_11188_amd", "csrc")):
        assert "oracle" not in open(os.path.join(ROOT, "paper_2012_11188_amd", "csrc", f)).read()


def _tiny_host_graph():
    import numpy as np

    # path 0 - 1 - 2 on the host
    return np.array([0, 1, 3, 4], np.int32), np.array([1, 0, 2, 1], np.int32)


@pytest.mark.parametrize("kind,kw,needle", [
    (scan.COSINE, {"gauss": [0.0] * 5}, "n * samples"),                 # 3 x 64 expected
    (scan.COSINE, {}, "n * samples"),                                   # no draws
    (scan.COSINE, {"gauss": [0.0] * 192, "perm": [0, 1, 2]}, "JACCARD only"),
    (scan.JACCARD, {"perm": [0, 1]}, "n = 3"),                          # short permutation
    (scan.JACCARD, {"perm": [0, 1, 2], "gauss": [0.0] * 192}, "cosine kinds only"),
    (scan.WEIGHTED_COSINE, {"gauss": [0.0] * 192, "weights": [1.0] * 3}, "nnz = 4"),
    (scan.WEIGHTED_COSINE, {"gauss": [0.0] * 192}, "nnz = 4"),           # no weights
    (scan.COSINE, {"gauss": [0.0] * 192, "weights": [1.0] * 4}, "WEIGHTED_COSINE only"),
    (9, {"gauss": [0.0] * 192}, "unknown similarity kind"),
])
def test_lsh_binding_rejects_wrong_sizes_before_device_work(kind, kw, needle):
    # raised by the binding before the library or the GPU is touched: an
    # undersized draw array would otherwise be read out of bounds
    off, adj = _tiny_host_graph()
    with pytest.raises(ValueError, match=re.escape(needle)):
        scan.scan_build_index_lsh(off, adj, kind, 64, **kw)


def test_weighted_binding_rejects_wrong_sizes_before_device_work():
    off, adj = _tiny_host_graph()
    with pytest.raises(ValueError, match="nnz = 4"):
        scan.scan_build_index_weighted(off, adj, [1.0, 1.0, 1.0])
    with pytest.raises(ValueError, match="nnz = 4"):
        scan.scan_build_index_weighted(off, adj, None)
