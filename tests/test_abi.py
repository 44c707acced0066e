"""The C-ABI library loads and exports every symbol include/ce.h declares (no GPU calls)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "ce.h")).read()
    return sorted(set(re.findall(r"\b(ce_[a-z_]+)\s*\(", text)))


def test_library_exports_declared_symbols():
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.skip("libce.so not built")
    lib = ce.load_library()
    syms = declared_symbols()
    assert set(syms) == {"ce_cluster_edges", "ce_cluster_batch", "ce_workspace_bytes", "ce_batch_workspace_bytes",
                         "ce_max_clusters", "ce_last_error", "ce_timing_enable", "ce_timing_read",
                         "ce_server_create", "ce_server_destroy", "ce_server_request_bytes", "ce_server_submit",
                         "ce_server_poll", "ce_server_get_stats", "ce_cluster_hyperedges",
                         "ce_hyper_workspace_bytes", "ce_level_components", "ce_cluster_edges_async",
                         "ce_cluster_batch_async", "ce_batch_workspace_bytes_for", "ce_result_status",
                         "ce_cluster_edges_noalloc", "ce_resolve_tuning"}
    for s in syms:
        assert hasattr(lib, s), s


def test_host_only_functions():
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.skip("libce.so not built")
    assert ce.max_clusters(10, 5) == 5 and ce.max_clusters(0, 5) == 1 and ce.max_clusters(9, 1) == 0
    b1 = ce.workspace_bytes(1000, 100, 5)
    b2 = ce.workspace_bytes(2000, 100, 5)
    assert 0 < b1 < b2
    assert ce.workspace_bytes(-1, 100, 5) == 0
    assert ce.workspace_bytes(10, 0, 5) == 0
    assert ce.workspace_bytes(10, 10, 1) == 0
    # about 100 bytes of workspace per record at scale
    assert ce.workspace_bytes(10 ** 7, 10 ** 6, 10) / 10 ** 7 < 170  # bytes of workspace per record


def test_host_argument_errors_need_no_gpu():
    """Argument checks happen on the host before any device call."""
    import ctypes
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.skip("libce.so not built")
    lib = ce.load_library()
    res, cnt = ce.CeResult(), ce.CeCounts()
    p = ce.make_params(1, 10)
    assert lib.ce_cluster_edges(None, None, None, 0, ctypes.byref(p), ctypes.byref(res), ctypes.byref(cnt), None, 0,
                                None) == ce.CE_EINVAL
    assert "min_cluster_size" in ce.last_error()
    p = ce.make_params(5, 10)
    assert lib.ce_cluster_edges(None, None, None, -1, ctypes.byref(p), ctypes.byref(res), ctypes.byref(cnt), None, 0,
                                None) == ce.CE_EINVAL
    assert lib.ce_cluster_edges(None, None, None, 5, ctypes.byref(p), ctypes.byref(res), ctypes.byref(cnt), None, 0,
                                None) == ce.CE_EINVAL
    p.mode = 7
    assert lib.ce_cluster_edges(None, None, None, 0, ctypes.byref(p), ctypes.byref(res), ctypes.byref(cnt), None, 0,
                                None) == ce.CE_EINVAL


def test_hypergraph_host_functions_and_errors():
    import ctypes
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.skip("libce.so not built")
    lib = ce.load_library()
    a = ce.hyper_workspace_bytes(1000, 3000, 100, 5)
    assert 0 < a < ce.hyper_workspace_bytes(1000, 30000, 100, 5)
    assert ce.hyper_workspace_bytes(1000, 3000, 100, 5, thresholds=[1, 2]) > a
    assert ce.hyper_workspace_bytes(-1, 3, 100, 5) == 0 and ce.hyper_workspace_bytes(10, -1, 100, 5) == 0
    p = ce.make_params(5, 100, causal=True)
    assert lib.ce_hyper_workspace_bytes(10, 30, ctypes.byref(p)) == 0
    res, cnt = ce.CeResult(), ce.CeCounts()
    assert lib.ce_cluster_hyperedges(None, None, None, 0, 0, ctypes.byref(p), ctypes.byref(res), ctypes.byref(cnt),
                                     None, 0, None) == ce.CE_EINVAL
    assert "undirected" in ce.last_error()
    p = ce.make_params(5, 100)
    assert lib.ce_cluster_hyperedges(None, None, None, 4, 9, ctypes.byref(p), ctypes.byref(res), ctypes.byref(cnt),
                                     None, 0, None) == ce.CE_EINVAL
    assert "input pointer" in ce.last_error()
    assert lib.ce_cluster_hyperedges(None, None, None, 4, -1, ctypes.byref(p), ctypes.byref(res), ctypes.byref(cnt),
                                     None, 0, None) == ce.CE_EINVAL


def test_batch_host_functions():
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.skip("libce.so not built")
    # one graph as a batch needs the same workspace as the single call
    assert ce.batch_workspace_bytes([0, 5000], [0, 300], 5) == ce.workspace_bytes(5000, 300, 5)
    many = ce.batch_workspace_bytes([0, 2000, 2000, 5000], [0, 100, 101, 300], 5)
    assert many >= ce.workspace_bytes(5000, 300, 5)
    assert ce.batch_workspace_bytes([0, 10, 5], [0, 3, 6], 5) == 0      # decreasing edge offsets
    assert ce.batch_workspace_bytes([0, 10, 20], [0, 3, 3], 5) == 0     # a graph without vertices
    assert ce.batch_workspace_bytes([1, 10], [0, 3], 5) == 0            # offsets must start at 0
    assert ce.batch_cluster_capacity([0, 10, 10, 33], 5) == 5 + 1 + 9


def test_batch_argument_errors_need_no_gpu():
    import ctypes
    import numpy as np
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.skip("libce.so not built")
    lib = ce.load_library()
    i64p = ctypes.POINTER(ctypes.c_int64)
    res = ce.CeResult()
    p = ce.make_params(5, 10)

    def call(eo, vo, G, counts=True, offsets=True):
        eo = np.asarray(eo, dtype=np.int64)
        vo = np.asarray(vo, dtype=np.int64)
        cnt = (ce.CeCounts * max(G, 1))()
        ro = np.zeros(max(G, 0) + 1, dtype=np.int64)
        co = np.zeros(max(G, 0) + 1, dtype=np.int64)
        return lib.ce_cluster_batch(None, None, None, eo.ctypes.data_as(i64p), vo.ctypes.data_as(i64p), G,
                                    ctypes.byref(p), ctypes.byref(res), cnt if counts else None,
                                    ro.ctypes.data_as(i64p) if offsets else None, co.ctypes.data_as(i64p), None, 0,
                                    None)

    assert call([0, 0], [0, 1], 0) == ce.CE_EINVAL
    assert "number of graphs" in ce.last_error()
    assert call([0, 4, 2], [0, 1, 2], 2) == ce.CE_EINVAL
    assert "non-decreasing" in ce.last_error()
    assert call([0, 4, 6], [0, 1, 1], 2) == ce.CE_EINVAL
    assert "vertex" in ce.last_error()
    assert call([0, 4], [0, 3], 1, counts=False) == ce.CE_EINVAL
    assert call([0, 4], [0, 3], 1, offsets=False) == ce.CE_EINVAL
    assert call([0, 4], [0, 3], 1) == ce.CE_EINVAL  # null record pointers with 4 records
    assert "input pointer" in ce.last_error()
    assert call([0, 1 << 31], [0, 3], 1) == ce.CE_EINVAL


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors have the sizes and field offsets a C compiler gives the header's structs."""
    import ctypes
    import shutil
    import subprocess
    import paper_2311_10337_amd as ce
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"ce_params": ce.CeParams, "ce_tuning": ce.CeTuning, "ce_result": ce.CeResult, "ce_counts": ce.CeCounts,
               "ce_server_config": ce.CeServerConfig, "ce_request": ce.CeRequest,
               "ce_request_status": ce.CeRequestStatus, "ce_server_stats": ce.CeServerStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ce.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line.strip():
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_server_host_checks_need_no_gpu():
    import ctypes
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.skip("libce.so not built")
    lib = ce.load_library()
    h = ctypes.c_void_p()
    for kw in ({"workers": 0}, {"workers": 17}, {"hbm_budget_bytes": 1000}, {"max_inflight": 0},
               {"input_fraction_pct": 0}, {"input_fraction_pct": 95}):
        cfg = dict(struct_size=ctypes.sizeof(ce.CeServerConfig), device=0, workers=2, input_fraction_pct=25,
                   hbm_budget_bytes=1 << 30, max_inflight=8, max_batch_records=0)
        cfg.update(kw)
        assert lib.ce_server_create(ctypes.byref(ce.CeServerConfig(**cfg)), ctypes.byref(h)) == ce.CE_EINVAL, kw
    # the admission footprint grows with n and is 0 for bad arguments
    a = ce.server_request_bytes(10_000, 1000, 10)
    b = ce.server_request_bytes(100_000, 1000, 10)
    assert 0 < a < b
    assert ce.server_request_bytes(-1, 1000, 10) == 0 and ce.server_request_bytes(10, 1000, 1) == 0


def test_earlier_params_layout_is_accepted():
    """A caller built against the 32-byte parameter struct (no max_dt) is read as "no cutoff"."""
    import ctypes
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.skip("libce.so not built")
    lib = ce.load_library()

    class ParamsV1(ctypes.Structure):
        _fields_ = ce.CeParams._fields_[:6]

    assert ctypes.sizeof(ParamsV1) == 32
    v1 = ParamsV1(32, 0, 5, 100, 0, 0)
    a = lib.ce_workspace_bytes(1000, 100, ctypes.cast(ctypes.pointer(v1), ctypes.POINTER(ce.CeParams)))
    assert a == ce.workspace_bytes(1000, 100, 5) > 0
    v1.struct_size = 24
    assert lib.ce_workspace_bytes(1000, 100, ctypes.cast(ctypes.pointer(v1), ctypes.POINTER(ce.CeParams))) == 0


def test_level_components_argument_errors_need_no_gpu():
    """ce_level_components checks its arguments and thresholds on the host; q = 0 or n = 0 does nothing."""
    import ctypes
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.skip("libce.so not built")
    lib = ce.load_library()
    arr = lambda *v: (ctypes.c_int64 * max(len(v), 1))(*v)
    call = lambda m, n, thr, q: lib.ce_level_components(None, None, None, m, n, thr, q, None, None)
    assert call(0, 5, arr(), 0) == ce.CE_OK
    assert call(0, 0, arr(3), 1) == ce.CE_OK
    assert call(0, -1, arr(3), 1) == ce.CE_EINVAL
    assert call(-1, 5, arr(3), 1) == ce.CE_EINVAL
    assert call(0, 5, None, 1) == ce.CE_EINVAL
    assert call(0, 5, arr(*range(65)), 65) == ce.CE_EINVAL
    for bad in ((3, 3), (4, 2), (-1, 2)):
        assert call(0, 5, arr(*bad), 2) == ce.CE_EINVAL
        assert "increasing" in ce.last_error()
    assert call(0, 5, arr(3), 1) == ce.CE_EINVAL  # labels NULL
