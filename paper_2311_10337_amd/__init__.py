"""MI355X-native hierarchical edge clustering of dynamic graphs (arXiv 2311.10337).

Thin Python binding over the C ABI of ``libce.so`` (see ``include/ce.h``): it
allocates output tensors with PyTorch on the GPU, passes raw device pointers
and the current HIP stream, and returns the trimmed tensors. Every step of the
computation runs in the library's HIP kernels; there is no CPU fallback, and a
missing library raises.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import threading
from typing import NamedTuple, Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libce.so")

CE_OK, CE_EINVAL, CE_ESELFLOOP, CE_ERANGE, CE_ENOMEM, CE_EDEVICE, CE_EBUSY = 0, -1, -2, -3, -4, -5, -6
CE_MODE_UNDIRECTED, CE_MODE_CAUSAL = 0, 1
NONE32 = 0xFFFFFFFF


class CeTuning(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("radix_keys_per_thread", ctypes.c_int32),
                ("list_grid", ctypes.c_int32), ("krt_level_bits", ctypes.c_int32), ("split_min_edges", ctypes.c_int64)]


TUNING_KNOBS = ("radix_keys_per_thread", "list_grid", "krt_level_bits", "split_min_edges")


class CeParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("mode", ctypes.c_uint32), ("min_cluster_size", ctypes.c_int64),
                ("num_vertices", ctypes.c_int64), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("max_dt", ctypes.c_int64), ("thresholds", ctypes.c_void_p), ("num_thresholds", ctypes.c_int64),
                ("time_bits", ctypes.c_int64), ("tuning", ctypes.c_void_p)]


_tuning_state = threading.local()


def set_tuning(knobs=None):
    """Launch choices (a dict over TUNING_KNOBS; missing or 0 = the library's next source) for the calls this
    thread makes from now on; None clears them. Outputs never depend on them."""
    if knobs:
        bad = set(knobs) - set(TUNING_KNOBS)
        if bad:
            raise ValueError("unknown tuning knobs: %s" % sorted(bad))
    _tuning_state.knobs = dict(knobs) if knobs else None


def current_tuning():
    return getattr(_tuning_state, "knobs", None)


@contextlib.contextmanager
def tuned(knobs):
    """``with tuned({...}):`` -- set_tuning for the block, then the previous choices again."""
    prev = current_tuning()
    set_tuning(knobs)
    try:
        yield
    finally:
        set_tuning(prev)


_RESULT_FIELDS = ["msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster",
                  "pt_lambda", "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo",
                  "cl_selected", "labels", "dd_level", "dd_top"]


class CeResult(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in _RESULT_FIELDS]


class CeCounts(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n_clusters", ctypes.c_int64), ("n_labels", ctypes.c_int64)]


class CeServerConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("device", ctypes.c_int32), ("workers", ctypes.c_uint32),
                ("input_fraction_pct", ctypes.c_uint32), ("hbm_budget_bytes", ctypes.c_uint64),
                ("max_inflight", ctypes.c_int64), ("max_batch_records", ctypes.c_int64)]


class CeRequest(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("src", ctypes.c_void_p),
                ("dst", ctypes.c_void_p), ("t", ctypes.c_void_p), ("n", ctypes.c_int64), ("params", CeParams),
                ("out", CeResult)]


class CeRequestStatus(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("reserved", ctypes.c_uint32), ("counts", CeCounts),
                ("queue_s", ctypes.c_double), ("latency_s", ctypes.c_double)]


_STAT_FIELDS = ["requests_submitted", "requests_done", "requests_batched", "batches", "max_batch_requests",
                "max_concurrent_batches", "input_peak_bytes", "work_peak_bytes", "input_capacity_bytes",
                "work_capacity_bytes"]


class CeServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in _STAT_FIELDS]


_EXPORTS = ["ce_cluster_edges", "ce_cluster_batch", "ce_workspace_bytes", "ce_batch_workspace_bytes",
            "ce_max_clusters", "ce_last_error", "ce_timing_enable", "ce_timing_read", "ce_server_create",
            "ce_server_destroy", "ce_server_request_bytes", "ce_server_submit", "ce_server_poll",
            "ce_server_get_stats", "ce_cluster_edges_async", "ce_cluster_batch_async", "ce_batch_workspace_bytes_for",
            "ce_result_status", "ce_cluster_edges_noalloc", "ce_resolve_tuning"]
CE_MAX_GRAPHS = 1 << 24
_lib = None


def load_library(path: str = LIB_PATH):
    """Load libce.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("libce.so is not built (%s); run __graft_entry__.build()" % path)
        lib = ctypes.CDLL(path)
        lib.ce_cluster_edges.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.POINTER(CeParams),
                                                                 ctypes.POINTER(CeResult), ctypes.POINTER(CeCounts),
                                                                 ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        lib.ce_cluster_edges.restype = ctypes.c_int
        lib.ce_cluster_hyperedges.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_int64,
                                                                      ctypes.POINTER(CeParams), ctypes.POINTER(CeResult),
                                                                      ctypes.POINTER(CeCounts), ctypes.c_void_p,
                                                                      ctypes.c_size_t, ctypes.c_void_p]
        lib.ce_cluster_hyperedges.restype = ctypes.c_int
        lib.ce_hyper_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(CeParams)]
        lib.ce_hyper_workspace_bytes.restype = ctypes.c_size_t
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.ce_cluster_batch.argtypes = [ctypes.c_void_p] * 3 + [i64p, i64p, ctypes.c_int64, ctypes.POINTER(CeParams),
                                                                 ctypes.POINTER(CeResult), ctypes.POINTER(CeCounts),
                                                                 i64p, i64p, ctypes.c_void_p, ctypes.c_size_t,
                                                                 ctypes.c_void_p]
        lib.ce_cluster_batch.restype = ctypes.c_int
        lib.ce_batch_workspace_bytes.argtypes = [i64p, i64p, ctypes.c_int64, ctypes.POINTER(CeParams)]
        lib.ce_batch_workspace_bytes.restype = ctypes.c_size_t
        lib.ce_batch_workspace_bytes_for.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(CeParams)]
        lib.ce_batch_workspace_bytes_for.restype = ctypes.c_size_t
        lib.ce_cluster_edges_async.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.POINTER(CeParams),
                                                                       ctypes.POINTER(CeResult), ctypes.c_void_p,
                                                                       ctypes.c_void_p, ctypes.c_size_t,
                                                                       ctypes.c_void_p]
        lib.ce_cluster_edges_async.restype = ctypes.c_int
        lib.ce_cluster_batch_async.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                                                       ctypes.c_int64, ctypes.c_int64,
                                                                       ctypes.POINTER(CeParams),
                                                                       ctypes.POINTER(CeResult), ctypes.c_void_p,
                                                                       ctypes.c_void_p, ctypes.c_size_t,
                                                                       ctypes.c_void_p]
        lib.ce_cluster_batch_async.restype = ctypes.c_int
        lib.ce_result_status.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(CeCounts), i64p, i64p,
                                         ctypes.c_void_p]
        lib.ce_result_status.restype = ctypes.c_int
        lib.ce_cluster_edges_noalloc.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.POINTER(CeParams),
                                                                         ctypes.POINTER(CeResult), ctypes.c_void_p,
                                                                         ctypes.c_void_p]
        lib.ce_cluster_edges_noalloc.restype = ctypes.c_int
        vp = ctypes.c_void_p
        lib.ce_server_create.argtypes = [ctypes.POINTER(CeServerConfig), ctypes.POINTER(vp)]
        lib.ce_server_create.restype = ctypes.c_int
        lib.ce_server_destroy.argtypes = [vp]
        lib.ce_server_destroy.restype = ctypes.c_int
        lib.ce_server_request_bytes.argtypes = [ctypes.c_int64, ctypes.POINTER(CeParams)]
        lib.ce_server_request_bytes.restype = ctypes.c_size_t
        lib.ce_server_submit.argtypes = [vp, ctypes.POINTER(CeRequest), ctypes.POINTER(ctypes.c_uint64)]
        lib.ce_server_submit.restype = ctypes.c_int
        lib.ce_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(CeRequestStatus)]
        lib.ce_server_poll.restype = ctypes.c_int
        lib.ce_server_get_stats.argtypes = [vp, ctypes.POINTER(CeServerStats)]
        lib.ce_server_get_stats.restype = ctypes.c_int
        lib.ce_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(CeParams)]
        lib.ce_workspace_bytes.restype = ctypes.c_size_t
        lib.ce_max_clusters.argtypes = [ctypes.c_int64, ctypes.c_int64]
        lib.ce_max_clusters.restype = ctypes.c_int64
        lib.ce_level_components.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_int64, i64p,
                                                                    ctypes.c_int64, ctypes.c_void_p,
                                                                    ctypes.c_void_p]
        lib.ce_level_components.restype = ctypes.c_int
        lib.ce_last_error.argtypes = []
        lib.ce_last_error.restype = ctypes.c_char_p
        lib.ce_timing_enable.argtypes = [ctypes.c_char_p]
        lib.ce_timing_enable.restype = ctypes.c_int
        lib.ce_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        lib.ce_timing_read.restype = ctypes.c_int
        lib.ce_resolve_tuning.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(CeParams),
                                          ctypes.POINTER(CeTuning)]
        lib.ce_resolve_tuning.restype = ctypes.c_int
        _lib = lib
    return _lib


def exported_symbols():
    lib = load_library()
    return {name: hasattr(lib, name) for name in _EXPORTS}


def make_params(min_cluster_size: int, num_vertices: int, causal: bool = False, max_dt: int = -1,
                thresholds=None, time_bits: int = 0) -> CeParams:
    """Parameters; `thresholds` (increasing weights) selects the discrete dendrogram; `time_bits` bounds the
    time span for asynchronous calls. The returned struct keeps a reference to the thresholds' host array."""
    import numpy as np
    mode = CE_MODE_CAUSAL if causal else CE_MODE_UNDIRECTED
    p = CeParams(ctypes.sizeof(CeParams), mode, int(min_cluster_size), int(num_vertices), 0, 0, int(max_dt), None, 0,
                 int(time_bits), None)
    knobs = current_tuning()
    if knobs:
        tu = CeTuning(ctypes.sizeof(CeTuning), *[int(knobs.get(k, 0)) for k in TUNING_KNOBS])
        p.tuning = ctypes.addressof(tu)
        p._keep_tuning = tu
    if thresholds is not None and len(thresholds) > 0:
        thr = np.ascontiguousarray(np.asarray(thresholds, dtype=np.int64))
        p.thresholds = thr.ctypes.data
        p.num_thresholds = thr.size
        p._keep = thr
    return p


def resolve_tuning(n: int, num_vertices: int, knobs=None) -> dict:
    """The launch choices the library takes for a call of n records over num_vertices vertices
    (``ce_resolve_tuning``): the given knobs, else the environment, the CE_TUNE_FILE entry, the rules."""
    lib = load_library()
    with tuned(knobs) if knobs is not None else contextlib.nullcontext():
        p = make_params(2, max(int(num_vertices), 1))
    out = CeTuning(ctypes.sizeof(CeTuning), 0, 0, 0, 0)
    st = lib.ce_resolve_tuning(int(n), int(num_vertices), ctypes.byref(p), ctypes.byref(out))
    if st != CE_OK:
        raise ClusterError(st, lib.ce_last_error().decode())
    return {k: int(getattr(out, k)) for k in TUNING_KNOBS}


def hdr_words(num_graphs: int = 1) -> int:
    """int64 words of an asynchronous call's device header (CE_HDR_WORDS)."""
    return 6 + 5 * int(num_graphs)


def workspace_bytes(n: int, num_vertices: int, min_cluster_size: int, thresholds=None) -> int:
    """Workspace for one graph; condensing on the discrete dendrogram (``thresholds``) needs more."""
    p = make_params(min_cluster_size, num_vertices, thresholds=thresholds)
    return int(load_library().ce_workspace_bytes(int(n), int(num_vertices), ctypes.byref(p)))


def max_clusters(n: int, min_cluster_size: int) -> int:
    return int(load_library().ce_max_clusters(int(n), int(min_cluster_size)))


def last_error() -> str:
    return load_library().ce_last_error().decode()


def timing_enable(kernel_name):
    """Time every launch of library kernels whose name contains kernel_name (None: off)."""
    load_library().ce_timing_enable(kernel_name.encode() if kernel_name else None)


def timing_read():
    """(total milliseconds, launches) accumulated since timing_enable."""
    ms, cnt = ctypes.c_double(), ctypes.c_int64()
    load_library().ce_timing_read(ctypes.byref(ms), ctypes.byref(cnt))
    return float(ms.value), int(cnt.value)


class ClusterError(RuntimeError):
    def __init__(self, status, msg, call="ce_cluster_edges"):
        super().__init__("%s failed (%d): %s" % (call, status, msg))
        self.status = status


class Result(NamedTuple):
    """Device tensors. u32/u64 fields are stored in int32/int64 tensors bit for bit. dd_level and dd_top are
    None unless the discrete dendrogram was asked for."""
    m: int
    n_clusters: int
    n_labels: int
    msf_tail: object
    msf_head: object
    msf_w: object
    sl_left: object
    sl_right: object
    sl_w: object
    sl_size: object
    pt_cluster: object
    pt_lambda: object
    cl_id: object
    cl_parent: object
    cl_size: object
    cl_lambda_birth: object
    cl_stab_hi: object
    cl_stab_lo: object
    cl_selected: object
    labels: object
    dd_level: object = None
    dd_top: object = None


class Outputs:
    """Preallocated device output buffers for n records (reusable across calls).

    ``clusters`` overrides the cluster-row capacity (a batch needs the sum of
    its graphs' ``max_clusters``); ``rows`` overrides the MSF-row capacity.
    """

    def __init__(self, n: int, min_cluster_size: int, device, clusters: Optional[int] = None,
                 rows: Optional[int] = None):
        import torch
        R = rows if rows is not None else max(n - 1, 1)
        C = clusters if clusters is not None else max_clusters(n, min_cluster_size)
        i32, i64, u8 = torch.int32, torch.int64, torch.uint8
        e = lambda k, dt: torch.empty(max(k, 1), dtype=dt, device=device)
        self.n, self.C, self.R = n, C, R
        self.t = {"msf_tail": e(R, i32), "msf_head": e(R, i32), "msf_w": e(R, i64), "sl_left": e(R, i32),
                  "sl_right": e(R, i32), "sl_w": e(R, i64), "sl_size": e(R, i32), "pt_cluster": e(n, i32),
                  "pt_lambda": e(n, i64), "cl_id": e(C, i32), "cl_parent": e(C, i32), "cl_size": e(C, i32),
                  "cl_lambda_birth": e(C, i64), "cl_stab_hi": e(C, i64), "cl_stab_lo": e(C, i64),
                  "cl_selected": e(C, u8), "labels": e(n, i32), "dd_level": e(R, i32), "dd_top": e(R, i32)}
        self.struct = CeResult(**{f: ctypes.c_void_p(self.t[f].data_ptr()) for f in _RESULT_FIELDS})

    def region(self, row0: int, rec0: int, cl0: int, n: int, min_cluster_size: int) -> "Outputs":
        """Outputs for n records whose buffers start inside this one's: rows at row0, per-record outputs at
        rec0, cluster rows at cl0 (the layout of graph g of a batch when given its row, edge and cluster
        offsets). The caller keeps the regions of different calls apart; the capacities are those of a call
        on n records, which writes only its own counts."""
        o = Outputs.__new__(Outputs)
        o.n, o.R, o.C = n, max(n - 1, 1), max_clusters(n, min_cluster_size)
        start = {f: (rec0 if f in _RECORD_FIELDS else cl0 if f in _CLUSTER_FIELDS else row0) for f in self.t}
        size = {f: (o.n if f in _RECORD_FIELDS else o.C if f in _CLUSTER_FIELDS else o.R) for f in self.t}
        for f, x in self.t.items():
            if start[f] + size[f] > x.numel():
                raise ValueError("region of %s [%d, %d) passes the buffer's %d entries"
                                 % (f, start[f], start[f] + size[f], x.numel()))
        o.t = {f: x[start[f]:start[f] + size[f]] for f, x in self.t.items()}
        o.struct = CeResult(**{f: ctypes.c_void_p(o.t[f].data_ptr()) for f in _RESULT_FIELDS})
        return o


_RECORD_FIELDS = ("pt_cluster", "pt_lambda", "labels")
_CLUSTER_FIELDS = ("cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected")


def cluster_edges(src, dst, t, min_cluster_size: int, num_vertices: int, outputs: Optional[Outputs] = None,
                  workspace=None, stream=None, causal: bool = False, max_dt: int = -1, thresholds=None) -> Result:
    """Cluster temporal edges (src[i], dst[i], t[i]) held in GPU tensors (int32, int32, int64).

    ``causal=True`` uses the increment-weighted (tip-to-tail) line graph
    instead of the undirected one; ``max_dt >= 0`` keeps only line-graph
    edges with w <= max_dt; ``thresholds`` selects the discrete dendrogram
    (Alg. 5) and its condensing.

    Runs ``ce_cluster_edges`` on the current (or given) HIP stream and returns
    when the results are written. ``workspace`` may be a uint8 device tensor of
    at least ``workspace_bytes(...)`` bytes; otherwise the library allocates.
    """
    import torch
    lib = load_library()
    for name, x, dt in (("src", src, torch.int32), ("dst", dst, torch.int32), ("t", t, torch.int64)):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == dt and x.is_contiguous() and x.dim() == 1):
            raise TypeError("%s must be a contiguous 1-D %s GPU tensor" % (name, dt))
    n = int(src.numel())
    if dst.numel() != n or t.numel() != n:
        raise ValueError("src, dst, t must have the same length")
    if outputs is None or outputs.n < n or outputs.C < max_clusters(n, min_cluster_size):
        outputs = Outputs(n, min_cluster_size, src.device)
    params = make_params(min_cluster_size, num_vertices, causal, max_dt, thresholds)
    counts = CeCounts()
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    ws_ptr, ws_len = None, 0
    if workspace is not None:
        ws_ptr, ws_len = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    st = lib.ce_cluster_edges(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                              ctypes.c_void_p(t.data_ptr()), n, ctypes.byref(params), ctypes.byref(outputs.struct),
                              ctypes.byref(counts), ctypes.c_void_p(ws_ptr), ws_len, ctypes.c_void_p(s.cuda_stream))
    if st != CE_OK:
        raise ClusterError(st, last_error())
    return _result(outputs, n, counts, params)


def _check_dev(name, x, dt):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == dt and x.is_contiguous() and x.dim() == 1):
        raise TypeError("%s must be a contiguous 1-D %s GPU tensor" % (name, dt))


def cluster_edges_async(src, dst, t, min_cluster_size: int, num_vertices: int, outputs: Outputs, workspace, hdr,
                        time_bits: int, stream=None, max_dt: int = -1, thresholds=None) -> None:
    """Enqueue the clustering of (src, dst, t) on the stream and return at once (``ce_cluster_edges_async``).

    ``outputs``, ``workspace`` (uint8, at least ``workspace_bytes``) and ``hdr`` (int64, ``hdr_words(1)``) are
    device tensors the caller keeps alive until the stream has run; ``time_bits`` bounds the time span
    (max t - min t < 2**time_bits). Read the counts with ``result_status`` or ``async_result``."""
    import torch
    lib = load_library()
    for name, x, dt in (("src", src, torch.int32), ("dst", dst, torch.int32), ("t", t, torch.int64),
                        ("workspace", workspace, torch.uint8), ("hdr", hdr, torch.int64)):
        _check_dev(name, x, dt)
    n = int(src.numel())
    if dst.numel() != n or t.numel() != n:
        raise ValueError("src, dst, t must have the same length")
    if hdr.numel() < hdr_words(1):
        raise ValueError("hdr needs %d int64 words" % hdr_words(1))
    if outputs.n < n or outputs.C < max_clusters(n, min_cluster_size):
        raise ValueError("outputs are too small for %d records" % n)
    params = make_params(min_cluster_size, num_vertices, False, max_dt, thresholds, time_bits)
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    st = lib.ce_cluster_edges_async(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                    ctypes.c_void_p(t.data_ptr()), n, ctypes.byref(params),
                                    ctypes.byref(outputs.struct), ctypes.c_void_p(hdr.data_ptr()),
                                    ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                    ctypes.c_void_p(s.cuda_stream))
    if st != CE_OK:
        raise ClusterError(st, last_error(), "ce_cluster_edges_async")


def batch_workspace_bytes_for(n: int, num_graphs: int, min_cluster_size: int, thresholds=None) -> int:
    """Workspace of a batch of num_graphs graphs with n records in all (no offsets needed)."""
    p = make_params(min_cluster_size, 1, thresholds=thresholds)
    return int(load_library().ce_batch_workspace_bytes_for(int(n), int(num_graphs), ctypes.byref(p)))


def cluster_batch_async(src, dst, t, edge_offsets, vertex_offsets, num_vertices: int, min_cluster_size: int,
                        outputs: Outputs, workspace, hdr, time_bits: int, stream=None, max_dt: int = -1,
                        thresholds=None) -> None:
    """Enqueue a batch (``ce_cluster_batch_async``): edge_offsets and vertex_offsets are int64 GPU tensors of
    G+1 offsets, num_vertices their total; hdr holds ``hdr_words(G)`` int64 words. Returns at once."""
    import torch
    lib = load_library()
    for name, x, dt in (("src", src, torch.int32), ("dst", dst, torch.int32), ("t", t, torch.int64),
                        ("edge_offsets", edge_offsets, torch.int64), ("vertex_offsets", vertex_offsets, torch.int64),
                        ("workspace", workspace, torch.uint8), ("hdr", hdr, torch.int64)):
        _check_dev(name, x, dt)
    n, G = int(src.numel()), int(edge_offsets.numel()) - 1
    if dst.numel() != n or t.numel() != n or vertex_offsets.numel() != G + 1 or G < 1:
        raise ValueError("src, dst, t need n records and both offset arrays G+1 entries")
    if hdr.numel() < hdr_words(G):
        raise ValueError("hdr needs %d int64 words" % hdr_words(G))
    params = make_params(min_cluster_size, num_vertices, False, max_dt, thresholds, time_bits)
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    st = lib.ce_cluster_batch_async(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                    ctypes.c_void_p(t.data_ptr()), n, ctypes.c_void_p(edge_offsets.data_ptr()),
                                    ctypes.c_void_p(vertex_offsets.data_ptr()), G, int(num_vertices),
                                    ctypes.byref(params), ctypes.byref(outputs.struct),
                                    ctypes.c_void_p(hdr.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                                    workspace.numel(), ctypes.c_void_p(s.cuda_stream))
    if st != CE_OK:
        raise ClusterError(st, last_error(), "ce_cluster_batch_async")


def result_status(hdr, num_graphs: int = 1, stream=None):
    """Wait for the stream and read an asynchronous call's header (``ce_result_status``): returns
    (counts int64[G, 3] as m, n_clusters, n_labels; row_offsets int64[G+1]; cluster_offsets int64[G+1]) or
    raises ClusterError with the call's status."""
    import numpy as np
    import torch
    G = int(num_graphs)
    counts = (CeCounts * G)()
    roff = np.zeros(G + 1, dtype=np.int64)
    coff = np.zeros(G + 1, dtype=np.int64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    s = stream if stream is not None else torch.cuda.current_stream(hdr.device)
    st = load_library().ce_result_status(ctypes.c_void_p(hdr.data_ptr()), G, counts, roff.ctypes.data_as(i64p),
                                         coff.ctypes.data_as(i64p), ctypes.c_void_p(s.cuda_stream))
    if st != CE_OK:
        raise ClusterError(st, last_error(), "ce_result_status")
    return np.ctypeslib.as_array(counts).view(np.int64).reshape(G, 3).copy(), roff, coff


def async_result(outputs: Outputs, n: int, hdr, stream=None) -> Result:
    """The Result of a finished ``cluster_edges_async`` call (waits for the stream)."""
    c, _, _ = result_status(hdr, 1, stream)
    cc = CeCounts(int(c[0, 0]), int(c[0, 1]), int(c[0, 2]))
    return _result(outputs, n, cc, make_params(2, 1))


def async_batch_result(outputs: Outputs, edge_offsets, hdr, stream=None) -> "BatchResult":
    """The BatchResult of a finished ``cluster_batch_async`` call; edge_offsets: host array of G+1 offsets."""
    eo = _offsets_array(edge_offsets, "edge_offsets")
    G, n = eo.size - 1, int(eo[-1])
    carr, roff, coff = result_status(hdr, G, stream)
    m_tot, c_tot = int(roff[-1]), int(coff[-1])
    o = outputs.t
    rows = {f: o[f][:m_tot] for f in ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size")}
    pts = {f: o[f][:n] for f in ("pt_cluster", "pt_lambda", "labels")}
    cls = {f: o[f][:c_tot] for f in ("cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo",
                                     "cl_selected")}
    res = Result(m=m_tot, n_clusters=c_tot, n_labels=int(carr[:, 2].sum()), **rows, **pts, **cls)
    return BatchResult(result=res, m=carr[:, 0].copy(), n_clusters=carr[:, 1].copy(), n_labels=carr[:, 2].copy(),
                       edge_offsets=eo, row_offsets=roff, cluster_offsets=coff)


def hyper_workspace_bytes(n: int, nnz: int, num_vertices: int, min_cluster_size: int, thresholds=None) -> int:
    """Workspace for a dynamic hypergraph of n hyperedges with nnz memberships."""
    p = make_params(min_cluster_size, num_vertices, thresholds=thresholds)
    return int(load_library().ce_hyper_workspace_bytes(int(n), int(nnz), ctypes.byref(p)))


def cluster_hyperedges(members, offsets, t, min_cluster_size: int, num_vertices: int,
                       outputs: Optional[Outputs] = None, workspace=None, stream=None, max_dt: int = -1,
                       thresholds=None) -> Result:
    """Cluster the hyperedges of a dynamic hypergraph (Sec. 5.3): hyperedge r is the vertex set
    members[offsets[r]:offsets[r+1]] at time t[r]; all three are contiguous GPU tensors (int32, int64,
    int64). Outputs are per hyperedge, in the layout of ``cluster_edges``."""
    import torch
    lib = load_library()
    for name, x, dt in (("members", members, torch.int32), ("offsets", offsets, torch.int64),
                        ("t", t, torch.int64)):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == dt and x.is_contiguous() and x.dim() == 1):
            raise TypeError("%s must be a contiguous 1-D %s GPU tensor" % (name, dt))
    n, nnz = int(t.numel()), int(members.numel())
    if offsets.numel() != n + 1:
        raise ValueError("offsets must have n + 1 entries")
    if outputs is None or outputs.n < n or outputs.C < max_clusters(n, min_cluster_size):
        outputs = Outputs(n, min_cluster_size, t.device)
    params = make_params(min_cluster_size, num_vertices, False, max_dt, thresholds)
    counts = CeCounts()
    s = stream if stream is not None else torch.cuda.current_stream(t.device)
    ws_ptr, ws_len = None, 0
    if workspace is not None:
        ws_ptr, ws_len = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    st = lib.ce_cluster_hyperedges(ctypes.c_void_p(members.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
                                   ctypes.c_void_p(t.data_ptr()), n, nnz, ctypes.byref(params),
                                   ctypes.byref(outputs.struct), ctypes.byref(counts), ctypes.c_void_p(ws_ptr),
                                   ws_len, ctypes.c_void_p(s.cuda_stream))
    if st != CE_OK:
        raise ClusterError(st, last_error())
    return _result(outputs, n, counts, params)


def level_components(msf_tail, msf_head, msf_w, n: int, thresholds, labels=None, stream=None):
    """Alg. 5 by connected components (``ce_level_components``): for each threshold, the partition of the n
    records into components of the line graph restricted to w <= threshold, computed from the sorted forest
    rows a clustering call returned (``Result.msf_tail``, ``msf_head``, ``msf_w``, GPU tensors). Returns an
    int32 GPU tensor of shape (len(thresholds), n): the smallest record id of each record's component per
    level. ``labels`` may be a preallocated contiguous int32 GPU tensor of at least len(thresholds) * n."""
    import numpy as np
    import torch
    lib = load_library()
    for name, x, dt in (("msf_tail", msf_tail, torch.int32), ("msf_head", msf_head, torch.int32),
                        ("msf_w", msf_w, torch.int64)):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == dt and x.is_contiguous() and x.dim() == 1):
            raise TypeError("%s must be a contiguous 1-D %s GPU tensor" % (name, dt))
    m = int(msf_tail.numel())
    if msf_head.numel() != m or msf_w.numel() != m:
        raise ValueError("msf_tail, msf_head, msf_w must have the same length")
    thr = np.ascontiguousarray(np.asarray(thresholds, dtype=np.int64).reshape(-1))
    q, n = int(thr.size), int(n)
    if labels is None:
        labels = torch.empty(max(q * n, 1), dtype=torch.int32, device=msf_tail.device)
    elif not (isinstance(labels, torch.Tensor) and labels.is_cuda and labels.dtype == torch.int32
              and labels.is_contiguous() and labels.numel() >= q * n):
        raise TypeError("labels must be a contiguous int32 GPU tensor of at least len(thresholds) * n entries")
    s = stream if stream is not None else torch.cuda.current_stream(msf_tail.device)
    st = lib.ce_level_components(ctypes.c_void_p(msf_tail.data_ptr()), ctypes.c_void_p(msf_head.data_ptr()),
                                 ctypes.c_void_p(msf_w.data_ptr()), m, n,
                                 thr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), q,
                                 ctypes.c_void_p(labels.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    if st != CE_OK:
        raise ClusterError(st, last_error(), call="ce_level_components")
    return labels[:q * n].view(q, n)


def _result(outputs, n, counts, params) -> Result:
    m, nc, nl = int(counts.m), int(counts.n_clusters), int(counts.n_labels)
    o = outputs.t
    rows = {f: o[f][:m] for f in ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size")}
    pts = {f: o[f][:n] for f in ("pt_cluster", "pt_lambda", "labels")}
    cls = {f: o[f][:nc] for f in ("cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo",
                                  "cl_selected")}
    dd = {f: o[f][:m] for f in ("dd_level", "dd_top")} if params.num_thresholds else {}
    return Result(m=m, n_clusters=nc, n_labels=nl, **rows, **pts, **cls, **dd)


def _offsets_array(x, name):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(x, dtype=np.int64))
    if a.ndim != 1 or a.size < 2:
        raise ValueError("%s must be a 1-D array of G+1 offsets" % name)
    return a


def batch_workspace_bytes(edge_offsets, vertex_offsets, min_cluster_size: int, thresholds=None) -> int:
    eo, vo = _offsets_array(edge_offsets, "edge_offsets"), _offsets_array(vertex_offsets, "vertex_offsets")
    if eo.size != vo.size:
        raise ValueError("edge_offsets and vertex_offsets must have the same length")
    p = make_params(min_cluster_size, max(int(vo[-1]), 1), thresholds=thresholds)
    i64p = ctypes.POINTER(ctypes.c_int64)
    return int(load_library().ce_batch_workspace_bytes(eo.ctypes.data_as(i64p), vo.ctypes.data_as(i64p),
                                                       eo.size - 1, ctypes.byref(p)))


def batch_cluster_capacity(edge_offsets, min_cluster_size: int) -> int:
    """Cluster rows a batch can produce: the sum of its graphs' max_clusters."""
    import numpy as np
    eo = _offsets_array(edge_offsets, "edge_offsets")
    ng = np.diff(eo)
    return int((2 * (ng // int(min_cluster_size)) + 1).sum())


def batch_outputs(edge_offsets, min_cluster_size: int, device) -> Outputs:
    eo = _offsets_array(edge_offsets, "edge_offsets")
    n = int(eo[-1])
    return Outputs(n, min_cluster_size, device, clusters=batch_cluster_capacity(eo, min_cluster_size),
                   rows=max(n, 1))


class BatchResult(NamedTuple):
    """Outputs of a batch: the device tensors of one Result laid out graph by
    graph, plus host arrays of per-graph counts and offsets."""
    result: Result
    m: object               # numpy int64[G]
    n_clusters: object      # numpy int64[G]
    n_labels: object        # numpy int64[G]
    edge_offsets: object    # numpy int64[G+1]
    row_offsets: object     # numpy int64[G+1]
    cluster_offsets: object  # numpy int64[G+1]

    def graph(self, g: int) -> dict:
        """Host copy (numpy, documented dtypes) of graph g's outputs, as cluster_edges gives them."""
        e0, e1 = int(self.edge_offsets[g]), int(self.edge_offsets[g + 1])
        r0, r1 = int(self.row_offsets[g]), int(self.row_offsets[g + 1])
        c0, c1 = int(self.cluster_offsets[g]), int(self.cluster_offsets[g + 1])
        parts = {}
        for f in Result._fields[3:]:
            x = getattr(self.result, f)
            if x is None:
                parts[f] = None
            elif f.startswith("msf_") or f.startswith("sl_") or f.startswith("dd_"):
                parts[f] = x[r0:r1]
            elif f.startswith("pt_") or f == "labels":
                parts[f] = x[e0:e1]
            else:
                parts[f] = x[c0:c1]
        return to_numpy(Result(m=int(self.m[g]), n_clusters=int(self.n_clusters[g]), n_labels=int(self.n_labels[g]),
                               **parts))


def cluster_batch(src, dst, t, edge_offsets, vertex_offsets, min_cluster_size: int,
                  outputs: Optional[Outputs] = None, workspace=None, stream=None, causal: bool = False,
                  max_dt: int = -1, thresholds=None) -> BatchResult:
    """Cluster a batch of independent graphs in one call (``ce_cluster_batch``).

    src/dst/t hold the graphs' records back to back (GPU tensors), vertex ids
    local to each graph; edge_offsets/vertex_offsets are host arrays of G+1
    offsets. Each graph's outputs equal a separate ``cluster_edges`` call.
    """
    import numpy as np
    import torch
    lib = load_library()
    for name, x, dt in (("src", src, torch.int32), ("dst", dst, torch.int32), ("t", t, torch.int64)):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == dt and x.is_contiguous() and x.dim() == 1):
            raise TypeError("%s must be a contiguous 1-D %s GPU tensor" % (name, dt))
    eo, vo = _offsets_array(edge_offsets, "edge_offsets"), _offsets_array(vertex_offsets, "vertex_offsets")
    if eo.size != vo.size:
        raise ValueError("edge_offsets and vertex_offsets must have the same length")
    G, n = eo.size - 1, int(src.numel())
    if dst.numel() != n or t.numel() != n or int(eo[-1]) != n:
        raise ValueError("src, dst, t must have edge_offsets[-1] records")
    cap = batch_cluster_capacity(eo, min_cluster_size)
    if outputs is None or outputs.n < n or outputs.C < cap or outputs.R < max(n, 1):
        outputs = batch_outputs(eo, min_cluster_size, src.device)
    params = make_params(min_cluster_size, max(int(vo[-1]), 1), causal, max_dt, thresholds)
    counts = (CeCounts * G)()
    roff = np.zeros(G + 1, dtype=np.int64)
    coff = np.zeros(G + 1, dtype=np.int64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    ws_ptr, ws_len = None, 0
    if workspace is not None:
        ws_ptr, ws_len = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    st = lib.ce_cluster_batch(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                              ctypes.c_void_p(t.data_ptr()), eo.ctypes.data_as(i64p), vo.ctypes.data_as(i64p), G,
                              ctypes.byref(params), ctypes.byref(outputs.struct), counts, roff.ctypes.data_as(i64p),
                              coff.ctypes.data_as(i64p), ctypes.c_void_p(ws_ptr), ws_len,
                              ctypes.c_void_p(s.cuda_stream))
    if st != CE_OK:
        raise ClusterError(st, last_error(), "ce_cluster_batch")
    carr = np.ctypeslib.as_array(counts).view(np.int64).reshape(G, 3) if G else np.zeros((0, 3), np.int64)
    m_tot, c_tot = int(roff[-1]), int(coff[-1])
    o = outputs.t
    rows = {f: o[f][:m_tot] for f in ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size")}
    pts = {f: o[f][:n] for f in ("pt_cluster", "pt_lambda", "labels")}
    cls = {f: o[f][:c_tot] for f in ("cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo",
                                     "cl_selected")}
    dd = {f: o[f][:m_tot] for f in ("dd_level", "dd_top")} if params.num_thresholds else {}
    res = Result(m=m_tot, n_clusters=c_tot, n_labels=int(carr[:, 2].sum()), **rows, **pts, **cls, **dd)
    return BatchResult(result=res, m=carr[:, 0].copy(), n_clusters=carr[:, 1].copy(), n_labels=carr[:, 2].copy(),
                       edge_offsets=eo, row_offsets=roff, cluster_offsets=coff)


class ServerBusy(ClusterError):
    """The server cannot admit the request now (in-flight limit or input memory); retry after polling."""


class RequestResult(NamedTuple):
    status: int            # the request's own outcome (CE_OK or an error code)
    error: str
    result: Optional[Result]
    queue_s: float
    latency_s: float


def server_request_bytes(n: int, num_vertices: int, min_cluster_size: int) -> int:
    """Device bytes one request of n records occupies while it runs alone (the admission footprint)."""
    p = make_params(min_cluster_size, num_vertices)
    return int(load_library().ce_server_request_bytes(int(n), ctypes.byref(p)))


class Server:
    """Continuous-batching clustering server on one GPU (``ce_server_*``).

    ``submit`` copies a request's host records to the GPU and returns a
    ticket; ``poll`` returns None while the request is pending, else a
    RequestResult with trimmed device tensors of its outputs.
    """

    def __init__(self, hbm_budget_bytes: int, workers: int = 2, max_inflight: int = 256,
                 input_fraction_pct: int = 25, max_batch_records: int = 0, device: int = 0):
        lib = load_library()
        cfg = CeServerConfig(ctypes.sizeof(CeServerConfig), int(device), int(workers), int(input_fraction_pct),
                             int(hbm_budget_bytes), int(max_inflight), int(max_batch_records))
        h = ctypes.c_void_p()
        st = lib.ce_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if st != CE_OK:
            raise ClusterError(st, last_error(), "ce_server_create")
        self._h = h
        self._pending = {}

    def submit(self, src, dst, t, min_cluster_size: int, num_vertices: int, outputs: Optional[Outputs] = None,
               device=None, causal: bool = False, max_dt: int = -1, thresholds=None) -> int:
        import numpy as np
        import torch
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        t = np.ascontiguousarray(t, dtype=np.int64)
        n = int(src.shape[0])
        if dst.shape[0] != n or t.shape[0] != n:
            raise ValueError("src, dst, t must have the same length")
        if outputs is None or outputs.n < n or outputs.C < max_clusters(n, min_cluster_size):
            outputs = Outputs(n, min_cluster_size, device if device is not None else torch.device("cuda:0"))
        req = CeRequest(ctypes.sizeof(CeRequest), 0, src.ctypes.data, dst.ctypes.data, t.ctypes.data, n,
                        make_params(min_cluster_size, num_vertices, causal, max_dt, thresholds), outputs.struct)
        ticket = ctypes.c_uint64()
        st = load_library().ce_server_submit(self._h, ctypes.byref(req), ctypes.byref(ticket))
        if st == CE_EBUSY:
            raise ServerBusy(st, last_error(), "ce_server_submit")
        if st != CE_OK:
            raise ClusterError(st, last_error(), "ce_server_submit")
        self._pending[int(ticket.value)] = (outputs, n, thresholds is not None and len(thresholds) > 0)
        return int(ticket.value)

    def poll(self, ticket: int, wait: bool = False) -> Optional[RequestResult]:
        rs = CeRequestStatus()
        st = load_library().ce_server_poll(self._h, int(ticket), 1 if wait else 0, ctypes.byref(rs))
        if st == CE_EBUSY:
            return None
        if st != CE_OK:
            raise ClusterError(st, last_error(), "ce_server_poll")
        outputs, n, discrete = self._pending.pop(int(ticket))
        err = last_error() if rs.status != CE_OK else ""
        res = None
        if rs.status == CE_OK:
            m, nc, nl = int(rs.counts.m), int(rs.counts.n_clusters), int(rs.counts.n_labels)
            o = outputs.t
            rows = {f: o[f][:m] for f in ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size")}
            pts = {f: o[f][:n] for f in ("pt_cluster", "pt_lambda", "labels")}
            cls = {f: o[f][:nc] for f in ("cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi",
                                          "cl_stab_lo", "cl_selected")}
            dd = {f: o[f][:m] for f in ("dd_level", "dd_top")} if discrete else {}
            res = Result(m=m, n_clusters=nc, n_labels=nl, **rows, **pts, **cls, **dd)
        return RequestResult(int(rs.status), err, res, float(rs.queue_s), float(rs.latency_s))

    def stats(self) -> dict:
        s = CeServerStats()
        load_library().ce_server_get_stats(self._h, ctypes.byref(s))
        return {f: int(getattr(s, f)) for f in _STAT_FIELDS}

    def close(self):
        if getattr(self, "_h", None):
            load_library().ce_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_UNSIGNED = {"msf_tail": "u4", "msf_head": "u4", "sl_left": "u4", "sl_right": "u4", "sl_size": "u4",
             "pt_cluster": "u4", "pt_lambda": "u8", "cl_id": "u4", "cl_parent": "u4", "cl_size": "u4",
             "cl_lambda_birth": "u8", "cl_stab_hi": "u8", "cl_stab_lo": "u8", "dd_level": "u4", "dd_top": "u4"}


def to_numpy(res: Result) -> dict:
    """Copy a Result to host numpy arrays with the documented (unsigned) dtypes."""
    out = {"m": res.m, "n_clusters": res.n_clusters, "n_labels": res.n_labels}
    for f in Result._fields[3:]:
        x = getattr(res, f)
        if x is None:
            continue
        a = x.cpu().numpy()
        out[f] = a.view(_UNSIGNED[f]) if f in _UNSIGNED else a
    return out
