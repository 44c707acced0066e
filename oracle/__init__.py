"""CPU oracle for the edge clustering of dynamic graphs -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The GPU library neither imports nor links
it; the two share no code. The arithmetic lives in ``ce_oracle.c`` (plain C,
host only); this module is argument marshalling.

Tier A (``tier=0``) is the definition: the full undirected line graph
(Sec. 1.2.2), or with ``causal=True`` the increment-weighted line graph of
Def. 1, and Kruskal in canonical-key order. Tier B (``tier=1``) follows the
method's own steps: per-vertex time-sorted incidence lists, then the path
skeleton (Alg. 3 with the undirected node-local MST of Sec. 5.3) or the
Alg. 2 windows, then Kruskal.
Both continue with the union-find dendrogram and the HDBSCAN condensing and
excess-of-mass extraction of Alg. 1. Dynamic hypergraphs (Sec. 5.3) have the
same two tiers: every pair of hyperedges whose vertex sets meet, or the
per-vertex time-sorted paths over incident hyperedges.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import NamedTuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

LG_EDGE = np.dtype([("w", "<i8"), ("tail", "<u4"), ("head", "<u4")])

OK, EINVAL, ESELFLOOP, ERANGE, ENOMEM = 0, -1, -2, -3, -4


def build_oracle(force: bool = False) -> str:
    src = os.path.join(_HERE, "ce_oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("CE_ORACLE_LIB")  # tests load planted-mistake builds this way
        if not path:
            if not os.path.exists(_LIB_PATH):
                build_oracle()
            path = _LIB_PATH
        lib = ctypes.CDLL(path)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.oracle_validate.argtypes = [i64, p, p, p, i64]
        lib.oracle_validate.restype = ctypes.c_int
        lib.oracle_full_line_graph.argtypes = [i64, p, p, p, i64, p]
        lib.oracle_full_line_graph.restype = i64
        lib.oracle_skeleton.argtypes = [i64, p, p, p, i64, p]
        lib.oracle_skeleton.restype = i64
        lib.oracle_kruskal.argtypes = [i64, i64, p, p, p, p, p]
        lib.oracle_kruskal.restype = i64
        lib.oracle_dendrogram.argtypes = [i64, i64, p, p, p, p, p, p, p]
        lib.oracle_dendrogram.restype = ctypes.c_int
        lib.oracle_joined_below.argtypes = [i64, i64, p, p, p, i64, p, p, p, p]
        lib.oracle_joined_below.restype = ctypes.c_int
        lib.oracle_level_components.argtypes = [i64, i64, p, p, p, i64, p, p]
        lib.oracle_level_components.restype = ctypes.c_int
        lib.oracle_condense.argtypes = [i64, i64, p, p, p, p, i64] + [p] * 10 + [p]
        lib.oracle_condense_discrete.argtypes = [i64, i64, p, p, p, p, i64, i64, p] + [p] * 10 + [p, p, p]
        lib.oracle_condense_discrete.restype = ctypes.c_int
        lib.oracle_condense.restype = ctypes.c_int
        lib.oracle_causal_line_graph.argtypes = [i64, p, p, p, i64, p]
        lib.oracle_causal_line_graph.restype = i64
        lib.oracle_causal_skeleton.argtypes = [i64, p, p, p, i64, p]
        lib.oracle_causal_skeleton.restype = i64
        lib.oracle_cluster.argtypes = [i64, p, p, p, i64, i64, ctypes.c_int, ctypes.c_int, i64] + [p] * 18
        lib.oracle_cluster.restype = ctypes.c_int
        lib.oracle_hyper_validate.argtypes = [i64, p, p, p, i64]
        lib.oracle_hyper_validate.restype = ctypes.c_int
        lib.oracle_hyper_line_graph.argtypes = [i64, p, p, p, i64, p]
        lib.oracle_hyper_line_graph.restype = i64
        lib.oracle_hyper_skeleton.argtypes = [i64, p, p, p, i64, p]
        lib.oracle_hyper_skeleton.restype = i64
        lib.oracle_cluster_hyper.argtypes = [i64, p, p, p, i64, i64, ctypes.c_int, i64] + [p] * 18
        lib.oracle_cluster_hyper.restype = ctypes.c_int
        _lib = lib
    return _lib


def _prep(src, dst, t):
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int64)
    assert src.shape == dst.shape == t.shape and src.ndim == 1
    return src, dst, t


def _V(src, dst, V):
    if V is None or V == 0:
        return int(max(src.max(initial=-1), dst.max(initial=-1)) + 1)
    return int(V)


def validate(src, dst, t, V=None) -> int:
    src, dst, t = _prep(src, dst, t)
    return int(_load().oracle_validate(src.size, src.ctypes.data, dst.ctypes.data, t.ctypes.data, _V(src, dst, V)))


def full_line_graph_size(src, dst, t, V=None) -> int:
    src, dst, t = _prep(src, dst, t)
    return int(_load().oracle_full_line_graph(src.size, src.ctypes.data, dst.ctypes.data, t.ctypes.data,
                                              _V(src, dst, V), None))


def full_line_graph(src, dst, t, V=None, limit=200_000_000) -> np.ndarray:
    """All undirected line-graph edges (tail, head, w), pairs sharing both endpoints once."""
    src, dst, t = _prep(src, dst, t)
    V = _V(src, dst, V)
    lib = _load()
    cnt = int(lib.oracle_full_line_graph(src.size, src.ctypes.data, dst.ctypes.data, t.ctypes.data, V, None))
    if cnt > limit:
        raise MemoryError("full line graph has %d edges (limit %d)" % (cnt, limit))
    out = np.empty(max(cnt, 1), dtype=LG_EDGE)
    lib.oracle_full_line_graph(src.size, src.ctypes.data, dst.ctypes.data, t.ctypes.data, V, out.ctypes.data)
    return out[:cnt]


def skeleton(src, dst, t, V=None) -> np.ndarray:
    """Path skeleton rows (tail, head, w), 2n - V' rows, in vertex then list order."""
    src, dst, t = _prep(src, dst, t)
    V = _V(src, dst, V)
    lib = _load()
    cnt = int(lib.oracle_skeleton(src.size, src.ctypes.data, dst.ctypes.data, t.ctypes.data, V, None))
    out = np.empty(max(cnt, 1), dtype=LG_EDGE)
    lib.oracle_skeleton(src.size, src.ctypes.data, dst.ctypes.data, t.ctypes.data, V, out.ctypes.data)
    return out[:cnt]


def _edges(fn, src, dst, t, V, limit):
    src, dst, t = _prep(src, dst, t)
    V = _V(src, dst, V)
    cnt = int(fn(src.size, src.ctypes.data, dst.ctypes.data, t.ctypes.data, V, None))
    if cnt < 0:
        raise RuntimeError("oracle edge generator: %d" % cnt)
    if cnt > limit:
        raise MemoryError("line graph has %d edges (limit %d)" % (cnt, limit))
    out = np.empty(max(cnt, 1), dtype=LG_EDGE)
    fn(src.size, src.ctypes.data, dst.ctypes.data, t.ctypes.data, V, out.ctypes.data)
    return out[:cnt]


def causal_line_graph(src, dst, t, V=None, limit=200_000_000) -> np.ndarray:
    """All arcs (tail, head, w) of the increment-weighted line graph (Def. 1)."""
    return _edges(_load().oracle_causal_line_graph, src, dst, t, V, limit)


def causal_skeleton(src, dst, t, V=None) -> np.ndarray:
    """Alg. 2 window rows (tail, head, w) at every vertex, in vertex then list order."""
    return _edges(_load().oracle_causal_skeleton, src, dst, t, V, 1 << 62)


def kruskal(n, edges, t):
    """MSF rows (tail, head, w) in ascending canonical key; edges are not modified."""
    e = np.array(edges, dtype=LG_EDGE, copy=True)
    t = np.ascontiguousarray(t, dtype=np.int64)
    cap = max(int(n) - 1, 1)
    mt = np.empty(cap, np.uint32)
    mh = np.empty(cap, np.uint32)
    mw = np.empty(cap, np.int64)
    m = int(_load().oracle_kruskal(int(n), e.size, e.ctypes.data, t.ctypes.data, mt.ctypes.data, mh.ctypes.data,
                                   mw.ctypes.data))
    if m < 0:
        raise RuntimeError("oracle_kruskal: %d" % m)
    return mt[:m], mh[:m], mw[:m]


def dendrogram(n, msf_tail, msf_head, msf_w):
    mt = np.ascontiguousarray(msf_tail, np.uint32)
    mh = np.ascontiguousarray(msf_head, np.uint32)
    mw = np.ascontiguousarray(msf_w, np.int64)
    m = mt.size
    left = np.empty(max(m, 1), np.uint32)
    right = np.empty(max(m, 1), np.uint32)
    lw = np.empty(max(m, 1), np.int64)
    size = np.empty(max(m, 1), np.uint32)
    rc = _load().oracle_dendrogram(int(n), m, mt.ctypes.data, mh.ctypes.data, mw.ctypes.data, left.ctypes.data,
                                   right.ctypes.data, lw.ctypes.data, size.ctypes.data)
    if rc:
        raise RuntimeError("oracle_dendrogram: %d" % rc)
    return left[:m], right[:m], lw[:m], size[:m]


def joined_below(n, msf_tail, msf_head, msf_w, q_tail, q_head, q_w) -> np.ndarray:
    """Cycle-property check: for each query edge, whether forest rows of smaller key already join its records."""
    mt = np.ascontiguousarray(msf_tail, np.uint32)
    mh = np.ascontiguousarray(msf_head, np.uint32)
    mw = np.ascontiguousarray(msf_w, np.int64)
    qt = np.ascontiguousarray(q_tail, np.uint32)
    qh = np.ascontiguousarray(q_head, np.uint32)
    qw = np.ascontiguousarray(q_w, np.int64)
    out = np.empty(max(qt.size, 1), np.uint8)
    rc = _load().oracle_joined_below(int(n), mt.size, mt.ctypes.data, mh.ctypes.data, mw.ctypes.data, qt.size,
                                     qt.ctypes.data, qh.ctypes.data, qw.ctypes.data, out.ctypes.data)
    if rc:
        raise RuntimeError("oracle_joined_below: %d" % rc)
    return out[:qt.size].astype(bool)


def level_components(n, tail, head, w, thresholds) -> np.ndarray:
    """Alg. 5 by components: labels[l, r] = smallest record id in r's component of the line graph restricted to
    edges with w <= thresholds[l] (the given edges: full line graph, skeleton or forest), each level from scratch."""
    tl = np.ascontiguousarray(tail, np.uint32)
    hd = np.ascontiguousarray(head, np.uint32)
    ww = np.ascontiguousarray(w, np.int64)
    thr = np.ascontiguousarray(thresholds, np.int64)
    out = np.empty(max(thr.size * int(n), 1), np.int32)
    rc = _load().oracle_level_components(int(n), tl.size, tl.ctypes.data, hd.ctypes.data, ww.ctypes.data, thr.size,
                                         thr.ctypes.data, out.ctypes.data)
    if rc:
        raise ValueError("oracle_level_components: %d" % rc)
    return out[:thr.size * int(n)].reshape(thr.size, int(n))


def max_clusters(n, M):
    return 2 * (int(n) // int(M)) + 1


class Condensed(NamedTuple):
    pt_cluster: np.ndarray
    pt_lambda: np.ndarray
    cl_id: np.ndarray
    cl_parent: np.ndarray
    cl_size: np.ndarray
    cl_lambda_birth: np.ndarray
    cl_stab_hi: np.ndarray
    cl_stab_lo: np.ndarray
    cl_selected: np.ndarray
    labels: np.ndarray
    n_labels: int


class _Counts(ctypes.Structure):
    _fields_ = [("n_clusters", ctypes.c_int64), ("n_labels", ctypes.c_int64)]


def condense(n, left, right, lw, size, M) -> Condensed:
    left = np.ascontiguousarray(left, np.uint32)
    right = np.ascontiguousarray(right, np.uint32)
    lw = np.ascontiguousarray(lw, np.int64)
    size = np.ascontiguousarray(size, np.uint32)
    m = left.size
    C = max_clusters(n, M)
    ptc = np.empty(max(n, 1), np.uint32)
    ptl = np.empty(max(n, 1), np.uint64)
    arrs = [np.empty(C, np.uint32), np.empty(C, np.uint32), np.empty(C, np.uint32), np.empty(C, np.uint64),
            np.empty(C, np.uint64), np.empty(C, np.uint64), np.empty(C, np.uint8)]
    labels = np.empty(max(n, 1), np.int32)
    cnt = _Counts()
    rc = _load().oracle_condense(int(n), m, left.ctypes.data, right.ctypes.data, lw.ctypes.data, size.ctypes.data,
                                 int(M), ptc.ctypes.data, ptl.ctypes.data, *[a.ctypes.data for a in arrs],
                                 labels.ctypes.data, ctypes.byref(cnt))
    if rc:
        raise RuntimeError("oracle_condense: %d" % rc)
    k = int(cnt.n_clusters)
    return Condensed(ptc[:n], ptl[:n], *[a[:k] for a in arrs], labels[:n], int(cnt.n_labels))


class Discrete(NamedTuple):
    condensed: Condensed
    dd_level: np.ndarray   # level (threshold index) of every dendrogram row
    dd_top: np.ndarray     # node n+j of the row's level top j (its D-node)


def condense_discrete(n, left, right, lw, size, M, thresholds) -> Discrete:
    """Alg. 5 discrete dendrogram cut from the exact one, condensed with several children per node. All rows
    must have w <= thresholds[-1]."""
    left = np.ascontiguousarray(left, np.uint32)
    right = np.ascontiguousarray(right, np.uint32)
    lw = np.ascontiguousarray(lw, np.int64)
    size = np.ascontiguousarray(size, np.uint32)
    thr = np.ascontiguousarray(thresholds, np.int64)
    m = left.size
    C = max_clusters(n, M)
    ptc = np.empty(max(n, 1), np.uint32)
    ptl = np.empty(max(n, 1), np.uint64)
    arrs = [np.empty(C, np.uint32), np.empty(C, np.uint32), np.empty(C, np.uint32), np.empty(C, np.uint64),
            np.empty(C, np.uint64), np.empty(C, np.uint64), np.empty(C, np.uint8)]
    labels = np.empty(max(n, 1), np.int32)
    dl = np.empty(max(m, 1), np.uint32)
    dt = np.empty(max(m, 1), np.uint32)
    cnt = _Counts()
    rc = _load().oracle_condense_discrete(int(n), m, left.ctypes.data, right.ctypes.data, lw.ctypes.data,
                                          size.ctypes.data, int(M), thr.size, thr.ctypes.data, ptc.ctypes.data,
                                          ptl.ctypes.data, *[a.ctypes.data for a in arrs], labels.ctypes.data,
                                          dl.ctypes.data, dt.ctypes.data, ctypes.byref(cnt))
    if rc:
        raise RuntimeError("oracle_condense_discrete: %d" % rc)
    k = int(cnt.n_clusters)
    cond = Condensed(ptc[:n], ptl[:n], *[a[:k] for a in arrs], labels[:n], int(cnt.n_labels))
    return Discrete(cond, dl[:m], dt[:m])


def cluster_discrete(src, dst, t, min_cluster_size, thresholds, num_vertices=None, tier=1, causal=False):
    """Whole pipeline with the discrete dendrogram: the forest up to the last threshold, its exact dendrogram
    (sl_* fields), then the Alg. 5 levels and the condensing on the discrete tree. Returns (Result, dd_level,
    dd_top); the Result's condensed fields are the discrete ones."""
    thr = np.asarray(thresholds, np.int64)
    r = cluster(src, dst, t, min_cluster_size, num_vertices, tier=tier, causal=causal, max_dt=int(thr[-1]))
    return _discrete_tail(r, len(src), min_cluster_size, thr)


def _discrete_tail(r, n, min_cluster_size, thr):
    if r.status != 0:
        return r, None, None
    d = condense_discrete(n, r.sl_left, r.sl_right, r.sl_w, r.sl_size, min_cluster_size, thr)
    c = d.condensed
    res = r._replace(pt_cluster=c.pt_cluster, pt_lambda=c.pt_lambda, cl_id=c.cl_id, cl_parent=c.cl_parent,
                     cl_size=c.cl_size, cl_lambda_birth=c.cl_lambda_birth, cl_stab_hi=c.cl_stab_hi,
                     cl_stab_lo=c.cl_stab_lo, cl_selected=c.cl_selected, labels=c.labels,
                     n_clusters=len(c.cl_id), n_labels=c.n_labels)
    return res, d.dd_level, d.dd_top


class Result(NamedTuple):
    status: int
    m: int
    msf_tail: np.ndarray
    msf_head: np.ndarray
    msf_w: np.ndarray
    sl_left: np.ndarray
    sl_right: np.ndarray
    sl_w: np.ndarray
    sl_size: np.ndarray
    pt_cluster: np.ndarray
    pt_lambda: np.ndarray
    cl_id: np.ndarray
    cl_parent: np.ndarray
    cl_size: np.ndarray
    cl_lambda_birth: np.ndarray
    cl_stab_hi: np.ndarray
    cl_stab_lo: np.ndarray
    cl_selected: np.ndarray
    labels: np.ndarray
    n_clusters: int
    n_labels: int


def cluster(src, dst, t, min_cluster_size, num_vertices=None, tier=1, causal=False, max_dt=-1) -> Result:
    """Whole pipeline. tier=0: full line graph (definition); tier=1: skeleton (Alg. 3). causal=True: the
    increment-weighted line graph of Def. 1 (tip-to-tail arcs, Alg. 2 windows in tier 1). max_dt >= 0: only
    line-graph edges with w <= max_dt (time-filtered line graph)."""
    src, dst, t = _prep(src, dst, t)
    V = _V(src, dst, num_vertices)
    return _pipeline(lambda M, bufs, hdr: _load().oracle_cluster(
        src.size, src.ctypes.data, dst.ctypes.data, t.ctypes.data, V, M, int(tier), int(bool(causal)), int(max_dt),
        *[b.ctypes.data for b in bufs], hdr.ctypes.data), src.size, min_cluster_size)


def _hyper_prep(members, offsets, t):
    members = np.ascontiguousarray(members, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    t = np.ascontiguousarray(t, dtype=np.int64)
    assert offsets.ndim == 1 and offsets.size == t.size + 1 and members.ndim == 1
    return members, offsets, t


def _hyper_V(members, V):
    return int(members.max(initial=-1) + 1) if V is None or V == 0 else int(V)


def hyper_validate(members, offsets, t, V=None) -> int:
    members, offsets, t = _hyper_prep(members, offsets, t)
    return int(_load().oracle_hyper_validate(t.size, offsets.ctypes.data, members.ctypes.data, t.ctypes.data,
                                             _hyper_V(members, V)))


def _hyper_edges(fn, members, offsets, t, V, limit):
    members, offsets, t = _hyper_prep(members, offsets, t)
    V = _hyper_V(members, V)
    args = (t.size, offsets.ctypes.data, members.ctypes.data, t.ctypes.data, V)
    cnt = int(fn(*args, None))
    if cnt < 0:
        raise RuntimeError("oracle edge generator: %d" % cnt)
    if cnt > limit:
        raise MemoryError("line graph has %d edges (limit %d)" % (cnt, limit))
    out = np.empty(max(cnt, 1), dtype=LG_EDGE)
    fn(*args, out.ctypes.data)
    return out[:cnt]


def hyper_line_graph(members, offsets, t, V=None, limit=200_000_000) -> np.ndarray:
    """Every line-graph edge of a dynamic hypergraph (hyperedges whose vertex sets meet), each pair once."""
    return _hyper_edges(_load().oracle_hyper_line_graph, members, offsets, t, V, limit)


def hyper_skeleton(members, offsets, t, V=None) -> np.ndarray:
    """Per-vertex time-sorted paths over incident hyperedges: sum_i (d_i - 1) rows, vertex then list order."""
    return _hyper_edges(_load().oracle_hyper_skeleton, members, offsets, t, V, 1 << 62)


def cluster_hyper(members, offsets, t, min_cluster_size, num_vertices=None, tier=1, max_dt=-1) -> Result:
    """Whole pipeline on a dynamic hypergraph (hyperedge r = members[offsets[r]:offsets[r+1]] at time t[r]).
    tier=0: full line graph; tier=1: per-vertex path skeleton. Per-record outputs are per hyperedge."""
    members, offsets, t = _hyper_prep(members, offsets, t)
    V = _hyper_V(members, num_vertices)
    return _pipeline(lambda M, bufs, hdr: _load().oracle_cluster_hyper(
        t.size, offsets.ctypes.data, members.ctypes.data, t.ctypes.data, V, M, int(tier), int(max_dt),
        *[b.ctypes.data for b in bufs], hdr.ctypes.data), t.size, min_cluster_size)


def cluster_hyper_discrete(members, offsets, t, min_cluster_size, thresholds, num_vertices=None, tier=1):
    """cluster_hyper with the discrete dendrogram, as cluster_discrete does for graphs."""
    thr = np.asarray(thresholds, np.int64)
    r = cluster_hyper(members, offsets, t, min_cluster_size, num_vertices, tier=tier, max_dt=int(thr[-1]))
    return _discrete_tail(r, t.size if hasattr(t, "size") else len(t), min_cluster_size, thr)


def _pipeline(call, n, min_cluster_size) -> Result:
    M = int(min_cluster_size)
    R = max(n - 1, 1)
    C = max_clusters(n, max(M, 2))
    bufs = [np.empty(R, np.uint32), np.empty(R, np.uint32), np.empty(R, np.int64),
            np.empty(R, np.uint32), np.empty(R, np.uint32), np.empty(R, np.int64), np.empty(R, np.uint32),
            np.empty(max(n, 1), np.uint32), np.empty(max(n, 1), np.uint64),
            np.empty(C, np.uint32), np.empty(C, np.uint32), np.empty(C, np.uint32), np.empty(C, np.uint64),
            np.empty(C, np.uint64), np.empty(C, np.uint64), np.empty(C, np.uint8),
            np.empty(max(n, 1), np.int32)]
    hdr = np.zeros(4, np.int64)
    call(M, bufs, hdr)
    st, m, nc, nl = (int(x) for x in hdr)
    if st != 0:
        e = [np.empty(0, b.dtype) for b in bufs]
        return Result(st, 0, *e, 0, 0)
    b = bufs
    return Result(st, m, b[0][:m], b[1][:m], b[2][:m], b[3][:m], b[4][:m], b[5][:m], b[6][:m],
                  b[7][:n], b[8][:n], *[x[:nc] for x in b[9:16]], b[16][:n], nc, nl)


def stability(res_or_cond, i):
    """Exact u128 stability of cluster row i as a Python int."""
    return (int(res_or_cond.cl_stab_hi[i]) << 64) | int(res_or_cond.cl_stab_lo[i])
