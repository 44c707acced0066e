"""Seeded synthetic temporal edge lists (inputs only; no clustering arithmetic).

The C library ``libsynth.so`` (built from ``synth.c`` by ``build_synth``) draws
every random number from counter-based SplitMix64 streams, so a (recipe, seed)
pair gives the same arrays on any machine and any OpenMP thread count. Both the
CPU oracle and the GPU library consume the arrays returned here.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

DAY = 86400


def build_synth(force: bool = False) -> str:
    """Compile synth.c into libsynth.so (gcc, OpenMP)."""
    src = os.path.join(_HERE, "synth.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_synth()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, u64, dbl, ptr = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
        lib.synth_chung_lu_bursts.argtypes = [i64, i64, dbl, i64, ctypes.c_int, ctypes.c_int, dbl, u64, ptr, ptr, ptr]
        lib.synth_chung_lu_bursts.restype = ctypes.c_int
        lib.synth_rmat_hawkes.argtypes = [i64, ctypes.c_int, dbl, dbl, dbl, i64, dbl, dbl, dbl, i64, u64, ptr, ptr, ptr]
        lib.synth_rmat_hawkes.restype = ctypes.c_int
        lib.synth_child_seed.argtypes = [u64, u64]
        lib.synth_child_seed.restype = u64
        lib.synth_lognormal_sizes.argtypes = [i64, dbl, dbl, i64, i64, u64, ptr]
        lib.synth_lognormal_sizes.restype = None
        lib.synth_exp_gaps.argtypes = [i64, dbl, u64, ptr]
        lib.synth_exp_gaps.restype = None
        _lib = lib
    return _lib


def _alloc(n):
    return (np.empty(n, dtype=np.int32), np.empty(n, dtype=np.int32), np.empty(n, dtype=np.int64))


def chung_lu_bursts(n, V, seed, gamma=2.1, T=30 * DAY, bmin=5, bmax=50, gap_mean=60.0):
    """Chung-Lu (power-law exponent gamma) endpoints, Poisson-burst int64 times."""
    lib = _load()
    src, dst, t = _alloc(n)
    rc = lib.synth_chung_lu_bursts(int(n), int(V), float(gamma), int(T), int(bmin), int(bmax), float(gap_mean),
                                   int(seed) & (2**64 - 1), src.ctypes.data, dst.ctypes.data, t.ctypes.data)
    if rc != 0:
        raise RuntimeError("synth_chung_lu_bursts failed: %d" % rc)
    return src, dst, t


def _outputs(n, out):
    """The caller's (src int32, dst int32, t int64) arrays of n contiguous elements, or new ones."""
    if out is None:
        return _alloc(n)
    src, dst, t = out
    for x, dt in ((src, np.int32), (dst, np.int32), (t, np.int64)):
        if x.dtype != dt or x.shape != (n,) or not x.flags["C_CONTIGUOUS"] or not x.flags["WRITEABLE"]:
            raise ValueError("out arrays must be writable contiguous int32, int32, int64 of length %d" % n)
    return src, dst, t


def rmat_hawkes(n, scale, seed, a=0.57, b=0.19, c=0.19, T=90 * DAY, mu=0.01, eta=0.7, beta=300.0, hub_extra=0,
                out=None):
    """R-MAT endpoints (2**scale vertices), per-pair Hawkes int64 times (written into `out` when given)."""
    lib = _load()
    src, dst, t = _outputs(n, out)
    rc = lib.synth_rmat_hawkes(int(n), int(scale), float(a), float(b), float(c), int(T), float(mu), float(eta),
                               float(beta), int(hub_extra), int(seed) & (2**64 - 1),
                               src.ctypes.data, dst.ctypes.data, t.ctypes.data)
    if rc != 0:
        raise RuntimeError("synth_rmat_hawkes failed: %d" % rc)
    return src, dst, t


def child_seed(seed, item):
    return int(_load().synth_child_seed(int(seed), int(item)))


def lognormal_sizes(count, median, sigma, lo, hi, seed):
    out = np.empty(count, dtype=np.int64)
    _load().synth_lognormal_sizes(int(count), float(median), float(sigma), int(lo), int(hi), int(seed), out.ctypes.data)
    return out


def exp_gaps(count, mean, seed):
    out = np.empty(count, dtype=np.float64)
    _load().synth_exp_gaps(int(count), float(mean), int(seed), out.ctypes.data)
    return out


@dataclass
class Workload:
    name: str
    src: np.ndarray
    dst: np.ndarray
    t: np.ndarray
    num_vertices: int
    min_cluster_size: int

    @property
    def n(self):
        return int(self.src.shape[0])


def plain_tiny(seed=0, n=200_000, V=10_000):
    """Tiny plain-method workload: 10k vertices, 200k edges, Chung-Lu 2.1, bursts over 30 days, M=5."""
    s, d, t = chung_lu_bursts(n, V, seed)
    return Workload("chung-lu-bursts n=%d V=%d M=5" % (n, V), s, d, t, V, 5)


def plain_mid(seed=1, n=50_000_000, scale=20):
    """Mid plain-method workload: R-MAT scale 20 (1M vertices), 50M edges, Hawkes times over 90 days, M=10."""
    s, d, t = rmat_hawkes(n, scale, seed, T=90 * DAY)
    return Workload("rmat-hawkes n=%d V=2^%d M=10" % (n, scale), s, d, t, 1 << scale, 10)


def plain_scale(seed=2, n=1 << 30, scale=26, hub_extra=8_300_000):
    """One GPU's share at scale: R-MAT scale 26, edge factor 16, planted 1e7-degree hub, Hawkes over 1 year, M=25."""
    s, d, t = rmat_hawkes(n, scale, seed, T=365 * DAY, hub_extra=hub_extra)
    return Workload("rmat-hawkes n=%d V=2^%d hub M=25" % (n, scale), s, d, t, 1 << scale, 25)


def batch_sizes(G=4096, seed=3):
    """Per-graph edge counts for the batching workload: lognormal(median 20k, sigma 1.5) clipped to [500, 2M]."""
    return lognormal_sizes(G, 20000.0, 1.5, 500, 2_000_000, seed)


def batch_graph(g, n_g, seed=3):
    """Graph g of the batching workload: Chung-Lu 2.1 endpoints over max(2, n_g/20) vertices, bursts over 30 days."""
    V = max(2, n_g // 20)
    s, d, t = chung_lu_bursts(int(n_g), int(V), child_seed(seed, g))
    return s, d, t, V


def batch_workload(G=4096, seed=3, sizes=None):
    """Concatenated batch: returns src, dst, t, edge_offsets[G+1], vertex_offsets[G+1] (local vertex ids per graph)."""
    if sizes is None:
        sizes = batch_sizes(G, seed)
    parts = [batch_graph(g, int(sizes[g]), seed) for g in range(G)]
    eoff = np.zeros(G + 1, dtype=np.int64)
    voff = np.zeros(G + 1, dtype=np.int64)
    for g, (s, d, t, V) in enumerate(parts):
        eoff[g + 1] = eoff[g] + s.shape[0]
        voff[g + 1] = voff[g] + V
    src = np.concatenate([p[0] for p in parts]) if G else np.empty(0, np.int32)
    dst = np.concatenate([p[1] for p in parts]) if G else np.empty(0, np.int32)
    t = np.concatenate([p[2] for p in parts]) if G else np.empty(0, np.int64)
    return src, dst, t, eoff, voff


def request_sizes(count=20000, seed=4):
    """Serving request sizes: lognormal(median 70711, sigma 1.42) clipped to [1e3, 5e6]."""
    return lognormal_sizes(count, 70711.0, 1.42, 1000, 5_000_000, seed)


def request_arrivals(count=20000, rate=200.0, seed=4):
    """Open-loop Poisson arrival times in seconds (exponential gaps of mean 1/rate)."""
    return np.cumsum(exp_gaps(count, 1.0 / rate, seed))


def request_graph(r, n_r, seed=4, out=None):
    """Request r: R-MAT over 2^ceil(log2(n_r/16)) vertices, Hawkes times over 90 days, M=10 (written into
    `out` when given)."""
    scale = max(1, int(math.ceil(math.log2(max(2.0, n_r / 16.0)))))
    s, d, t = rmat_hawkes(int(n_r), scale, child_seed(seed, r), T=90 * DAY, out=out)
    return s, d, t, 1 << scale


@dataclass
class HyperWorkload:
    name: str
    members: np.ndarray   # int32[nnz]
    offsets: np.ndarray   # int64[n+1]
    t: np.ndarray         # int64[n]
    num_vertices: int
    min_cluster_size: int

    @property
    def n(self):
        return int(self.t.shape[0])

    @property
    def nnz(self):
        return int(self.members.shape[0])


def hyper_bursts(n, V, seed, median=2.0, sigma=1.0, dmax=64, T=30 * DAY):
    """Dynamic hypergraph of multi-recipient messages: hyperedge r is a Chung-Lu burst record (sender, first
    recipient, time) plus k_r - 1 further Chung-Lu recipients, k_r ~ lognormal(median, sigma) clipped to
    [1, dmax]. A recipient may repeat within a message (the hyperedge is the set). Returns (members, offsets, t)."""
    s, d, t = chung_lu_bursts(n, V, seed, T=T)
    k = lognormal_sizes(n, median, sigma, 1, dmax, child_seed(seed, 1))
    extra = int((k - 1).sum())
    _, xd, _ = chung_lu_bursts(max(extra, 1), V, child_seed(seed, 2), T=T)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(k + 1, out=off[1:])
    members = np.empty(int(off[-1]), dtype=np.int32)
    first = np.ones(members.shape[0], dtype=bool)
    members[off[:-1]] = s
    members[off[:-1] + 1] = d
    first[off[:-1]] = False
    first[off[:-1] + 1] = False
    members[first] = xd[:extra]
    return members, off, t


def hyper_tiny(seed=5, n=200_000, V=10_000):
    """Tiny hypergraph workload: 200k multi-recipient messages over 10k Chung-Lu vertices, bursts over 30 days,
    M=5."""
    mem, off, t = hyper_bursts(n, V, seed)
    return HyperWorkload("hyper-bursts n=%d V=%d M=5" % (n, V), mem, off, t, V, 5)


def hyper_mid(seed=6, n=20_000_000, V=1 << 20):
    """Mid hypergraph workload: 2e7 multi-recipient messages over 2^20 Chung-Lu vertices, bursts over 90 days,
    M=10."""
    mem, off, t = hyper_bursts(n, V, seed, T=90 * DAY)
    return HyperWorkload("hyper-bursts n=%d V=2^20 M=10" % n, mem, off, t, V, 10)
