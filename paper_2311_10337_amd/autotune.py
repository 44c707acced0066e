"""Autotuner for the launch choices of a call (``ce_tuning``).

The knobs are the ones the kernels leave open: the dendrogram's largest level
width (``krt_level_bits``: sub-intervals run one after another, each over
m / 2^k rows), the row count from which Boruvka splits its edge list at a
pivot key (``split_min_edges``), the workgroups of the passes over live lists
(``list_grid``, which with a list's length sets its items per thread, i.e. the
compaction tile), and the keys per thread of every radix sort
(``radix_keys_per_thread``, the sort tile). None of them changes an output.

A sweep is coordinate descent over the knobs in that order, starting from the
built-in choices: each candidate is timed as the median wall time of ``reps``
complete calls after one warm-up call, and it is kept only if every output it
produces is identical to the built-in choices' outputs (a digest of every
field, taken on the device). A knob moves only for a gain of more than 2%, and
the final choice is timed again against the built-in one.

Choices are kept per bucket (bits(n), bits(V), bits(max degree)) in a text
file, one line per bucket::

    n_bits V_bits maxdeg_bits radix list_grid krt_bits split default_ms tuned_ms

(0 = the built-in choice, split -1 = never). The library reads the file named
by CE_TUNE_FILE on every call and takes the first line whose n_bits and V_bits
match the call; ``knobs_for`` also matches the max degree when it is given.
``python -m paper_2311_10337_amd.autotune --workload mid`` tunes one of the
synthetic workloads and writes its line.
"""
from __future__ import annotations

import os
import statistics
import time
from typing import Callable, Dict, Optional, Tuple

from . import tuned

CANDIDATES: Dict[str, Tuple[int, ...]] = {
    "krt_level_bits": (3, 4, 5, 6, 7, 8, 9, 10, 11, 12),
    "split_min_edges": (1 << 18, 1 << 22, -1),
    "list_grid": (1024, 2048, 8192, 16384),
    "radix_keys_per_thread": (4, 16),
}
ORDER = ("krt_level_bits", "split_min_edges", "list_grid", "radix_keys_per_thread")
PACKAGE_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "mi355x.tune")
HEADER = "# n_bits V_bits maxdeg_bits radix list_grid krt_bits split default_ms tuned_ms\n"


def bits(x: int) -> int:
    """Bits needed to represent x >= 0 (0 -> 0), as the library counts them."""
    return int(x).bit_length()


def bucket(n: int, V: int, maxdeg: int) -> Tuple[int, int, int]:
    return bits(n), bits(V), bits(maxdeg)


def tune_file(path: Optional[str] = None) -> str:
    return path or os.environ.get("CE_TUNE_FILE") or PACKAGE_FILE


# ------------------------------------------------------------------ digests
_MUL = 0x9E3779B97F4A7C15 - (1 << 64)  # odd multipliers as signed 64-bit values
_ADD = 0x632BE59BD9B4E019


def device_digest(tensors) -> Tuple[int, ...]:
    """Two position-weighted wrap-around sums per tensor, computed on the device: equal outputs give equal
    digests, and a changed or moved element changes them."""
    import torch
    out = []
    for x in tensors:
        if x is None:
            out.append(None)
            continue
        v = x.reshape(-1).to(torch.int64)
        i = torch.arange(v.numel(), dtype=torch.int64, device=v.device)
        out.append(int(((i * _MUL + _ADD) * (v + 1)).sum().item()))
        out.append(int(((i | 1) * (v ^ 0x5851F42D)).sum().item()))
        out.append(v.numel())
    return tuple(out)


def result_digest(r) -> Tuple[int, ...]:
    from . import Result
    return (r.m, r.n_clusters, r.n_labels) + device_digest([getattr(r, f) for f in Result._fields[3:]])


# ------------------------------------------------------------------- sweep
def sweep(run: Callable[[], object], digest: Callable[[object], tuple], reps: int = 3, order=ORDER,
          candidates=CANDIDATES, log: Optional[Callable[[str], None]] = None) -> dict:
    """Coordinate descent over the knobs. run() makes one complete call (returning when its outputs are
    written) and returns what digest() reads. Returns {"knobs", "default_ms", "tuned_ms", "trials"}."""
    import torch

    def measure(knobs):
        with tuned(knobs):
            d = digest(run())
            times = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                run()
                torch.cuda.synchronize()
                times.append((time.perf_counter() - t0) * 1e3)
        return statistics.median(times), d

    base_ms, base = measure({})
    if log:
        log("built-in choices: %.3f ms" % base_ms)
    best, best_ms = {}, base_ms
    trials = [({}, base_ms)]
    for knob in order:
        for v in candidates[knob]:
            k = dict(best)
            k[knob] = v
            ms, d = measure(k)
            if d != base:
                raise RuntimeError("outputs changed under launch choices %s" % k)
            trials.append((k, ms))
            if log:
                log("%s: %.3f ms" % (k, ms))
            if ms < best_ms * 0.98:
                best, best_ms = k, ms
    # the choice against the built-in one, timed again side by side
    if best:
        again_default, _ = measure({})
        again_best, _ = measure(best)
        if again_best >= again_default:
            best, best_ms, base_ms = {}, again_default, again_default
        else:
            base_ms, best_ms = again_default, again_best
    return {"knobs": best, "default_ms": base_ms, "tuned_ms": best_ms, "trials": trials}


# ------------------------------------------------------------------- files
def read_entries(path: Optional[str] = None) -> Dict[Tuple[int, int, int], dict]:
    path = tune_file(path)
    entries = {}
    if not os.path.exists(path):
        return entries
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            nb, vb, db, ipt, grid, kb, split = (int(x) for x in p[:7])
            names = ("radix_keys_per_thread", "list_grid", "krt_level_bits", "split_min_edges")
            knobs = {k: v for k, v in zip(names, (ipt, grid, kb, split)) if v}
            entry = {"knobs": knobs, "default_ms": float(p[7]) if len(p) > 7 else None,
                     "tuned_ms": float(p[8]) if len(p) > 8 else None}
            entries.setdefault((nb, vb, db), entry)
    return entries


def write_entry(bkt: Tuple[int, int, int], knobs: dict, default_ms: float, tuned_ms: float,
                path: Optional[str] = None) -> str:
    """Adds or replaces the bucket's line."""
    path = tune_file(path)
    entries = read_entries(path)
    entries[tuple(bkt)] = {"knobs": dict(knobs), "default_ms": default_ms, "tuned_ms": tuned_ms}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        f.write(HEADER)
        for (nb, vb, db), e in sorted(entries.items()):
            k = e["knobs"]
            f.write("%d %d %d %d %d %d %d %.3f %.3f\n" % (
                nb, vb, db, k.get("radix_keys_per_thread", 0), k.get("list_grid", 0), k.get("krt_level_bits", 0),
                k.get("split_min_edges", 0), e["default_ms"] or 0.0, e["tuned_ms"] or 0.0))
    os.replace(tmp, path)
    return path


def knobs_for(n: int, V: int, maxdeg: Optional[int] = None, path: Optional[str] = None) -> Optional[dict]:
    """The file's choice for a call of n records over V vertices (the max degree's bucket when given and
    present, else the first line of the (n, V) bucket), or None."""
    nb, vb = bits(n), bits(V)
    entries = read_entries(path)
    if maxdeg is not None and (nb, vb, bits(maxdeg)) in entries:
        return dict(entries[(nb, vb, bits(maxdeg))]["knobs"])
    for (a, b, _), e in entries.items():
        if (a, b) == (nb, vb):
            return dict(e["knobs"])
    return None


# --------------------------------------------------------------- workloads
def max_degree(src, dst, V: int) -> int:
    import torch
    deg = torch.bincount(src.long(), minlength=V) + torch.bincount(dst.long(), minlength=V)
    return int(deg.max().item()) if deg.numel() else 0


def tune_edges(src, dst, t, min_cluster_size: int, num_vertices: int, reps: int = 3,
               path: Optional[str] = None, write: bool = True, log=None) -> dict:
    """Sweeps one graph (device tensors) and records its bucket's choice."""
    import torch
    from . import Outputs, cluster_edges, workspace_bytes
    n = int(t.numel())
    outs = Outputs(n, min_cluster_size, src.device)
    ws = torch.empty(workspace_bytes(n, num_vertices, min_cluster_size), dtype=torch.uint8, device=src.device)
    run = lambda: cluster_edges(src, dst, t, min_cluster_size, num_vertices, outputs=outs, workspace=ws)
    res = sweep(run, result_digest, reps=reps, log=log)
    res["bucket"] = bucket(n, num_vertices, max_degree(src, dst, num_vertices))
    if write:
        res["file"] = write_entry(res["bucket"], res["knobs"], res["default_ms"], res["tuned_ms"], path)
    return res


def tune_batch(src, dst, t, edge_offsets, vertex_offsets, min_cluster_size: int, reps: int = 3,
               path: Optional[str] = None, write: bool = True, log=None) -> dict:
    """Sweeps one batch (device records, host offsets); the bucket is the packed batch's."""
    import numpy as np
    import torch
    from . import batch_outputs, batch_workspace_bytes, cluster_batch
    eo, vo = np.asarray(edge_offsets, np.int64), np.asarray(vertex_offsets, np.int64)
    outs = batch_outputs(eo, min_cluster_size, src.device)
    ws = torch.empty(batch_workspace_bytes(eo, vo, min_cluster_size), dtype=torch.uint8, device=src.device)
    run = lambda: cluster_batch(src, dst, t, eo, vo, min_cluster_size, outputs=outs, workspace=ws)

    def digest(br):
        return (tuple(br.m), tuple(br.n_clusters), tuple(br.row_offsets)) + result_digest(br.result)

    res = sweep(run, digest, reps=reps, log=log)
    V = int(vo[-1])
    gid = torch.repeat_interleave(torch.arange(len(eo) - 1, device=src.device),
                                  torch.from_numpy(np.diff(eo)).to(src.device))
    voff = torch.from_numpy(vo[:-1]).to(src.device)[gid]
    res["bucket"] = bucket(int(eo[-1]), V, max_degree(src.long() + voff, dst.long() + voff, V))
    if write:
        res["file"] = write_entry(res["bucket"], res["knobs"], res["default_ms"], res["tuned_ms"], path)
    return res


def main(argv=None):
    import argparse
    import sys
    import torch
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth
    ap = argparse.ArgumentParser(description="tune the launch choices for one synthetic workload")
    ap.add_argument("--workload", default="mid", choices=["small", "tiny", "mid", "scale", "batch"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None, help="tuning file (default: CE_TUNE_FILE, else the package's)")
    a = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    log = lambda s: print("[autotune] " + s, flush=True)
    to = lambda *xs: [torch.from_numpy(x).to(dev) for x in xs]
    if a.workload == "batch":
        src, dst, t, eoff, voff = synth.batch_workload(4096, seed=3)
        log("batch: %d graphs, %d records" % (len(eoff) - 1, int(eoff[-1])))
        res = tune_batch(*to(src, dst, t), eoff, voff, 5, reps=a.reps, path=a.out, log=log)
    else:
        if a.workload == "small":
            s, d, t = synth.chung_lu_bursts(57_000, 2850, 7)
            V, M = 2850, 5
        else:
            w = {"tiny": synth.plain_tiny, "mid": synth.plain_mid, "scale": synth.plain_scale}[a.workload]()
            s, d, t, V, M = w.src, w.dst, w.t, w.num_vertices, w.min_cluster_size
        log("%s: n=%d V=%d M=%d" % (a.workload, len(t), V, M))
        res = tune_edges(*to(s, d, t), M, V, reps=a.reps, path=a.out, log=log)
    log("bucket %s: %s, %.3f ms -> %.3f ms (%s)" % (res["bucket"], res["knobs"] or "built-in", res["default_ms"],
                                                    res["tuned_ms"], res.get("file")))
    return res


if __name__ == "__main__":
    main()
