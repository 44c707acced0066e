"""Roofline bookkeeping for bench.py: algorithmic bytes per kernel and HBM
traffic from rocprofv3 counter runs.

Algorithmic bytes are the bytes a kernel must move at minimum width, with each
input and output touched once (random gathers count their element size, not
the cache line they pull). ``traffic`` comes from two rocprofv3 ``--pmc`` runs
(FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the same
counter reads for a plain copy kernel of known size.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def dendrogram_levels(m: int, lds_bits: int = 9, level_bits: int = 0) -> int:
    """Global levels of the rank-interval dendrogram for m rows, as the library plans them: level_bits (a
    tuning choice) when given, else the level count of least modelled time (a pass of random accesses per
    level, about 0.4 ns per row, against 20 us per sub-interval and 15 us per level)."""
    if m <= 1:
        return 0
    gbits = (m - 1).bit_length() - lds_bits
    if gbits <= 0:
        return 0
    if level_bits:
        return -(-gbits // level_bits)
    best, kbest = None, gbits
    for nlev in range(1, gbits + 1):
        hi, lo, nhi = -(-gbits // nlev), gbits // nlev, gbits % nlev
        if hi > 12:
            continue
        steps = nhi * 2 ** hi + (nlev - nhi) * 2 ** lo
        t = nlev * (0.4e-9 * m + 15e-6) + steps * 20e-6
        if best is None or t < best:
            best, kbest = t, hi
    return -(-gbits // kbest)


# kernel -> (unit, algorithmic bytes per unit, units per step as a function of the run)
def algorithmic_bytes_per_step(kernel: str, n: int, m: int, level_bits: int = 0) -> tuple:
    """(unit description, bytes per unit, units per step) for a kernel of the pipeline."""
    if kernel == "k_krt_accum":
        # per row and global level: hooked root id (4), its size (4), the parent of that root (4),
        # the row id it offers (4); the per-root atomics are combined in LDS
        return ("MSF row x global level", 16, dendrogram_levels(m, level_bits=level_bits) * m)
    if kernel == "k_krt_union":
        # per row and global level: two labels read (8), the two root entries read (2 x 16), the new labels
        # and sizes written (16), one 8-byte CAS (8), the hooked root written (4)
        return ("MSF row x global level", 68, dendrogram_levels(m, level_bits=level_bits) * m)
    if kernel == "k_krt_relabel":
        # per row and level: two labels (8) read and rewritten (8), two sizes rewritten (8), two roots
        # written (8), two root entries read (2 x 12)
        return ("MSF row x global level", 56, dendrogram_levels(m, level_bits=level_bits) * m)
    if kernel == "k_krt_lds":
        # per row: two labels and two sizes read (16), two children and the size written (12)
        return ("MSF row", 28, m)
    if kernel == "k_rs_scatter":
        return ("element x pass (u64 key + u64 value)", 32, None)
    raise KeyError(kernel)


def source_hash(files=None) -> str:
    """Hash of every kernel source under csrc/ (sorted by name)."""
    if files is None:
        files = sorted(os.path.relpath(f, HERE) for f in glob.glob(os.path.join(HERE, "csrc", "*"))
                       if f.endswith((".hip", ".h")))
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _counter_rows(d):
    paths = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    rows = []
    for p in paths:
        with open(p) as fh:
            rows.extend(csv.DictReader(fh))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def _is_library(name: str) -> bool:
    return name.startswith("ce::") or name.startswith("void ce::")


def _calibration_kib(rows):
    """Counter value of the calibration copy: the largest runtime copy issued before the first library
    kernel (the pipeline's own device copies come later and can be larger)."""
    first = next((i for i, r in enumerate(rows) if _is_library(r["Kernel_Name"])), len(rows))
    copies = [float(r["Counter_Value"]) for r in rows[:first] if "copyBuffer" in r["Kernel_Name"]]
    return max(copies) if copies else None


def summarize_pmc(fetch_dir: str, write_dir: str, kernel: str, copy_bytes: int) -> dict:
    """Per-dispatch HBM traffic of `kernel`, calibrated against the largest copy dispatch."""
    out = {"kernel": kernel, "copy_bytes": copy_bytes}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter_rows(d) if r["Counter_Name"] == name]
        ref_kib = _calibration_kib(rows)
        factor = (copy_bytes / 1024.0) / ref_kib if ref_kib else None
        mine = [float(r["Counter_Value"]) for r in rows if kernel in r["Kernel_Name"]]
        out[name] = {"dispatches": len(mine), "avg_kib": (sum(mine) / len(mine)) if mine else None,
                     "copy_kib": ref_kib, "scale": factor}
    f, w = out["FETCH_SIZE"], out["WRITE_SIZE"]
    if f["avg_kib"] is not None and w["avg_kib"] is not None and f["scale"] and w["scale"]:
        out["traffic_bytes_per_launch"] = 1024.0 * (f["avg_kib"] * f["scale"] + w["avg_kib"] * w["scale"])
    else:
        out["traffic_bytes_per_launch"] = None
    out["source_hash"] = source_hash()
    return out


def _is_host_side(name: str) -> bool:
    # torch's own kernels (input fills and copies made by the benchmark harness)
    return "at::native" in name


def summarize_pipeline_pmc(fetch_dir: str, write_dir: str, copy_bytes: int, steps: int = 1) -> dict:
    """HBM traffic of the whole pipeline per step: every dispatch from the first to the last library
    kernel (library kernels and the runtime copies they issue), calibrated like summarize_pmc."""
    out = {"scope": "pipeline", "copy_bytes": copy_bytes, "steps": steps}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter_rows(d) if r["Counter_Name"] == name]
        ref_kib = _calibration_kib(rows)
        factor = (copy_bytes / 1024.0) / ref_kib if ref_kib else None
        lib = [i for i, r in enumerate(rows) if _is_library(r["Kernel_Name"])]
        span = rows[lib[0]:lib[-1] + 1] if lib else []
        mine = [float(r["Counter_Value"]) for r in span if not _is_host_side(r["Kernel_Name"])]
        out[name] = {"dispatches": len(mine), "total_kib": sum(mine), "copy_kib": ref_kib, "scale": factor}
    f, w = out["FETCH_SIZE"], out["WRITE_SIZE"]
    if f["scale"] and w["scale"]:
        out["traffic_bytes_per_step"] = 1024.0 * (f["total_kib"] * f["scale"] + w["total_kib"] * w["scale"]) / steps
    else:
        out["traffic_bytes_per_step"] = None
    out["source_hash"] = source_hash()
    return out


def load_pipeline_traffic(path: str) -> float | None:
    """Pipeline traffic per step from a committed summary, or None if the kernels changed since."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        text = fh.read()
    start = text.find("```json")
    if start < 0:
        return None
    blob = json.loads(text[start + 7:text.find("```", start + 7)])
    if blob.get("scope") != "pipeline" or blob.get("source_hash") != source_hash():
        return None
    return blob.get("traffic_bytes_per_step")


# algorithmic bytes per temporal edge of the whole path, by stage: each intermediate written once and read
# once at minimal width (input 16, incidence 48, skeleton 64, MSF rows 32, dendrogram rows 20, per-record
# outputs 12, labels 4)
STAGE_BYTES = {"input": 16, "incidence": 48, "skeleton": 64, "msf": 32, "dendrogram": 20, "condensed": 12,
               "labels": 4}
PATH_BYTES_PER_EDGE = sum(STAGE_BYTES.values())


def load_traffic(kernel: str, path: str) -> float | None:
    """Traffic per launch from a committed PMC summary, or None if the kernels changed since."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        text = fh.read()
    start = text.find("```json")
    if start < 0:
        return None
    blob = json.loads(text[start + 7:text.find("```", start + 7)])
    if blob.get("kernel") != kernel or blob.get("source_hash") != source_hash():
        return None
    return blob.get("traffic_bytes_per_launch")


if __name__ == "__main__":
    import sys
    fetch_dir, write_dir, kernel, copy_bytes = sys.argv[1], sys.argv[2], sys.argv[3], int(sys.argv[4])
    if kernel == "pipeline":
        steps = int(sys.argv[5]) if len(sys.argv) > 5 else 1
        print(json.dumps(summarize_pipeline_pmc(fetch_dir, write_dir, copy_bytes, steps), indent=1))
    else:
        print(json.dumps(summarize_pmc(fetch_dir, write_dir, kernel, copy_bytes), indent=1))
