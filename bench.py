#!/usr/bin/env python3
"""Benchmark: temporal edges clustered per second on one MI355X.

One step = one full clustering of the workload through the C ABI (group and
sort by vertex and time, path skeleton, Boruvka MSF, sorted MSF, exact
dendrogram, condensed tree, stability, excess of mass, labels), with the input
records already resident in HBM and the workspace and outputs preallocated.
Prints one JSON line.

Default workload (N=1): one GPU's share at scale -- R-MAT scale 26 (2^26
vertices), 2^30 records, a planted hub of degree about 1e7, per-pair Hawkes
timestamps over 365 days, min_cluster_size 25, seed 2. The 5e7-record R-MAT
workload is timed beside it, then the 4096-graph batch and the serving stream
(each against one call per graph or request, with every result compared), and
the CPU oracle on a prefix of the same records, compared with the GPU on that
prefix.
"""
import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "temporal edges clustered/sec (bit-exact) + % HBM roofline; batched vs single"
FIELDS = ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster", "pt_lambda",
          "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected", "labels")
T0 = time.perf_counter()


def log(msg):
    print("[bench %6.1fs] %s" % (time.perf_counter() - T0, msg), file=sys.stderr, flush=True)


WORKLOADS = {
    "tiny": ("chung-lu-bursts-tiny", "plain_tiny", {"n_edges": 200_000, "n_vertices": 10_000, "min_cluster_size": 5,
                                                      "seed": 0, "timestamps": "poisson bursts, 30 days"}),
    "mid": ("rmat-hawkes-mid", "plain_mid", {"n_edges": 50_000_000, "n_vertices": 1 << 20, "min_cluster_size": 10,
                                             "seed": 1, "timestamps": "per-pair hawkes, 90 days"}),
    "scale": ("rmat-hawkes-scale", "plain_scale", {"n_edges": 1 << 30, "n_vertices": 1 << 26,
                                                   "min_cluster_size": 25, "seed": 2,
                                                   "timestamps": "per-pair hawkes, 365 days, planted 1e7 hub"}),
}


def make_workload(name):
    import synth
    label, fn, cfg = WORKLOADS[name]
    return getattr(synth, fn)(), dict({"workload": label}, **cfg)


# ----------------------------------------------------------------------------------------------- CPU oracle
def cpu_oracle_single(w, sample, causal=False, thresholds=None):
    """The CPU oracle (plain single-threaded C, skeleton tier) on the first `sample` records; returns the timing
    record and the oracle's result for the parity check against the GPU on the same records."""
    import oracle
    ns = min(sample, w.n)
    t0 = time.perf_counter()
    if thresholds:
        r = oracle.cluster_discrete(w.src[:ns], w.dst[:ns], w.t[:ns], w.min_cluster_size, thresholds,
                                    w.num_vertices, tier=1, causal=causal)[0]
    else:
        r = oracle.cluster(w.src[:ns], w.dst[:ns], w.t[:ns], w.min_cluster_size, w.num_vertices, tier=1,
                           causal=causal)
    dt = time.perf_counter() - t0
    assert r.status == 0
    rec = {"value": ns / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
           "sample": "first %d of %d records of the same workload (%s oracle%s, one host thread, %.1f s)"
                     % (ns, w.n, "Alg. 2 window" if causal else "path-skeleton",
                        ", discrete dendrogram with %d thresholds" % len(thresholds) if thresholds else "", dt)}
    return rec, r, ns


_CHILD = r"""
import sys, time, numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
d = np.load(sys.argv[2])
t0 = time.perf_counter()
r = oracle.cluster(d["src"], d["dst"], d["t"], int(d["M"]), int(d["V"]), tier=1)
assert r.status == 0
print(time.perf_counter() - t0)
"""


def cpu_oracle_all_cores(w, sample):
    """The same plain oracle on every host core at once: one process per core, each clustering its own copy
    of the first `sample` records (independent jobs; the oracle itself stays single-threaded). Runs before
    this process touches the GPU."""
    import numpy as np
    procs = min(os.cpu_count() or 1, 16)
    ns = min(sample, w.n)
    path = "/dev/shm/ce_bench_prefix_%d.npz" % os.getpid()
    np.savez(path, src=w.src[:ns], dst=w.dst[:ns], t=w.t[:ns], M=w.min_cluster_size, V=w.num_vertices)
    try:
        t0 = time.perf_counter()
        ps = [subprocess.Popen([sys.executable, "-c", _CHILD, ROOT, path], stdout=subprocess.PIPE, text=True)
              for _ in range(procs)]
        outs = [p.communicate()[0] for p in ps]
        wall = time.perf_counter() - t0
        if any(p.returncode != 0 for p in ps):
            return {"skipped": "an oracle process failed"}
        each = [float(o.strip().splitlines()[-1]) for o in outs]
    finally:
        os.unlink(path)
    return {"value": procs * ns / wall, "unit": "edges/s", "cores": procs, "kind": "oracle",
            "sample": "%d processes at once, each the plain single-threaded oracle on its own copy of the first %d "
                      "records (%.1f s wall; per process %.1f-%.1f s)" % (procs, ns, wall, min(each), max(each))}


def compare_numpy(got, ref, fields=FIELDS):
    """Names of the fields where the GPU result (to_numpy dict) differs from the oracle's."""
    import numpy as np
    bad = [f for f in fields if not np.array_equal(got[f], getattr(ref, f))]
    for f in ("m", "n_clusters", "n_labels"):
        if int(got[f]) != int(getattr(ref, f)):
            bad.append(f)
    return bad


# ---------------------------------------------------------------------------------------------- roofline
def roofline_line(ce, profiling, kernel, kms, kcnt, w, m, steps, tag, level_bits=0):
    """Roofline of the dominant kernel against the path's algorithmic bytes: the dendrogram stage's share of
    the per-edge model (bytes of the dendrogram rows per MSF row) spread over the kernel's launches, divided by
    its average launch time. The kernel's own access model and the counter traffic are given beside it."""
    per_row = profiling.STAGE_BYTES["dendrogram"]
    per_launch = per_row * m * steps / kcnt
    avg_s = kms / kcnt * 1e-3
    achieved = per_launch / avg_s / 1e9
    unit, model_per_unit, model_units = profiling.algorithmic_bytes_per_step(kernel, w.n, m, level_bits)
    model_per_launch = model_per_unit * model_units * steps / kcnt
    traffic = profiling.load_traffic(kernel, os.path.join(ROOT, "profiles", "%s_%s_pmc.md" % (kernel, tag)))
    return {"bound": "hbm", "achieved": achieved, "peak": profiling.HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / profiling.HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
            "algorithmic_bytes_per_launch": per_launch, "launches": kcnt, "avg_launch_us": 1e6 * avg_s,
            "unit_of_work": "MSF row (dendrogram rows: %d B per row, all of the stage given to this kernel)" % per_row,
            "amplification": traffic / per_launch if traffic else None,
            "kernel_model": {"unit": unit, "bytes_per_unit": model_per_unit, "bytes_per_launch": model_per_launch,
                             "achieved": model_per_launch / avg_s / 1e9,
                             "frac": model_per_launch / avg_s / 1e9 / profiling.HBM_PEAK_GBS,
                             "amplification": traffic / model_per_launch if traffic else None}}


# --------------------------------------------------------------------------------------------- workloads
class tuning_file:
    """CE_TUNE_FILE set to path (None: unset) for the block, for calls the library resolves itself."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        self.prev = os.environ.get("CE_TUNE_FILE")
        if self.path:
            os.environ["CE_TUNE_FILE"] = self.path
        else:
            os.environ.pop("CE_TUNE_FILE", None)

    def __exit__(self, *exc):
        if self.prev is None:
            os.environ.pop("CE_TUNE_FILE", None)
        else:
            os.environ["CE_TUNE_FILE"] = self.prev


def tuned_knobs(ce, n, V):
    """The autotuner's choice for this bucket from the package's tuning file (None: built-in choices)."""
    from paper_2311_10337_amd import autotune
    return autotune.knobs_for(n, V)


def time_single_graph(ce, w, dev, steps, warmup, causal=False, thr=None, roofline_kernel=None, knobs=None,
                      default_steps=0, timing_steps=0):
    """Times `steps` calls under the launch choices `knobs` (None: built-in), with no instrumentation; then,
    with roofline_kernel, `timing_steps` more calls in which that kernel's launches are timed by events in
    their own dispatches; with default_steps, then that many calls with the built-in choices, whose outputs
    must be the same. Returns (result, seconds, (kernel ms, kernel launches, steps they cover), device
    buffers, tuning record or None, per-step milliseconds of the timed calls)."""
    import torch
    from paper_2311_10337_amd import autotune
    src = torch.from_numpy(w.src).to(dev)
    dst = torch.from_numpy(w.dst).to(dev)
    tt = torch.from_numpy(w.t).to(dev)
    M, V = w.min_cluster_size, w.num_vertices
    outs = ce.Outputs(w.n, M, dev)
    ws = torch.empty(ce.workspace_bytes(w.n, V, M, thresholds=thr), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step():
        return ce.cluster_edges(src, dst, tt, M, V, outputs=outs, workspace=ws, causal=causal, thresholds=thr)

    r = None
    with ce.tuned(knobs):
        for i in range(warmup):
            r = step()
            log("warmup %d done: m=%d clusters=%d labels=%d" % (i, r.m, r.n_clusters, r.n_labels))
        torch.cuda.synchronize()
        stamps = []
        t0 = time.perf_counter()
        for i in range(steps):
            r = step()  # returns when the call's results are written
            stamps.append(time.perf_counter())
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        step_ms = [1e3 * (b - a) for a, b in zip([t0] + stamps[:-1], stamps)]
        kms, kcnt, ksteps = 0.0, 0, 0
        if roofline_kernel and timing_steps:
            ce.timing_enable(roofline_kernel)
            for i in range(timing_steps):
                step()
            torch.cuda.synchronize()
            kms, kcnt = ce.timing_read()
            ce.timing_enable(None)
            ksteps = timing_steps
    log("timed %d steps in %.3f s (%.1f ms per step, median %.1f)%s"
        % (steps, el, 1e3 * el / steps, sorted(step_ms)[len(step_ms) // 2],
           ", launch choices %s" % knobs if knobs else ""))
    tune = None
    if knobs and default_steps:
        d_tuned = autotune.result_digest(r)
        r0 = step()  # built-in choices: warm-up, and the outputs to compare
        same = autotune.result_digest(r0) == d_tuned
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(default_steps):
            r = step()
        torch.cuda.synchronize()
        el0 = time.perf_counter() - t0
        tune = {"knobs": knobs, "tuned_ms_per_step": 1e3 * el / steps, "default_ms_per_step": 1e3 * el0 / default_steps,
                "default_steps": default_steps, "speedup": (el0 / default_steps) / (el / steps),
                "outputs_identical": same, "resolved": ce.resolve_tuning(w.n, V, knobs)}
        log("built-in choices: %.1f ms per step, outputs %s" % (1e3 * el0 / default_steps,
                                                               "identical" if same else "DIFFER"))
    elif not knobs:
        tune = {"knobs": {}, "note": "no tuning-file entry for this bucket: built-in choices",
                "resolved": ce.resolve_tuning(w.n, V)}
    del ws
    return r, el, (kms, kcnt, ksteps), (src, dst, tt, outs), tune, step_ms


def bench_small_calls(ce, dev, n=57_000, calls=50):
    """One call on a median batch graph (57k records of the batch recipe's generator): synchronous,
    asynchronous (enqueue, then one wait) and a captured HIP graph replayed; with the launch count."""
    import torch
    import synth
    V = max(2, n // 20)
    s, d, t = synth.chung_lu_bursts(n, V, 7)
    ins = [torch.from_numpy(x).to(dev) for x in (s, d, t)]
    M = 5
    outs = ce.Outputs(n, M, dev)
    ws = torch.empty(ce.workspace_bytes(n, V, M), dtype=torch.uint8, device=dev)
    hdr = torch.zeros(ce.hdr_words(1), dtype=torch.int64, device=dev)
    for _ in range(5):
        ce.cluster_edges(*ins, M, V, outputs=outs, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        ce.cluster_edges(*ins, M, V, outputs=outs, workspace=ws)
    sync_ms = (time.perf_counter() - t0) / calls * 1e3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        ce.cluster_edges_async(*ins, M, V, outs, ws, hdr, time_bits=24)
    enq_ms = (time.perf_counter() - t0) / calls * 1e3
    torch.cuda.synchronize()
    async_ms = (time.perf_counter() - t0) / calls * 1e3
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            ce.cluster_edges_async(*ins, M, V, outs, ws, hdr, time_bits=24, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        g.replay()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) / calls * 1e3
    ce.timing_enable("k_")
    ce.cluster_edges(*ins, M, V, outputs=outs, workspace=ws)
    _, launches = ce.timing_read()
    ce.timing_enable(None)
    log("one %d-record call: sync %.3f ms, async %.3f ms (enqueue %.3f), graph replay %.3f ms, %d launches"
        % (n, sync_ms, async_ms, enq_ms, graph_ms, launches))
    return {"n_edges": n, "n_vertices": V, "min_cluster_size": M, "calls": calls, "sync_ms": sync_ms,
            "async_ms": async_ms, "enqueue_ms": enq_ms, "graph_replay_ms": graph_ms, "launches": launches}


def bench_level_components(ce, r, n, thr, calls=3):
    """Alg. 5 the paper's way, one connected-components pass per threshold (ce_level_components over the
    forest the timed steps produced), next to the discrete dendrogram cut from the exact one in those steps."""
    import torch
    need = 4 * len(thr) * n
    free, _ = torch.cuda.mem_get_info(r.msf_tail.device)
    if need > free:
        log("per-level components skipped: %d levels of %d labels need %.1f GiB, %.1f GiB free"
            % (len(thr), n, need / 2 ** 30, free / 2 ** 30))
        return {"skipped": "labels of %d levels need %d bytes, %d free" % (len(thr), need, free)}
    labels = torch.empty(len(thr) * n, dtype=torch.int32, device=r.msf_tail.device)
    ce.level_components(r.msf_tail, r.msf_head, r.msf_w, n, thr, labels=labels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        ce.level_components(r.msf_tail, r.msf_head, r.msf_w, n, thr, labels=labels)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / calls
    log("discrete dendrogram by per-level components: %.1f ms for %d levels" % (ms, len(thr)))
    return {"ms_per_call": ms, "levels": len(thr), "rows": r.m, "records": n,
            "note": "ce_level_components on the forest of the timed steps: one components pass per threshold "
                    "(Alg. 5 as the paper computes it); the timed steps cut the same discrete dendrogram from "
                    "the exact one"}


def bench_hyper(dev, steps, warmup):
    """Dynamic hypergraph (Sec. 5.3): the 2e7-hyperedge multi-recipient workload through
    ce_cluster_hyperedges, inputs resident in HBM, workspace and outputs preallocated."""
    import torch
    import synth
    import paper_2311_10337_amd as ce
    t0 = time.perf_counter()
    w = synth.hyper_mid()
    log("hypergraph workload: %d hyperedges, %d memberships (%.1f s)" % (w.n, w.nnz, time.perf_counter() - t0))
    mem = torch.from_numpy(w.members).to(dev)
    off = torch.from_numpy(w.offsets).to(dev)
    tt = torch.from_numpy(w.t).to(dev)
    M, V = w.min_cluster_size, w.num_vertices
    outs = ce.Outputs(w.n, M, dev)
    ws = torch.empty(ce.hyper_workspace_bytes(w.n, w.nnz, V, M), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step():
        return ce.cluster_hyperedges(mem, off, tt, M, V, outputs=outs, workspace=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    log("hypergraph: %.1f ms per step" % (1e3 * el))
    out = {"workload": "hyper-bursts-mid", "n_hyperedges": w.n, "memberships": w.nnz, "n_vertices": V,
           "min_cluster_size": M, "seed": 6,
           "recipe": "Chung-Lu 2.1 sender + recipients, recipients per message lognormal median 2 sigma 1 "
                     "clipped [1, 64], Poisson bursts over 90 days",
           "hyperedges_per_s": w.n / el, "memberships_per_s": w.nnz / el, "ms_per_step": 1e3 * el, "steps": steps,
           "m_msf": r.m, "n_clusters": r.n_clusters, "n_labels": r.n_labels}
    del mem, off, tt, outs, ws
    torch.cuda.empty_cache()
    return out


def equal_fields(a, b, counts):
    """Fields (of two Outputs) that differ on the leading counts: rows, records, cluster rows."""
    import torch
    rows, recs, cls = counts
    bad = []
    for f in FIELDS:
        k = recs if f in ("pt_cluster", "pt_lambda", "labels") else cls if f.startswith("cl_") else rows
        if not torch.equal(a.t[f][:k], b.t[f][:k]):
            bad.append(f)
    return bad


def bench_batched(dev, steps, warmup, tuning=True):
    """The 4096-graph batch in one call vs one call per graph, same GPU and inputs. Every one-graph call
    writes into its graph's region of a second output buffer laid out like the batch, and the two buffers
    are compared whole."""
    import numpy as np
    import torch
    import synth
    import paper_2311_10337_amd as ce
    G, M = 4096, 5
    t0 = time.perf_counter()
    src, dst, t, eoff, voff = synth.batch_workload(G, seed=3)
    n = int(eoff[-1])
    log("batch workload: %d graphs, %d records (%.1f s)" % (G, n, time.perf_counter() - t0))
    s_d = torch.from_numpy(src).to(dev)
    d_d = torch.from_numpy(dst).to(dev)
    t_d = torch.from_numpy(t).to(dev)
    outs = ce.batch_outputs(eoff, M, dev)
    ws = torch.empty(ce.batch_workspace_bytes(eoff, voff, M), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def batch_step():
        return ce.cluster_batch(s_d, d_d, t_d, eoff, voff, M, outputs=outs, workspace=ws)

    from paper_2311_10337_amd import autotune
    knobs = autotune.knobs_for(n, int(voff[-1])) if tuning else None
    with ce.tuned(knobs):
        for _ in range(warmup):
            batch_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            br = batch_step()
        torch.cuda.synchronize()
        el_b = (time.perf_counter() - t0) / steps
    log("batched: %.1f ms per batch%s" % (1e3 * el_b, ", launch choices %s" % knobs if knobs else ""))
    tune = None
    if knobs:
        d_tuned = autotune.result_digest(br.result)
        same = autotune.result_digest(batch_step().result) == d_tuned
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            batch_step()
        torch.cuda.synchronize()
        el0 = (time.perf_counter() - t0) / steps
        tune = {"knobs": knobs, "tuned_ms": 1e3 * el_b, "default_ms": 1e3 * el0, "speedup": el0 / el_b,
                "outputs_identical": same}
        log("batched, built-in choices: %.1f ms per batch, outputs %s" % (1e3 * el0, "identical" if same else "DIFFER"))
    del ws
    torch.cuda.empty_cache()
    captured = time_captured_batch(ce, (s_d, d_d, t_d), eoff, voff, M, steps, dev, knobs,
                                   autotune.result_digest(br.result), int(t.max() - t.min()).bit_length())
    ng = np.diff(eoff)
    vg = np.diff(voff)
    nmax = int(ng.max())
    roff, coff = br.row_offsets, br.cluster_offsets
    single = ce.Outputs(n, M, dev, clusters=int(coff[-1]) + ce.max_clusters(nmax, M), rows=n + nmax)
    regions = [single.region(int(roff[g]), int(eoff[g]), int(coff[g]), int(ng[g]), M) for g in range(G)]
    sws = torch.empty(ce.workspace_bytes(nmax, int(vg.max()), M), dtype=torch.uint8, device=dev)

    def one(g):
        a, b = int(eoff[g]), int(eoff[g + 1])
        return ce.cluster_edges(s_d[a:b], d_d[a:b], t_d[a:b], M, int(vg[g]), outputs=regions[g], workspace=sws)

    # one-graph calls take their own buckets' choices from the tuning file (the library reads it)
    with tuning_file(autotune.PACKAGE_FILE if tuning else None):
        for g in range(min(G, 64)):
            one(g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        counts = [one(g) for g in range(G)]
        torch.cuda.synchronize()
        el_s = time.perf_counter() - t0
    log("one graph per call: %.1f ms for the %d graphs" % (1e3 * el_s, G))
    same_counts = all(c.m == br.m[g] and c.n_clusters == br.n_clusters[g] and c.n_labels == br.n_labels[g]
                      for g, c in enumerate(counts))
    bad = equal_fields(outs, single, (int(roff[-1]), n, int(coff[-1])))
    equal = same_counts and not bad
    log("batch vs one call per graph: %s" % ("all %d graphs equal" % G if equal else "DIFFER in %s" % bad))
    out = {"workload": "chung-lu-bursts-batch-4096", "graphs": G, "n_edges": n, "min_cluster_size": M, "seed": 3,
           "sizes": "lognormal median 20000 sigma 1.5 clipped [500, 2e6]; V_g = n_g/20",
           "batched_edges_per_s": n / el_b, "batched_ms": 1e3 * el_b, "batched_steps": steps,
           "single_edges_per_s": n / el_s, "single_ms": 1e3 * el_s,
           "ratio": el_s / el_b, "n_clusters": int(br.n_clusters.sum()), "n_labels": int(br.n_labels.sum()),
           "equal_to_single_calls": equal, "graphs_compared": G,
           "captured": dict(captured, edges_per_s=n / (1e-3 * captured["ms"]),
                            ratio=el_s / (1e-3 * captured["ms"]))}
    if tune is not None:
        out["tuning"] = tune
    del s_d, d_d, t_d, outs, single, regions, sws
    torch.cuda.empty_cache()
    return out


def time_captured_batch(ce, ins, eoff, voff, M, steps, dev, knobs, want, time_bits):
    """The batch as one HIP graph: the enqueue-only call (device offsets, counts in a device header) captured
    once under the same launch choices, then replayed; its outputs are compared with the synchronous call's
    (digest `want`)."""
    import numpy as np
    import torch
    from paper_2311_10337_amd import autotune
    G, n = len(eoff) - 1, int(eoff[-1])
    eo = torch.from_numpy(np.ascontiguousarray(eoff, dtype=np.int64)).to(dev)
    vo = torch.from_numpy(np.ascontiguousarray(voff, dtype=np.int64)).to(dev)
    outs = ce.batch_outputs(eoff, M, dev)
    ws = torch.empty(ce.batch_workspace_bytes_for(n, G, M), dtype=torch.uint8, device=dev)
    hdr = torch.zeros(ce.hdr_words(G), dtype=torch.int64, device=dev)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with ce.tuned(knobs), torch.cuda.stream(side), torch.cuda.graph(graph, stream=side):
        ce.cluster_batch_async(*ins, eo, vo, int(voff[-1]), M, outs, ws, hdr, time_bits=max(1, time_bits),
                               stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    cap_s = time.perf_counter() - t0
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    same = autotune.result_digest(ce.async_batch_result(outs, eoff, hdr).result) == want
    log("batched, captured HIP graph: %.1f ms per replay (capture %.1f ms), outputs %s"
        % (1e3 * el, 1e3 * cap_s, "identical" if same else "DIFFER"))
    del graph, outs, ws, hdr, eo, vo
    torch.cuda.empty_cache()
    return {"ms": 1e3 * el, "replays": steps, "capture_ms": 1e3 * cap_s, "outputs_identical": same,
            "call": "ce_cluster_batch_async captured once in a HIP graph and replayed"}


class Digest:
    """Two random linear 64-bit hashes of every output field of a result (on the GPU): results whose digests
    agree are equal except with probability about 2^-128 per comparison."""

    def __init__(self, dev, length):
        import torch
        g = torch.Generator(device="cpu").manual_seed(12345)
        self.c = torch.randint(-(2 ** 62), 2 ** 62, (2, length), generator=g, dtype=torch.int64).to(dev)

    def __call__(self, res, n):
        import torch
        parts = []
        groups = {}
        for f in FIELDS:  # fields of one length are stacked and digested together
            x = getattr(res, f)
            groups.setdefault(x.numel(), []).append(x.to(torch.int64))
        for k, xs in groups.items():
            X = torch.stack(xs)
            parts.append((X * self.c[0, :k]).sum(dim=1))
            parts.append((X * self.c[1, :k]).sum(dim=1))
        return torch.cat(parts).cpu().tolist() + [res.m, res.n_clusters, res.n_labels]


class OutputPool:
    """Output buffers for served requests by size class (capacity 2^c records), made on demand up to a byte
    cap and recycled after each request is polled and digested."""

    def __init__(self, ce, M, dev, cap_bytes, per_record=72):
        self.ce, self.M, self.dev, self.cap, self.per = ce, M, dev, cap_bytes, per_record
        self.free, self.bytes, self.stalls = {}, 0, 0

    def take(self, n, idle):
        c = max(10, (max(n, 1) - 1).bit_length())
        for k in sorted(self.free):
            if k >= c and self.free[k]:
                return self.free[k].pop()
        need = (1 << c) * self.per
        while self.bytes + need > self.cap:  # make room by dropping cached buffers, largest first
            ks = [k for k in self.free if self.free[k]]
            if not ks:
                break
            k = max(ks)
            self.free[k].pop()
            self.bytes -= (1 << k) * self.per
        if self.bytes + need > self.cap and not idle:
            self.stalls += 1
            return None
        self.bytes += need
        o = self.ce.Outputs(1 << c, self.M, self.dev)
        o.size_class = c
        return o

    def give(self, o):
        self.free.setdefault(o.size_class, []).append(o)


def bench_serving(dev, count, workers=3, budget_gib=64, inflight=512, out_gib=24):
    """Open-loop replay of the request stream (Poisson arrivals at 200/s) through the continuous-batching
    server, then the same requests submitted all at once, against one call per request. Each request's
    outputs are digested on the GPU when it is polled and its buffer goes back to a pool; the one-call-per-
    request results are digested the same way and every request's digests are compared."""
    import numpy as np
    import torch
    import synth
    import paper_2311_10337_amd as ce
    from concurrent.futures import ThreadPoolExecutor
    M = 10
    sizes = synth.request_sizes(20000, seed=4)[:count]
    arr = synth.request_arrivals(20000, seed=4)[:count]
    arr = arr - arr[0]
    # the stream's records live in pinned host memory, as a server's receive buffers would, so submissions
    # copy to the GPU by DMA instead of staging pageable pages
    total = int(sizes.sum())
    offs = np.zeros(count + 1, np.int64)
    np.cumsum(sizes, out=offs[1:])
    t0 = time.perf_counter()
    pinned = [torch.empty(total, dtype=dt, pin_memory=True) for dt in (torch.int32, torch.int32, torch.int64)]
    hs, hd, ht = (x.numpy() for x in pinned)
    log("pinned host buffers for the stream: %.1f GB (%.1f s)" % (total * 16 / 1e9, time.perf_counter() - t0))
    t0 = time.perf_counter()

    def gen(r):
        a, b = int(offs[r]), int(offs[r + 1])
        return synth.request_graph(r, int(sizes[r]), seed=4, out=(hs[a:b], hd[a:b], ht[a:b]))

    with ThreadPoolExecutor(max_workers=16) as ex:
        reqs = list(ex.map(gen, range(count)))
    log("serving workload: %d requests, %d records (%.1f s)" % (count, total, time.perf_counter() - t0))
    nmax = int(sizes.max())
    pool = OutputPool(ce, M, dev, out_gib << 30)
    digest = Digest(dev, nmax)
    srv = ce.Server(budget_gib << 30, workers=workers, max_inflight=inflight)
    served = [None] * count

    def replay(arrivals, keep):
        lat = np.zeros(count)
        pending = {}
        k = 0
        first_sub, last_done = None, 0.0
        start = time.perf_counter()
        while k < count or pending:
            progressed = False
            now = time.perf_counter() - start
            while k < count and now >= arrivals[k] and len(pending) < inflight:
                s, d, t, V = reqs[k]
                buf = pool.take(len(s), not pending)
                if buf is None:
                    break
                sub = time.perf_counter() - start
                try:
                    tk = srv.submit(s, d, t, M, V, outputs=buf)
                except ce.ServerBusy:
                    pool.give(buf)
                    break
                first_sub = sub if first_sub is None else first_sub
                pending[tk] = (k, sub, buf)
                k += 1
                progressed = True
                now = time.perf_counter() - start
            for tk in list(pending):
                r = srv.poll(tk)
                if r is not None:
                    kk, sub, buf = pending.pop(tk)
                    if r.status != ce.CE_OK:
                        raise RuntimeError("request %d failed: %s" % (kk, r.error))
                    lat[kk] = (sub - arrivals[kk]) + r.latency_s
                    last_done = max(last_done, sub + r.latency_s)
                    if keep:
                        served[kk] = digest(r.result, len(reqs[kk][0]))
                    pool.give(buf)
                    progressed = True
            if not progressed:
                time.sleep(0.0002)
        return lat, last_done - arrivals[0]

    replay(np.zeros(count), True)  # warm-up pass, everything at once; digests of every served result
    log("served results digested")
    st0 = srv.stats()
    lat, wall_open = replay(arr, False)
    st1 = srv.stats()
    log("open-loop replay done")
    stalls0 = pool.stalls
    _, wall_sat = replay(np.zeros(count), False)
    st2 = srv.stats()
    stalls_sat = pool.stalls - stalls0
    srv.close()
    del pool
    torch.cuda.empty_cache()
    # one call per request, inputs already on the GPU: timed one after another on every tenth request (the
    # rate is scaled by records), then every request once more, four host threads with a stream each, its
    # outputs digested and compared with the served ones
    dins = [tuple(torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in r[:3]) + (r[3],) for r in reqs]
    vmax = max(r[3] for r in reqs)
    lanes = 4
    souts = [ce.Outputs(nmax, M, dev) for _ in range(lanes)]
    sws = [torch.empty(ce.workspace_bytes(nmax, vmax, M), dtype=torch.uint8, device=dev) for _ in range(lanes)]
    sample = list(range(0, count, 10))
    for k in sample[:16]:
        s, d, t, V = dins[k]
        ce.cluster_edges(s, d, t, M, V, outputs=souts[0], workspace=sws[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in sample:
        s, d, t, V = dins[k]
        ce.cluster_edges(s, d, t, M, V, outputs=souts[0], workspace=sws[0])
    torch.cuda.synchronize()
    wall_sample = time.perf_counter() - t0
    rec_sample = int(sum(int(sizes[k]) for k in sample))
    wall_single = wall_sample * total / rec_sample
    log("one call per request: %.2f s for %d of the %d requests (%d records), %.2f s scaled to all"
        % (wall_sample, len(sample), count, rec_sample, wall_single))
    streams = [torch.cuda.Stream(device=dev) for _ in range(lanes)]

    def check(lane):
        bad = []
        with torch.cuda.stream(streams[lane]):
            for k in range(lane, count, lanes):
                s, d, t, V = dins[k]
                r = ce.cluster_edges(s, d, t, M, V, outputs=souts[lane], workspace=sws[lane], stream=streams[lane])
                if digest(r, len(reqs[k][0])) != served[k]:
                    bad.append(k)
        return bad

    with ThreadPoolExecutor(max_workers=lanes) as ex:
        mismatch = sorted(k for b in ex.map(check, range(lanes)) for k in b)
    log("served vs one call per request: %s" % ("all %d equal" % count if not mismatch
                                                 else "%d DIFFER (first %s)" % (len(mismatch), mismatch[:5])))
    del dins, souts, sws, reqs, hs, hd, ht, pinned
    torch.cuda.empty_cache()
    log("serving: p50 %.1f ms p99 %.1f ms; saturated %.2f s, one call per request %.2f s"
        % (1e3 * np.percentile(lat, 50), 1e3 * np.percentile(lat, 99), wall_sat, wall_single))
    return {"workload": "rmat-hawkes-requests", "requests": count, "n_edges": total, "min_cluster_size": M,
            "seed": 4, "arrivals": "poisson 200 req/s (open loop)",
            "inputs": "host, pinned (copied to the GPU at submit)",
            "sizes": "lognormal median 70711 sigma 1.42 clipped [1e3, 5e6]; V = 2^ceil(log2(n/16))",
            "workers": workers, "hbm_budget_bytes": budget_gib << 30, "max_inflight": inflight,
            "output_pool_bytes": out_gib << 30, "saturated_pool_stalls": stalls_sat,
            "latency_p50_ms": 1e3 * float(np.percentile(lat, 50)), "latency_p99_ms": 1e3 * float(np.percentile(lat, 99)),
            "latency_mean_ms": 1e3 * float(lat.mean()), "open_loop_edges_per_s": total / wall_open,
            "open_loop_batches": st1["batches"] - st0["batches"],
            "saturated_edges_per_s": total / wall_sat, "saturated_batches": st2["batches"] - st1["batches"],
            "max_batch_requests": st2["max_batch_requests"], "max_concurrent_batches": st2["max_concurrent_batches"],
            "single_edges_per_s": total / wall_single, "ratio": wall_single / wall_sat,
            "single_timed_on": "every tenth request (%d requests, %d records), one call after another; rate "
                               "scaled by records" % (len(sample), rec_sample),
            "equal_to_single_calls": not mismatch, "requests_compared": count,
            "comparison": "two random 64-bit linear digests of every output field per request"}


def make_parser():
    ap = argparse.ArgumentParser(description="Temporal edges clustered per second on one MI355X (one JSON line).")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="scale", choices=sorted(WORKLOADS))
    ap.add_argument("--also", default="mid",
                    help="comma list of further single-graph workloads timed beside the main one ('' for none)")
    ap.add_argument("--mode", default="undirected", choices=["undirected", "causal"],
                    help="line graph: undirected (shared vertex, |dt|) or causal (tip-to-tail, increment weights)")
    ap.add_argument("--thresholds", default="none",
                    help="discrete dendrogram: 'none' (exact dendrogram), 'paper' (2^0 .. 2^28 s) or a comma list")
    ap.add_argument("--cpu-sample", type=int, default=20_000_000)
    ap.add_argument("--cpu-sample-all-cores", type=int, default=4_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=20000,
                    help="requests of the serving stream to replay (0 skips the serving measurement)")
    ap.add_argument("--hyper", action="store_true",
                    help="also time the dynamic-hypergraph workload (2e7 multi-recipient messages)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-vs-one-graph-per-call measurement on the 4096-graph batch")
    ap.add_argument("--roofline-kernel", default="k_krt_union",
                    help="dominant kernel: its launches are timed with HIP events on its stream for the roofline")
    ap.add_argument("--timing-steps", type=int, default=3,
                    help="steps after the timed ones in which the roofline kernel's launches are timed (0: none)")
    ap.add_argument("--no-small-call", action="store_true",
                    help="skip the one-call cost of a 57k-record graph (sync, async, replayed HIP graph)")
    ap.add_argument("--no-tuning", action="store_true",
                    help="built-in launch choices only (no tuning-file lookup, no tuned-vs-default comparison)")
    ap.add_argument("--default-steps", type=int, default=2,
                    help="calls timed with the built-in launch choices beside tuned ones (0: none)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="before the steps, copy a buffer of this many bytes once (a plain copy kernel of known "
                         "size for calibrating HBM counters)")
    return ap


def main():
    args = make_parser().parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported (run with --gpus 1)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    if args.thresholds == "none":
        thr = None
    elif args.thresholds == "paper":
        thr = [1 << k for k in range(29)]
    else:
        thr = [int(x) for x in args.thresholds.split(",")]
    causal = args.mode == "causal"

    log("generating workload %s" % args.workload)
    w, cfg = make_workload(args.workload)
    log("generated n=%d" % w.n)
    # CPU legs first, before this process touches the GPU (the all-core leg starts child processes)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu oracle on a prefix (one thread)")
        cpu, cpu_ref, cpu_n = cpu_oracle_single(w, args.cpu_sample, causal, thr)
        log("cpu oracle: %.3g edges/s" % cpu["value"])
        if not causal and not thr:
            cpu_all = cpu_oracle_all_cores(w, args.cpu_sample_all_cores)
            log("cpu oracle on all cores: %s" % cpu_all.get("value"))

    import torch
    from paper_2311_10337_amd import profiling
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        a = torch.ones(args.copy_calibration, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("copy calibration: %d bytes copied" % args.copy_calibration)
    cfg["line_graph"] = args.mode
    tag = cfg["workload"] + ("_causal" if causal else "") + ("_discrete" if thr else "")
    if thr:
        cfg["dendrogram"] = "discrete, %d thresholds %d..%d s" % (len(thr), thr[0], thr[-1])
    knobs = None if args.no_tuning else tuned_knobs(ce, w.n, w.num_vertices)
    r, el, (kms, kcnt, ksteps), keep, tune, step_ms = time_single_graph(
        ce, w, dev, args.steps, args.warmup, causal, thr, args.roofline_kernel, knobs, args.default_steps,
        args.timing_steps)
    roof = None
    if args.roofline_kernel and kcnt:
        log("kernel %s: %d launches in %d steps of their own, %.3f ms total, %.1f us avg"
            % (args.roofline_kernel, kcnt, ksteps, kms, 1e3 * kms / kcnt))
        roof = roofline_line(ce, profiling, args.roofline_kernel, kms, kcnt, w, r.m, ksteps, tag,
                             (knobs or {}).get("krt_level_bits", 0))
        roof["timed_in"] = "%d steps after the timed ones (events in the kernel's own dispatches)" % ksteps
    value = w.n * args.steps / el
    # whole path: HBM traffic per step from the committed counter summary (calibrated FETCH_SIZE +
    # WRITE_SIZE over every dispatch of one step), over the step's wall time; and the algorithmic model
    step_s = el / args.steps
    pipe = profiling.load_pipeline_traffic(os.path.join(ROOT, "profiles", "pipeline_%s_pmc.md" % tag))
    algo = profiling.PATH_BYTES_PER_EDGE * w.n
    hbm = {"peak_GBs": profiling.HBM_PEAK_GBS, "algorithmic_bytes_per_step": algo,
           "algorithmic_GBs": algo / step_s / 1e9, "algorithmic_frac": algo / step_s / 1e9 / profiling.HBM_PEAK_GBS,
           "counter_traffic_bytes_per_step": pipe, "counter_GBs": pipe / step_s / 1e9 if pipe else None,
           "counter_frac": pipe / step_s / 1e9 / profiling.HBM_PEAK_GBS if pipe else None,
           "amplification": pipe / algo if pipe else None,
           "note": "algorithmic = %d B per temporal edge over this run's wall time per step; counter traffic from "
                   "rocprofv3 FETCH_SIZE + WRITE_SIZE of the same workload (profiles/), null when the kernels "
                   "changed since" % profiling.PATH_BYTES_PER_EDGE}
    line = {"metric": METRIC, "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1000.0 * el / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
            "config": dict(cfg, m_msf=r.m, n_clusters=r.n_clusters, n_labels=r.n_labels),
            "step_ms": {"median": sorted(step_ms)[len(step_ms) // 2], "min": min(step_ms), "max": max(step_ms),
                        "note": "host clock around each timed call (each returns when its results are written)"}}
    if roof is not None:
        line["roofline"] = roof
    line["hbm_pipeline"] = hbm
    if tune is not None:
        line["tuning"] = {cfg["workload"]: tune}
    if thr:
        line["discrete_by_components"] = bench_level_components(ce, r, w.n, thr)
    del keep, r
    torch.cuda.empty_cache()
    if cpu is not None:
        # the GPU on the oracle's records: every output field must be byte-equal
        sub = torch.from_numpy(w.src[:cpu_n]).to(dev), torch.from_numpy(w.dst[:cpu_n]).to(dev), \
            torch.from_numpy(w.t[:cpu_n]).to(dev)
        got = ce.to_numpy(ce.cluster_edges(*sub, w.min_cluster_size, w.num_vertices, causal=causal,
                                           thresholds=thr))
        bad = compare_numpy(got, cpu_ref)
        cpu["parity"] = not bad
        cpu["parity_records"] = cpu_n
        if bad:
            cpu["parity_fields_differing"] = bad
        log("gpu vs cpu oracle on the first %d records: %s" % (cpu_n, "byte-equal" if not bad else "DIFFER %s" % bad))
        del sub, got, cpu_ref
        torch.cuda.empty_cache()
    del w
    workloads = {}
    for name in [x for x in args.also.split(",") if x and x != args.workload]:
        wx, cfgx = make_workload(name)
        kn = None if args.no_tuning else tuned_knobs(ce, wx.n, wx.num_vertices)
        sx = max(1, min(args.steps, 10))
        rx, elx, _, kx, tx, _ = time_single_graph(ce, wx, dev, sx, 1, causal, thr, knobs=kn, default_steps=sx)
        workloads[cfgx["workload"]] = dict(cfgx, edges_per_s=wx.n * sx / elx, ms_per_step=1e3 * elx / sx,
                                           m_msf=rx.m, n_clusters=rx.n_clusters, n_labels=rx.n_labels)
        if tx is not None:
            line.setdefault("tuning", {})[cfgx["workload"]] = tx
        del kx, rx, wx
        torch.cuda.empty_cache()
    if workloads:
        line["other_workloads"] = workloads
    if not args.no_small_call:
        line["small_call"] = bench_small_calls(ce, dev)
    if not args.no_batch:
        line["batched"] = bench_batched(dev, max(1, min(args.steps, 3)), 1, tuning=not args.no_tuning)
    if args.serve_requests > 0:
        from paper_2311_10337_amd import autotune
        with tuning_file(None if args.no_tuning else autotune.PACKAGE_FILE):
            line["serving"] = bench_serving(dev, args.serve_requests)
    if args.hyper:
        line["hypergraph"] = bench_hyper(dev, max(1, min(args.steps, 3)), 1)
    if cpu is not None:
        line["cpu_baseline"] = cpu
        if not causal and not thr:
            line["cpu_baseline_all_cores"] = cpu_all
    line["host"] = {"cpu": platform.processor() or platform.machine(), "nproc": os.cpu_count()}
    log("done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
