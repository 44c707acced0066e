#!/usr/bin/env python3
"""Benchmark: temporal edges clustered per second on one MI355X.

One step = one full clustering of the workload through the C ABI
(group+sort by vertex and time, path skeleton, Boruvka MSF, sorted MSF,
exact dendrogram, condensed tree, stability, excess of mass, labels), with
the input records already resident in HBM and the workspace and outputs
preallocated. Prints one JSON line.

Default workload (N=1): R-MAT scale 20 (1M vertices), 50M records,
per-pair Hawkes timestamps over 90 days, min_cluster_size 10, seed 1.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "temporal edges clustered/sec (bit-exact) + % HBM roofline; batched vs single"


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_workload(name):
    import synth
    if name == "tiny":
        return synth.plain_tiny(), {"workload": "chung-lu-bursts-tiny", "n_edges": 200_000, "n_vertices": 10_000,
                                    "min_cluster_size": 5, "seed": 0, "timestamps": "poisson bursts, 30 days"}
    if name == "mid":
        return synth.plain_mid(), {"workload": "rmat-hawkes-mid", "n_edges": 50_000_000, "n_vertices": 1 << 20,
                                   "min_cluster_size": 10, "seed": 1, "timestamps": "per-pair hawkes, 90 days"}
    if name == "scale":
        return synth.plain_scale(), {"workload": "rmat-hawkes-scale", "n_edges": 1 << 30, "n_vertices": 1 << 26,
                                     "min_cluster_size": 25, "seed": 2,
                                     "timestamps": "per-pair hawkes, 365 days, planted 1e7 hub"}
    raise ValueError(name)


def cpu_baseline(w, sample, causal=False, thresholds=None):
    """Time the CPU oracle (single-threaded plain C) on the first `sample` records."""
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
    return {"value": ns / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of %d records of the same workload (%s oracle%s, one host thread, %.1f s)"
                      % (ns, w.n, "Alg. 2 window" if causal else "path-skeleton",
                         ", discrete dendrogram with %d thresholds" % len(thresholds) if thresholds else "", dt)}


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


def bench_batched(dev, steps, warmup):
    """The 4096-graph batch in one call vs one call per graph, same GPU and inputs."""
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

    for _ in range(warmup):
        batch_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        br = batch_step()
    torch.cuda.synchronize()
    el_b = (time.perf_counter() - t0) / steps
    log("batched: %.1f ms per batch" % (1e3 * el_b))
    del ws
    ng = np.diff(eoff)
    vg = np.diff(voff)
    nmax = int(ng.max())
    souts = ce.Outputs(nmax, M, dev)
    sws = torch.empty(ce.workspace_bytes(nmax, int(vg.max()), M), dtype=torch.uint8, device=dev)

    def single(g):
        a, b = int(eoff[g]), int(eoff[g + 1])
        return ce.cluster_edges(s_d[a:b], d_d[a:b], t_d[a:b], M, int(vg[g]), outputs=souts, workspace=sws)

    for g in range(min(G, 64)):
        single(g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in range(G):
        single(g)
    torch.cuda.synchronize()
    el_s = time.perf_counter() - t0
    log("one graph per call: %.1f ms for the %d graphs" % (1e3 * el_s, G))
    out = {"workload": "chung-lu-bursts-batch-4096", "graphs": G, "n_edges": n, "min_cluster_size": M, "seed": 3,
           "sizes": "lognormal median 20000 sigma 1.5 clipped [500, 2e6]; V_g = n_g/20",
           "batched_edges_per_s": n / el_b, "batched_ms": 1e3 * el_b, "batched_steps": steps,
           "single_edges_per_s": n / el_s, "single_ms": 1e3 * el_s,
           "ratio": el_s / el_b, "n_clusters": int(br.n_clusters.sum()), "n_labels": int(br.n_labels.sum())}
    del s_d, d_d, t_d, outs, souts, sws
    torch.cuda.empty_cache()
    return out


def bench_serving(dev, count, workers=3, budget_gib=64):
    """Open-loop replay of the request stream (Poisson arrivals at 200/s) through the
    continuous-batching server, then the same requests submitted all at once,
    against one call per request."""
    import numpy as np
    import torch
    import synth
    import paper_2311_10337_amd as ce
    M = 10
    sizes = synth.request_sizes(20000, seed=4)[:count]
    arr = synth.request_arrivals(20000, seed=4)[:count]
    arr = arr - arr[0]
    t0 = time.perf_counter()
    reqs = [synth.request_graph(r, int(sizes[r]), seed=4) for r in range(count)]
    total = int(sum(len(r[0]) for r in reqs))
    log("serving workload: %d requests, %d records (%.1f s)" % (count, total, time.perf_counter() - t0))
    outs = [ce.Outputs(len(r[0]), M, dev) for r in reqs]
    srv = ce.Server(budget_gib << 30, workers=workers, max_inflight=count)

    def replay(arrivals):
        lat = np.zeros(count)
        pending = {}
        k = 0
        first_sub, last_done = None, 0.0
        start = time.perf_counter()
        while k < count or pending:
            progressed = False
            now = time.perf_counter() - start
            while k < count and now >= arrivals[k]:
                s, d, t, V = reqs[k]
                sub = time.perf_counter() - start
                try:
                    tk = srv.submit(s, d, t, M, V, outputs=outs[k])
                except ce.ServerBusy:
                    break
                first_sub = sub if first_sub is None else first_sub
                pending[tk] = (k, sub)
                k += 1
                progressed = True
                now = time.perf_counter() - start
            for tk in list(pending):
                r = srv.poll(tk)
                if r is not None:
                    kk, sub = pending.pop(tk)
                    if r.status != ce.CE_OK:
                        raise RuntimeError("request %d failed: %s" % (kk, r.error))
                    lat[kk] = (sub - arrivals[kk]) + r.latency_s
                    last_done = max(last_done, sub + r.latency_s)
                    progressed = True
            if not progressed:
                time.sleep(0.0002)
        return lat, last_done - arrivals[0]

    replay(np.zeros(count))  # warm-up pass, everything at once
    st0 = srv.stats()
    lat, wall_open = replay(arr)
    st1 = srv.stats()
    _, wall_sat = replay(np.zeros(count))
    st2 = srv.stats()
    srv.close()
    # one call per request, inputs already on the GPU
    dins = [tuple(torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in r[:3]) + (r[3],) for r in reqs]
    nmax = max(len(r[0]) for r in reqs)
    souts = ce.Outputs(nmax, M, dev)
    sws = torch.empty(ce.workspace_bytes(nmax, max(r[3] for r in reqs), M), dtype=torch.uint8, device=dev)
    for k in range(min(count, 16)):
        s, d, t, V = dins[k]
        ce.cluster_edges(s, d, t, M, V, outputs=souts, workspace=sws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, d, t, V in dins:
        ce.cluster_edges(s, d, t, M, V, outputs=souts, workspace=sws)
    torch.cuda.synchronize()
    wall_single = time.perf_counter() - t0
    del dins, souts, sws, outs
    torch.cuda.empty_cache()
    log("serving: p50 %.1f ms p99 %.1f ms; saturated %.2f s, one call per request %.2f s"
        % (1e3 * np.percentile(lat, 50), 1e3 * np.percentile(lat, 99), wall_sat, wall_single))
    return {"workload": "rmat-hawkes-requests", "requests": count, "n_edges": total, "min_cluster_size": M,
            "seed": 4, "arrivals": "poisson 200 req/s (open loop)",
            "sizes": "lognormal median 70711 sigma 1.42 clipped [1e3, 5e6]; V = 2^ceil(log2(n/16))",
            "workers": workers, "hbm_budget_bytes": budget_gib << 30,
            "latency_p50_ms": 1e3 * float(np.percentile(lat, 50)), "latency_p99_ms": 1e3 * float(np.percentile(lat, 99)),
            "latency_mean_ms": 1e3 * float(lat.mean()), "open_loop_edges_per_s": total / wall_open,
            "open_loop_batches": st1["batches"] - st0["batches"],
            "saturated_edges_per_s": total / wall_sat, "saturated_batches": st2["batches"] - st1["batches"],
            "max_batch_requests": st2["max_batch_requests"], "max_concurrent_batches": st2["max_concurrent_batches"],
            "single_edges_per_s": total / wall_single, "ratio": wall_single / wall_sat}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mid", choices=["tiny", "mid", "scale"])
    ap.add_argument("--mode", default="undirected", choices=["undirected", "causal"],
                    help="line graph: undirected (shared vertex, |dt|) or causal (tip-to-tail, increment weights)")
    ap.add_argument("--thresholds", default="none",
                    help="discrete dendrogram: 'none' (exact dendrogram), 'paper' (2^0 .. 2^28 s) or a comma list")
    ap.add_argument("--cpu-sample", type=int, default=20_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of the serving stream to replay (0 skips the serving measurement)")
    ap.add_argument("--no-hyper", action="store_true",
                    help="skip the dynamic-hypergraph measurement (2e7 multi-recipient messages)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-vs-one-graph-per-call measurement on the 4096-graph batch")
    ap.add_argument("--roofline-kernel", default="k_krt_union",
                    help="dominant kernel: its launches are timed with HIP events on its stream for the roofline")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="before the steps, copy a buffer of this many bytes once (a plain copy kernel of known "
                         "size for calibrating HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported (run with --gpus 1)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()

    log("generating workload %s" % args.workload)
    t0 = time.perf_counter()
    w, cfg = make_workload(args.workload)
    log("generated n=%d in %.1f s" % (w.n, time.perf_counter() - t0))
    dev = torch.device("cuda:0")
    src = torch.from_numpy(w.src).to(dev)
    dst = torch.from_numpy(w.dst).to(dev)
    tt = torch.from_numpy(w.t).to(dev)
    M, V = w.min_cluster_size, w.num_vertices
    if args.copy_calibration:
        a = torch.ones(args.copy_calibration, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("copy calibration: %d bytes copied" % args.copy_calibration)
    if args.thresholds == "none":
        thr = None
    elif args.thresholds == "paper":
        thr = [1 << k for k in range(29)]
    else:
        thr = [int(x) for x in args.thresholds.split(",")]
    outs = ce.Outputs(w.n, M, dev)
    ws = torch.empty(ce.workspace_bytes(w.n, V, M, thresholds=thr), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    causal = args.mode == "causal"
    cfg["line_graph"] = args.mode
    tag = cfg["workload"] + ("_causal" if causal else "") + ("_discrete" if thr else "")
    if thr:
        cfg["dendrogram"] = "discrete, %d thresholds %d..%d s" % (len(thr), thr[0], thr[-1])

    def step():
        return ce.cluster_edges(src, dst, tt, M, V, outputs=outs, workspace=ws, causal=causal, thresholds=thr)

    for i in range(args.warmup):
        r = step()
        log("warmup %d done: m=%d clusters=%d labels=%d" % (i, r.m, r.n_clusters, r.n_labels))
    torch.cuda.synchronize()
    if args.roofline_kernel:
        ce.timing_enable(args.roofline_kernel)
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    log("timed %d steps in %.3f s" % (args.steps, el))
    roof = None
    if args.roofline_kernel:
        from paper_2311_10337_amd import profiling
        kms, kcnt = ce.timing_read()
        ce.timing_enable(None)
        log("kernel %s: %d launches, %.3f ms total, %.1f us avg" % (args.roofline_kernel, kcnt, kms,
                                                                  1e3 * kms / max(kcnt, 1)))
        try:
            unit, per_unit, units = profiling.algorithmic_bytes_per_step(args.roofline_kernel, w.n, r.m)
        except KeyError:
            log("no algorithmic model for %s: roofline left out" % args.roofline_kernel)
            unit, per_unit, units = None, None, None
        if kcnt and units:
            per_launch = per_unit * units * args.steps / kcnt
            achieved = per_launch / (kms / kcnt * 1e-3) / 1e9
            traffic = profiling.load_traffic(args.roofline_kernel, os.path.join(
                ROOT, "profiles", "%s_%s_pmc.md" % (args.roofline_kernel, tag)))
            roof = {"bound": "hbm", "achieved": achieved, "peak": profiling.HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / profiling.HBM_PEAK_GBS, "traffic": traffic, "kernel": args.roofline_kernel,
                    "algorithmic_bytes_per_launch": per_launch, "launches": kcnt,
                    "avg_launch_us": 1e3 * kms / kcnt, "unit_of_work": unit, "bytes_per_unit": per_unit}
    value = w.n * args.steps / el
    # whole path: HBM traffic per step from the committed counter summary (calibrated FETCH_SIZE +
    # WRITE_SIZE over every dispatch of one step), over the step's wall time; and the algorithmic model
    from paper_2311_10337_amd import profiling
    step_s = el / args.steps
    pipe = profiling.load_pipeline_traffic(os.path.join(ROOT, "profiles", "pipeline_%s_pmc.md" % tag))
    algo = profiling.PATH_BYTES_PER_EDGE * w.n
    hbm = {"peak_GBs": profiling.HBM_PEAK_GBS, "traffic_bytes_per_step": pipe,
           "achieved_GBs": pipe / step_s / 1e9 if pipe else None,
           "frac": pipe / step_s / 1e9 / profiling.HBM_PEAK_GBS if pipe else None,
           "algorithmic_bytes_per_step": algo, "algorithmic_GBs": algo / step_s / 1e9,
           "algorithmic_frac": algo / step_s / 1e9 / profiling.HBM_PEAK_GBS,
           "note": "traffic from rocprofv3 counters of the same workload (profiles/), time = this run's wall "
                   "time per step; algorithmic = %d B per temporal edge" % profiling.PATH_BYTES_PER_EDGE}
    line = {"metric": METRIC, "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1000.0 * el / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
            "config": dict(cfg, m_msf=r.m, n_clusters=r.n_clusters, n_labels=r.n_labels)}
    if roof is not None:
        line["roofline"] = roof
    line["hbm_pipeline"] = hbm
    del ws
    torch.cuda.empty_cache()
    if thr:
        line["discrete_by_components"] = bench_level_components(ce, r, w.n, thr)
    del src, dst, tt, outs
    torch.cuda.empty_cache()
    if not args.no_batch:
        line["batched"] = bench_batched(dev, max(1, min(args.steps, 3)), 1)
    if args.serve_requests > 0:
        line["serving"] = bench_serving(dev, args.serve_requests)
    if not args.no_hyper:
        line["hypergraph"] = bench_hyper(dev, max(1, min(args.steps, 3)), 1)
    if not args.no_cpu_baseline:
        log("cpu baseline on a sample")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample, causal, thr)
    line["host"] = {"cpu": platform.processor() or platform.machine(), "nproc": os.cpu_count()}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
