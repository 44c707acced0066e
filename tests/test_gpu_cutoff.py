"""GPU parity of the time-filtered line graph (only line-graph edges with
w <= max_dt): every output field against the oracle, in both line-graph modes,
for single graphs, batches and served requests."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster", "pt_lambda",
          "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected", "labels")


def _ce():
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.fail("libce.so is not built")
    return ce


def note(msg):
    print("[gpu-cutoff] " + msg, flush=True)
    sys.stdout.flush()


def dev_arrays(src, dst, t):
    dev = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(src, np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(dst, np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(t, np.int64)).to(dev))


def ref_dict(s, d, t, V, M, causal, cut):
    r = oracle.cluster(s, d, t, M, V, tier=1, causal=causal, max_dt=cut)
    assert r.status == 0
    out = {"m": r.m, "n_clusters": r.n_clusters, "n_labels": r.n_labels}
    for f in FIELDS:
        out[f] = getattr(r, f)
    return out


def same(got, ref, label):
    assert (got["m"], got["n_clusters"], got["n_labels"]) == (ref["m"], ref["n_clusters"], ref["n_labels"]), label
    for f in FIELDS:
        if not np.array_equal(got[f], ref[f]):
            raise AssertionError("%s: field %s differs" % (label, f))


def check(s, d, t, V, M, causal, cut, label):
    ce = _ce()
    note("%s n=%d causal=%s max_dt=%d" % (label, len(s), causal, cut))
    got = ce.to_numpy(ce.cluster_edges(*dev_arrays(s, d, t), M, V, causal=causal, max_dt=cut))
    same(got, ref_dict(s, d, t, V, M, causal, cut), label)
    return got


def test_random_graphs_and_cutoffs():
    rng = np.random.default_rng(31)
    for k in range(60):
        n = int(rng.integers(1, 400))
        V = int(rng.integers(2, 30))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V - 1, n).astype(np.int32)
        d[d >= s] += 1
        t = rng.integers(0, int(rng.choice([10, 1000])), n).astype(np.int64)
        for causal in (False, True):
            cut = int(rng.choice([0, 1, 5, 50, 1 << 40]))
            check(s, d, t, V, int(rng.choice([2, 3, 5])), causal, cut, "random%d" % k)


def test_tiny_workload_with_an_hour_cutoff():
    w = synth.plain_tiny()
    for causal in (False, True):
        check(w.src, w.dst, w.t, w.num_vertices, w.min_cluster_size, causal, 3600, "tiny")


def test_huge_cutoff_equals_none():
    ce = _ce()
    w = synth.plain_tiny()
    a = ce.to_numpy(ce.cluster_edges(*dev_arrays(w.src, w.dst, w.t), 5, w.num_vertices, max_dt=(1 << 63) - 1))
    b = ce.to_numpy(ce.cluster_edges(*dev_arrays(w.src, w.dst, w.t), 5, w.num_vertices))
    same(a, b, "huge cutoff")


def test_batch_and_server_with_cutoff():
    ce = _ce()
    rng = np.random.default_rng(2)
    graphs = []
    for g in range(20):
        n = int(rng.choice([0, 3, 200, 2000]))
        V = int(rng.integers(2, 50))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V - 1, n).astype(np.int32)
        d[d >= s] += 1
        t = rng.integers(0, 500, n).astype(np.int64)
        graphs.append((s, d, t, V))
    eoff = np.cumsum([0] + [len(x[0]) for x in graphs]).astype(np.int64)
    voff = np.cumsum([0] + [x[3] for x in graphs]).astype(np.int64)
    cat = lambda k, dt: np.concatenate([np.asarray(x[k], dt) for x in graphs])
    br = ce.cluster_batch(*dev_arrays(cat(0, np.int32), cat(1, np.int32), cat(2, np.int64)), eoff, voff, 3,
                          max_dt=20)
    for g, (s, d, t, V) in enumerate(graphs):
        same(br.graph(g), ref_dict(s, d, t, V, 3, False, 20), "batch graph %d" % g)
    with ce.Server(1 << 30, workers=2, max_inflight=64) as srv:
        tickets = [(srv.submit(s, d, t, 3, V, max_dt=cut), k, cut) for k, (s, d, t, V) in enumerate(graphs)
                   for cut in (-1, 20)]
        for tk, k, cut in tickets:
            r = srv.poll(tk, wait=True)
            assert r.status == ce.CE_OK
            s, d, t, V = graphs[k]
            same(ce.to_numpy(r.result), ref_dict(s, d, t, V, 3, False, cut), "served graph %d cut %d" % (k, cut))
