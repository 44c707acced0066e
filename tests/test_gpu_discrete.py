"""GPU parity of the discrete dendrogram (Alg. 5) and of condensing on it:
every output field, the per-row levels and level tops included, against the
oracle, for single graphs in both line-graph modes, batches and served
requests, up to the 5e7-record workload with the paper's thresholds
2^0 .. 2^28 s."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster", "pt_lambda",
          "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected", "labels",
          "dd_level", "dd_top")
PAPER_THRESHOLDS = [1 << k for k in range(29)]


def _ce():
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.fail("libce.so is not built")
    return ce


def note(msg):
    print("[gpu-discrete] " + msg, flush=True)
    sys.stdout.flush()


def dev_arrays(src, dst, t):
    dev = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(src, np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(dst, np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(t, np.int64)).to(dev))


def ref_dict(s, d, t, V, M, thr, causal=False):
    r, dl, dt = oracle.cluster_discrete(s, d, t, M, thr, V, causal=causal)
    assert r.status == 0
    out = {"m": r.m, "n_clusters": r.n_clusters, "n_labels": r.n_labels, "dd_level": dl, "dd_top": dt}
    for f in FIELDS[:-2]:
        out[f] = getattr(r, f)
    return out


def same(got, ref, label):
    assert (got["m"], got["n_clusters"], got["n_labels"]) == (ref["m"], ref["n_clusters"], ref["n_labels"]), label
    for f in FIELDS:
        a, b = got[f], ref[f]
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0][:10] if a.shape == b.shape else "shape %s vs %s" % (a.shape, b.shape)
            raise AssertionError("%s: field %s differs at %s" % (label, f, bad))


def check(s, d, t, V, M, thr, label, causal=False):
    ce = _ce()
    note("%s n=%d q=%d causal=%s" % (label, len(s), len(thr), causal))
    got = ce.to_numpy(ce.cluster_edges(*dev_arrays(s, d, t), M, V, causal=causal, thresholds=thr))
    same(got, ref_dict(s, d, t, V, M, thr, causal), label)
    return got


def test_three_bursts_one_level():
    s = np.zeros(15, np.int32)
    d = np.arange(1, 16, dtype=np.int32)
    t = np.array([0, 1, 2, 3, 4, 100, 101, 102, 103, 104, 200, 201, 202, 203, 204], np.int64)
    got = check(s, d, t, 16, 3, [1, 128], "bursts")
    assert got["n_clusters"] == 4 and got["n_labels"] == 3


def test_random_graphs_and_thresholds():
    rng = np.random.default_rng(41)
    for k in range(80):
        n = int(rng.integers(1, 500))
        V = int(rng.integers(2, 40))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V - 1, n).astype(np.int32)
        d[d >= s] += 1
        t = rng.integers(0, int(rng.choice([20, 2000, 10 ** 6])), n).astype(np.int64)
        thr = PAPER_THRESHOLDS if k % 4 == 0 else sorted(set(int(x) for x in rng.integers(0, 3000, 5)))
        check(s, d, t, V, int(rng.choice([2, 3, 5])), thr, "random%d" % k, causal=bool(k % 2))


def test_tiny_workload_paper_thresholds():
    w = synth.plain_tiny()
    for causal in (False, True):
        check(w.src, w.dst, w.t, w.num_vertices, w.min_cluster_size, PAPER_THRESHOLDS, "tiny", causal)


def test_rmat_hawkes_scaled():
    s, d, t = synth.rmat_hawkes(2_000_000, 16, 11)
    check(s, d, t, 1 << 16, 10, PAPER_THRESHOLDS, "rmat2M")


def test_threshold_argument_errors():
    ce = _ce()
    w = synth.plain_tiny()
    a = dev_arrays(w.src[:100], w.dst[:100], w.t[:100])
    for bad in ([5, 5], [3, 1], [-1, 4], list(range(65))):
        with pytest.raises(ce.ClusterError) as ei:
            ce.cluster_edges(*a, 5, w.num_vertices, thresholds=bad)
        assert ei.value.status == ce.CE_EINVAL


def test_batch_and_server_discrete():
    ce = _ce()
    rng = np.random.default_rng(6)
    graphs = []
    for g in range(24):
        n = int(rng.choice([0, 1, 50, 900, 4000]))
        V = int(rng.integers(2, 60))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V - 1, n).astype(np.int32)
        d[d >= s] += 1
        t = rng.integers(0, 5000, n).astype(np.int64)
        graphs.append((s, d, t, V))
    thr = [1, 4, 16, 64, 256, 1024]
    eoff = np.cumsum([0] + [len(x[0]) for x in graphs]).astype(np.int64)
    voff = np.cumsum([0] + [x[3] for x in graphs]).astype(np.int64)
    cat = lambda k, dt: np.concatenate([np.asarray(x[k], dt) for x in graphs])
    br = ce.cluster_batch(*dev_arrays(cat(0, np.int32), cat(1, np.int32), cat(2, np.int64)), eoff, voff, 3,
                          thresholds=thr)
    for g, (s, d, t, V) in enumerate(graphs):
        same(br.graph(g), ref_dict(s, d, t, V, 3, thr), "batch graph %d" % g)
    with ce.Server(1 << 30, workers=2, max_inflight=64) as srv:
        tickets = [(srv.submit(s, d, t, 3, V, thresholds=th), k, th) for k, (s, d, t, V) in enumerate(graphs)
                   for th in (thr, [2, 2048])]
        for tk, k, th in tickets:
            r = srv.poll(tk, wait=True)
            assert r.status == ce.CE_OK
            s, d, t, V = graphs[k]
            same(ce.to_numpy(r.result), ref_dict(s, d, t, V, 3, th), "served graph %d" % k)


@pytest.mark.timeout(1200)
def test_mid_workload_discrete_full_size():
    w = synth.plain_mid()
    check(w.src, w.dst, w.t, w.num_vertices, w.min_cluster_size, PAPER_THRESHOLDS, "mid-discrete")
