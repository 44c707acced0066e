"""GPU parity of CAUSAL mode (the increment-weighted line graph of Def. 1 with
Alg. 2 windows): the HIP path through the C ABI equals the oracle element by
element on every output field."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from conftest import load_golden

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
    print("[gpu-causal] " + msg, flush=True)
    sys.stdout.flush()


def dev_arrays(src, dst, t):
    dev = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(src, np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(dst, np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(t, np.int64)).to(dev))


def run_gpu(src, dst, t, V, M):
    ce = _ce()
    return ce.to_numpy(ce.cluster_edges(*dev_arrays(src, dst, t), M, V, causal=True))


def ref_dict(src, dst, t, V, M):
    r = oracle.cluster(src, dst, t, M, V, tier=1, causal=True)
    assert r.status == 0
    out = {"m": r.m, "n_clusters": r.n_clusters, "n_labels": r.n_labels}
    for f in FIELDS:
        out[f] = getattr(r, f)
    return out


def same(got, ref, label):
    assert (got["m"], got["n_clusters"], got["n_labels"]) == (ref["m"], ref["n_clusters"], ref["n_labels"]), label
    for f in FIELDS:
        a, b = got[f], ref[f]
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0][:10] if a.shape == b.shape else "shape %s vs %s" % (a.shape, b.shape)
            raise AssertionError("%s: field %s differs at %s" % (label, f, bad))


def assert_parity(src, dst, t, V, M, label):
    note("case %s n=%d V=%d M=%d" % (label, len(src), V, M))
    got = run_gpu(src, dst, t, V, M)
    same(got, ref_dict(src, dst, t, V, M), label)
    return got


def test_golden_and_hand_fixtures():
    s, d, t = load_golden("table2_chain.txt")
    V = int(max(s.max(), d.max()) + 1)
    got = assert_parity(s, d, t, V, 2, "table2")
    assert list(got["msf_w"]) == [291, 651, 1708, 1977]
    s, d, t = load_golden("table3_long.txt")
    assert_parity(s, d, t, int(max(s.max(), d.max()) + 1), 3, "table3")
    # the window example: in a, in b, out x, out y, in c, out z at vertex 9
    assert_parity(np.array([1, 2, 9, 9, 5, 9], np.int32), np.array([9, 9, 3, 4, 9, 6], np.int32),
                  np.array([1, 2, 3, 5, 6, 8], np.int64), 10, 2, "window")
    # sink and source pairs are not arcs; equal times put in-edges first; a 2-cycle at equal times
    assert_parity(np.array([0, 2], np.int32), np.array([1, 1], np.int32), np.array([0, 5], np.int64), 3, 2, "sink")
    assert_parity(np.array([1, 1], np.int32), np.array([0, 2], np.int32), np.array([0, 5], np.int64), 3, 2, "source")
    assert_parity(np.array([9, 1], np.int32), np.array([2, 9], np.int32), np.array([4, 4], np.int64), 10, 2, "tie")
    assert_parity(np.array([0, 1], np.int32), np.array([1, 0], np.int32), np.array([3, 3], np.int64), 2, 2, "2cycle")


def test_degenerate_sizes():
    z32, z64 = np.zeros(0, np.int32), np.zeros(0, np.int64)
    got = run_gpu(z32, z32, z64, 4, 5)
    assert got["m"] == 0 and got["n_clusters"] == 1
    assert_parity(np.array([0], np.int32), np.array([1], np.int32), np.array([7], np.int64), 2, 2, "n1")
    # two records with no arc between them (wrong order)
    assert_parity(np.array([1, 0], np.int32), np.array([2, 1], np.int32), np.array([5, 9], np.int64), 3, 2, "n2")


def test_random_tie_heavy_small():
    rng = np.random.default_rng(21)
    for k in range(150):
        n = int(rng.integers(1, 300))
        V = int(rng.integers(2, 30))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V - 1, n).astype(np.int32)
        d[d >= s] += 1
        t = (rng.integers(0, int(rng.choice([2, 5, 40])), n) * int(rng.choice([1, 1000]))).astype(np.int64)
        assert_parity(s, d, t, V, int(rng.choice([2, 3, 5])), "random%d" % k)


def test_long_windows_and_ragged_sizes():
    """A hub receiving thousands of records before it sends (windows far longer than a wave), plus sizes
    that end in ragged tiles."""
    rng = np.random.default_rng(4)
    n_in = 5000
    s = np.concatenate([rng.integers(1, 400, n_in), np.zeros(40, np.int64), rng.integers(1, 400, 300),
                        np.zeros(7, np.int64)]).astype(np.int32)
    d = np.concatenate([np.zeros(n_in, np.int64), rng.integers(1, 400, 40), np.zeros(300, np.int64),
                        rng.integers(1, 400, 7)]).astype(np.int32)
    t = np.concatenate([rng.integers(0, 1000, n_in), rng.integers(1000, 1100, 40), rng.integers(1100, 1200, 300),
                        rng.integers(1150, 1300, 7)]).astype(np.int64)
    assert_parity(s, d, t, 400, 5, "hub")
    for n in (4095, 4097, 65537):
        s = rng.integers(0, 500, n).astype(np.int32)
        d = rng.integers(0, 499, n).astype(np.int32)
        d[d >= s] += 1
        t = rng.integers(0, 20000, n).astype(np.int64)
        assert_parity(s, d, t, 500, 5, "ragged%d" % n)


def test_tiny_workload_full():
    w = synth.plain_tiny()
    assert_parity(w.src, w.dst, w.t, w.num_vertices, w.min_cluster_size, "tiny")


def test_rmat_hawkes_scaled():
    s, d, t = synth.rmat_hawkes(2_000_000, 16, 11)
    assert_parity(s, d, t, 1 << 16, 10, "rmat2M")


def test_wide_key_with_a_long_equal_time_run():
    """Many records arriving at one vertex at one time over a wide time span: w << wshift does not fit the
    key, so the key holds the weight's rank among the skeleton's distinct weights; outputs equal the oracle."""
    k = 1500
    s = np.concatenate([np.arange(1, k + 1), [0]]).astype(np.int32)
    d = np.concatenate([np.zeros(k), [5]]).astype(np.int32)
    t = np.concatenate([np.zeros(k), [1 << 52]]).astype(np.int64)
    same(run_gpu(s, d, t, k + 1, 2), ref_dict(s, d, t, k + 1, 2), "long equal-time run, wide span")


def test_batch_causal_per_graph():
    ce = _ce()
    rng = np.random.default_rng(9)
    graphs = []
    for g in range(40):
        n = int(rng.choice([0, 1, 2, 50, 700, 3000]))
        V = int(rng.integers(2, 40))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V - 1, n).astype(np.int32)
        d[d >= s] += 1
        t = rng.integers(0, 30, n).astype(np.int64)
        graphs.append((s, d, t, V))
    eoff = np.zeros(len(graphs) + 1, np.int64)
    voff = np.zeros(len(graphs) + 1, np.int64)
    for g, (s, d, t, V) in enumerate(graphs):
        eoff[g + 1] = eoff[g] + len(s)
        voff[g + 1] = voff[g] + V
    cat = lambda k, dt: np.concatenate([np.asarray(x[k], dt) for x in graphs])
    br = ce.cluster_batch(*dev_arrays(cat(0, np.int32), cat(1, np.int32), cat(2, np.int64)), eoff, voff, 3,
                          causal=True)
    for g, (s, d, t, V) in enumerate(graphs):
        same(br.graph(g), ref_dict(s, d, t, V, 3), "batch graph %d" % g)


def test_server_mixes_modes():
    """Causal and undirected requests served together: each equals its own mode alone."""
    ce = _ce()
    reqs = []
    for r in range(12):
        s, d, t, V = synth.request_graph(r, 20_000 + 5_000 * r, seed=4)
        reqs.append((s, d, t, V, r % 2 == 1))
    with ce.Server(4 << 30, workers=2, max_inflight=32) as srv:
        tickets = [srv.submit(s, d, t, 10, V, causal=c) for (s, d, t, V, c) in reqs]
        res = [srv.poll(tk, wait=True) for tk in tickets]
    for k, ((s, d, t, V, c), g) in enumerate(zip(reqs, res)):
        assert g.status == ce.CE_OK
        alone = ce.to_numpy(ce.cluster_edges(*dev_arrays(s, d, t), 10, V, causal=c))
        same(ce.to_numpy(g.result), alone, "served request %d causal=%s" % (k, c))
        if c and k < 4:
            same(alone, ref_dict(s, d, t, V, 10), "request %d vs oracle" % k)


@pytest.mark.timeout(1200)
def test_mid_workload_causal_full_size():
    w = synth.plain_mid()
    assert_parity(w.src, w.dst, w.t, w.num_vertices, w.min_cluster_size, "mid-causal")
