"""GPU parity of batches: every graph of a packed batch gets exactly the outputs
the oracle gives for that graph alone (local ids, its own root and labels).

Small and mid-sized batches are checked graph by graph against the oracle; the
full 4096-graph batch (about 2.4e8 records) is checked on every graph against
the oracle (digests of every field, the oracle run in 16 host processes), on
sampled graphs field by field and against one-graph-per-call runs, and on
properties that hold for every graph.
"""
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
    print("[gpu-batch] " + msg, flush=True)
    sys.stdout.flush()


def pack(graphs):
    """graphs: list of (src, dst, t, V) -> concatenated arrays and offsets."""
    G = len(graphs)
    eoff = np.zeros(G + 1, np.int64)
    voff = np.zeros(G + 1, np.int64)
    for g, (s, d, t, V) in enumerate(graphs):
        eoff[g + 1] = eoff[g] + len(s)
        voff[g + 1] = voff[g] + V
    cat = lambda k, dt: (np.concatenate([np.asarray(x[k], dt) for x in graphs]) if G else np.zeros(0, dt))
    return cat(0, np.int32), cat(1, np.int32), cat(2, np.int64), eoff, voff


def run_batch(src, dst, t, eoff, voff, M):
    ce = _ce()
    dev = torch.device("cuda:0")
    s = torch.from_numpy(np.ascontiguousarray(src, np.int32)).to(dev)
    d = torch.from_numpy(np.ascontiguousarray(dst, np.int32)).to(dev)
    tt = torch.from_numpy(np.ascontiguousarray(t, np.int64)).to(dev)
    return ce.cluster_batch(s, d, tt, eoff, voff, M)


def run_single(src, dst, t, V, M):
    ce = _ce()
    dev = torch.device("cuda:0")
    s = torch.from_numpy(np.ascontiguousarray(src, np.int32)).to(dev)
    d = torch.from_numpy(np.ascontiguousarray(dst, np.int32)).to(dev)
    tt = torch.from_numpy(np.ascontiguousarray(t, np.int64)).to(dev)
    return ce.to_numpy(ce.cluster_edges(s, d, tt, M, V))


def same(got, ref, label):
    assert (got["m"], got["n_clusters"], got["n_labels"]) == (ref["m"], ref["n_clusters"], ref["n_labels"]), label
    for f in FIELDS:
        a, b = got[f], ref[f]
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0][:10] if a.shape == b.shape else "shape %s vs %s" % (a.shape, b.shape)
            raise AssertionError("%s: field %s differs at %s" % (label, f, bad))


def oracle_dict(s, d, t, V, M):
    r = oracle.cluster(s, d, t, M, V, tier=1)
    assert r.status == 0
    out = {"m": r.m, "n_clusters": r.n_clusters, "n_labels": r.n_labels}
    for f in FIELDS:
        out[f] = getattr(r, f)
    return out


def check_batch_vs_oracle(graphs, M, label):
    src, dst, t, eoff, voff = pack(graphs)
    note("%s: G=%d n=%d M=%d" % (label, len(graphs), len(src), M))
    br = run_batch(src, dst, t, eoff, voff, M)
    assert list(br.edge_offsets) == list(eoff)
    for g, (s, d, tt, V) in enumerate(graphs):
        same(br.graph(g), oracle_dict(np.asarray(s, np.int32), np.asarray(d, np.int32), np.asarray(tt, np.int64), V,
                                      M), "%s graph %d" % (label, g))
    # offsets agree with the per-graph counts
    assert np.array_equal(np.diff(br.row_offsets), br.m)
    assert np.array_equal(np.diff(br.cluster_offsets), br.n_clusters)
    return br


def test_batch_golden_and_hand_graphs():
    graphs = []
    for name in ("table2_chain.txt", "table3_long.txt"):
        s, d, t = load_golden(name)
        graphs.append((s, d, t, int(max(s.max(), d.max()) + 1)))
    graphs.append((np.zeros(6, np.int32), np.arange(1, 7, dtype=np.int32), np.array([0, 2, 5, 7, 13, 14], np.int64),
                   7))
    graphs.append((np.zeros(7, np.int32), np.arange(1, 8, dtype=np.int32), np.full(7, 5, np.int64), 8))
    for M in (2, 3, 5):
        check_batch_vs_oracle(graphs, M, "golden+hand M=%d" % M)


def test_batch_with_empty_and_single_record_graphs():
    e32, e64 = np.zeros(0, np.int32), np.zeros(0, np.int64)
    one = (np.array([0], np.int32), np.array([1], np.int32), np.array([5], np.int64), 2)
    two = (np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([7, 9], np.int64), 3)
    star = (np.zeros(9, np.int32), np.arange(1, 10, dtype=np.int32), np.array([0, 1, 2, 3, 50, 51, 52, 53, 54],
                                                                                np.int64), 10)
    graphs = [(e32, e32, e64, 4), one, star, (e32, e32, e64, 1), two, one, star, (e32, e32, e64, 3)]
    check_batch_vs_oracle(graphs, 2, "mixed-degenerate")
    check_batch_vs_oracle([(e32, e32, e64, 4)] * 5, 2, "all-empty")
    check_batch_vs_oracle([one, (e32, e32, e64, 4)], 2, "one-record")
    check_batch_vs_oracle([star], 3, "single-graph-batch")


def test_batch_random_ragged_tie_heavy():
    rng = np.random.default_rng(11)
    graphs = []
    for g in range(96):
        n = int(rng.choice([0, 1, 2, 3, 17, 200, 1000, 4097, 9000]))
        V = int(rng.integers(2, 60))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V - 1, n).astype(np.int32)
        d[d >= s] += 1
        t = rng.integers(0, 40, n).astype(np.int64) * int(rng.choice([1, 1000]))
        graphs.append((s, d, t, V))
    for M in (2, 5):
        check_batch_vs_oracle(graphs, M, "random-ragged M=%d" % M)


def test_batch_recipe_reduced():
    """The batching recipe (Chung-Lu bursts, lognormal sizes) with 256 graphs capped at 2e5 records."""
    sizes = np.minimum(synth.batch_sizes(256, seed=3), 200_000)
    graphs = []
    for g in range(256):
        s, d, t, V = synth.batch_graph(g, int(sizes[g]), seed=3)
        graphs.append((s, d, t, V))
    check_batch_vs_oracle(graphs, 5, "recipe-256")


def test_batch_data_errors_fail_the_call():
    ce = _ce()
    ok = (np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([7, 9], np.int64), 3)
    loop = (np.array([0, 1], np.int32), np.array([1, 1], np.int32), np.array([7, 9], np.int64), 3)
    # vertex 3 is valid for the batch as a whole but outside [0, 3) of its own graph
    oor = (np.array([0, 1], np.int32), np.array([1, 3], np.int32), np.array([7, 9], np.int64), 3)
    for bad, status in ((loop, ce.CE_ESELFLOOP), (oor, ce.CE_ERANGE)):
        src, dst, t, eoff, voff = pack([ok, bad, ok])
        with pytest.raises(ce.ClusterError) as ei:
            run_batch(src, dst, t, eoff, voff, 2)
        assert ei.value.status == status


@pytest.mark.timeout(1500)
def test_batch_full_size_sampled():
    """4096 graphs as in the batching workload, in one call (the launch bench.py times)."""
    ce = _ce()
    note("generating the 4096-graph batch")
    src, dst, t, eoff, voff = synth.batch_workload(4096, seed=3)
    G, n = 4096, len(src)
    M = 5
    note("batch n=%d" % n)
    br = run_batch(src, dst, t, eoff, voff, M)
    ng = np.diff(eoff)
    # properties every graph satisfies
    assert np.all(br.m <= np.maximum(ng - 1, 0))
    assert np.all(br.n_clusters >= 1) and np.all(br.n_clusters <= 2 * (ng // M) + 1)
    assert int(br.row_offsets[-1]) == br.result.m
    labels = br.result.labels.cpu().numpy()
    nl = br.n_labels
    for g in range(G):
        lg = labels[eoff[g]:eoff[g + 1]]
        assert lg.max(initial=-1) == nl[g] - 1
    sizes_h = br.result.cl_size.cpu().numpy().view(np.uint32)
    roots = br.cluster_offsets[1:] - 1
    assert np.array_equal(sizes_h[roots].astype(np.int64), ng)
    # sampled graphs against the oracle and against one graph per call
    rng = np.random.default_rng(5)
    order = np.argsort(ng)
    pick = sorted(set([int(order[0]), int(order[-1]), int(order[G // 2])] + list(rng.choice(G, 5, replace=False))))
    for g in pick:
        a, b = int(eoff[g]), int(eoff[g + 1])
        V = int(voff[g + 1] - voff[g])
        note("graph %d n=%d vs oracle" % (g, b - a))
        same(br.graph(g), oracle_dict(src[a:b], dst[a:b], t[a:b], V, M), "full batch graph %d" % g)
    for g in rng.choice(G, 24, replace=False):
        a, b = int(eoff[g]), int(eoff[g + 1])
        V = int(voff[g + 1] - voff[g])
        same(br.graph(int(g)), run_single(src[a:b], dst[a:b], t[a:b], V, M), "full batch graph %d vs single" % g)


@pytest.fixture
def live(capsys):
    """Progress lines that reach the terminal while the test runs (long tests print as they go)."""
    import time

    def say(msg):
        with capsys.disabled():
            print("[gpu-batch] %s %s" % (time.strftime("%H:%M:%S"), msg), flush=True)
    return say


@pytest.mark.timeout(900)
def test_batch_every_graph_against_the_oracle(live):
    """Every graph of the 4096-graph batch (one call on the GPU) against the oracle run on that graph alone:
    digests of every output field, the oracle in worker processes that regenerate each graph from its seed."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor, as_completed
    import oracle_digests
    ce = _ce()
    G, M, seed = 4096, 5, 3
    sizes = synth.batch_sizes(G, seed)
    src, dst, t, eoff, voff = synth.batch_workload(G, seed=seed, sizes=sizes)
    live("batch n=%d: GPU" % len(src))
    br = run_batch(src, dst, t, eoff, voff, M)
    whole = ce.to_numpy(br.result)  # the documented (unsigned) dtypes, as the oracle's
    res = {f: whole[f] for f in FIELDS}
    ro, co = br.row_offsets, br.cluster_offsets
    gpu = []
    for g in range(G):
        e0, e1, r0, r1, c0, c1 = eoff[g], eoff[g + 1], ro[g], ro[g + 1], co[g], co[g + 1]

        def get(f):
            x = res[f]
            if f.startswith(("msf_", "sl_")):
                return x[r0:r1]
            return x[e0:e1] if f in ("pt_cluster", "pt_lambda", "labels") else x[c0:c1]
        gpu.append(oracle_digests.digest_fields(get, br.m[g], br.n_clusters[g], br.n_labels[g]))
        if (g + 1) % 1024 == 0:
            live("digested %d GPU graphs" % (g + 1))
    live("oracle on every graph in 16 processes")
    order = np.argsort(-sizes)  # largest first, so the pool drains evenly
    jobs = [(int(g), int(sizes[g]), seed, M) for g in order]
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1),
                             mp_context=multiprocessing.get_context("spawn")) as ex:
        ref = {}
        for fut in as_completed([ex.submit(oracle_digests.batch_graph_digest, j) for j in jobs]):
            g, dg = fut.result()
            ref[g] = dg
            if len(ref) % 512 == 0:
                live("oracle %d graphs" % len(ref))
    bad = [g for g in range(G) if ref[g] != gpu[g]]
    assert not bad, "graphs differing from the oracle: %s" % bad[:10]
    live("all %d graphs equal the oracle" % G)
