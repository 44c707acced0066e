"""GPU parity of ce_level_components (Alg. 5 by one connected-components pass
per threshold) against the oracle's per-level components, and a GPU cross-check
of the two ways to the discrete dendrogram: the discrete nodes read off these
per-level components equal those of the dendrogram the clustering call cuts
from the exact one (dd_level / dd_top)."""
import os
import sys
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
import synth
from test_oracle_discrete import d_from_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PAPER = [1 << k for k in range(29)]


def _ce():
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.fail("libce.so is not built")
    return ce


def note(msg):
    print("[gpu-levels] " + msg, flush=True)
    sys.stdout.flush()


def dev(*arrays):
    d = torch.device("cuda:0")
    return [torch.from_numpy(np.ascontiguousarray(a)).to(d) for a in arrays]


def gpu_forest(src, dst, t, V, causal=False, thresholds=None):
    ce = _ce()
    s, d, tt = dev(src.astype(np.int32), dst.astype(np.int32), t.astype(np.int64))
    return ce.cluster_edges(s, d, tt, 2, V, causal=causal, thresholds=thresholds)


def gpu_levels(res, n, thr):
    ce = _ce()
    return ce.level_components(res.msf_tail, res.msf_head, res.msf_w, n, thr).cpu().numpy()


def oracle_levels(src, dst, t, thr, causal=False):
    sk = (oracle.causal_skeleton if causal else oracle.skeleton)(src, dst, t)
    return oracle.level_components(len(t), sk["tail"], sk["head"], sk["w"], thr)


def check(src, dst, t, V, thr, label, causal=False):
    note("%s n=%d levels=%d causal=%s" % (label, len(t), len(thr), causal))
    res = gpu_forest(src, dst, t, V, causal)
    got = gpu_levels(res, len(t), thr)
    ref = oracle_levels(src, dst, t, thr, causal)
    if not np.array_equal(got, ref):
        l, r = np.argwhere(got != ref)[0]
        # which side: the forest rows, or the components computed from them
        mt, mh, mw = (x.cpu().numpy() for x in (res.msf_tail, res.msf_head, res.msf_w))
        own = oracle.level_components(len(t), mt.view(np.uint32), mh.view(np.uint32), mw, thr)
        o = oracle.cluster(src, dst, t, 2, V, tier=1, causal=causal)
        same_rows = (np.array_equal(mt.view(np.uint32), o.msf_tail) and np.array_equal(mh.view(np.uint32), o.msf_head)
                     and np.array_equal(mw, o.msf_w))
        raise AssertionError("%s: level %d record %d: %d vs %d; forest rows equal the oracle's: %s; components of "
                             "the GPU rows equal the GPU labels: %s (%d of %d labels differ)"
                             % (label, l, r, got[l, r], ref[l, r], same_rows, np.array_equal(own, got),
                                int((got != ref).sum()), got.size))
    return got


def d_from_labels(lab):
    """Discrete nodes from per-level smallest-member labels: a component of two or more records that did not
    exist one level lower, keyed (level, smallest member, size), with the key of the node it first grows into."""
    q, n = lab.shape
    sizes = [np.bincount(lab[i], minlength=n) for i in range(q)]
    nodes = {}
    for i in range(q):
        for c in np.nonzero(sizes[i] >= 2)[0]:
            c = int(c)
            if i > 0 and sizes[i - 1][lab[i - 1][c]] == sizes[i][c]:
                continue
            nodes[(i, c, int(sizes[i][c]))] = None
    for (i, c, sz) in list(nodes):
        for j in range(i + 1, q):
            cj = int(lab[j][c])
            if sizes[j][cj] != sz:
                nodes[(i, c, sz)] = (j, cj, int(sizes[j][cj]))
                break
    return nodes


def test_hand_star():
    src = np.zeros(4, np.int32)
    dst = np.arange(1, 5, dtype=np.int32)
    t = np.array([0, 1, 10, 11], np.int64)
    got = check(src, dst, t, 5, [0, 1, 5, 9, 100], "star")
    assert got.tolist() == [[0, 1, 2, 3], [0, 0, 2, 2], [0, 0, 2, 2], [0, 0, 0, 0], [0, 0, 0, 0]]


@pytest.mark.parametrize("causal", [False, True])
def test_random_graphs(causal):
    rng = np.random.default_rng(223 if causal else 227)
    for k in range(40):
        n = int(rng.integers(2, 3000))
        V = int(rng.integers(2, 300))
        src, dst, t = synth.chung_lu_bursts(n, V, int(rng.integers(1, 1 << 30)))
        thr = np.unique(rng.integers(0, 20000, int(rng.integers(1, 12))))
        check(src, dst, t, V, thr, "random%d" % k, causal)


def test_hypergraph():
    import test_gpu_hyper as hyper
    ce = _ce()
    rng = np.random.default_rng(229)
    for k in range(10):
        n = int(rng.integers(2, 2000))
        V = int(rng.integers(2, 200))
        mem, off = hyper.csr(hyper.random_sets(rng, n, V, 5))
        t = rng.integers(0, 5000, n).astype(np.int64)
        thr = np.unique(rng.integers(0, 3000, 6))
        note("hyper%d n=%d" % (k, n))
        res = ce.cluster_hyperedges(*hyper.dev(mem, off, t), 2, V)
        got = gpu_levels(res, n, thr)
        sk = oracle.hyper_skeleton(mem, off, t)
        ref = oracle.level_components(n, sk["tail"], sk["head"], sk["w"], thr)
        assert np.array_equal(got, ref), k


def test_one_graph_of_a_batch():
    """The rows of graph g of a batch (local ids, contiguous) give that graph's levels."""
    import test_gpu_batch as batch
    ce = _ce()
    rng = np.random.default_rng(239)
    graphs = []
    for g in range(12):
        s, d, t, V = synth.batch_graph(g, int(rng.integers(1, 4000)), seed=17)
        graphs.append((s, d, t, V))
    src, dst, t, eoff, voff = batch.pack(graphs)
    note("batch of %d graphs n=%d" % (len(graphs), len(src)))
    br = batch.run_batch(src, dst, t, eoff, voff, 5)
    thr = [0, 60, 3600, 86400]
    for g, (s, d, tt, V) in enumerate(graphs):
        r0, r1 = int(br.row_offsets[g]), int(br.row_offsets[g + 1])
        res = br.result
        got = ce.level_components(res.msf_tail[r0:r1], res.msf_head[r0:r1], res.msf_w[r0:r1], len(tt),
                                  thr).cpu().numpy()
        assert np.array_equal(got, oracle_levels(s, d, tt, thr)), g


def test_same_discrete_nodes_as_the_cut_dendrogram():
    ce = _ce()
    rng = np.random.default_rng(233)
    for k in range(16):
        causal = bool(k & 1)
        n = int(rng.integers(10, 1500))
        V = int(rng.integers(2, 120))
        src, dst, t = synth.chung_lu_bursts(n, V, int(rng.integers(1, 1 << 30)))
        thr = sorted(set(int(x) for x in rng.integers(0, 5000, int(rng.integers(1, 8)))))
        note("cut vs components %d n=%d causal=%s" % (k, n, causal))
        res = gpu_forest(src, dst, t, V, causal, thresholds=thr)
        r = ce.to_numpy(res)
        # the cut dendrogram holds the rows up to the last threshold; components need the whole forest
        full = gpu_forest(src, dst, t, V, causal)
        lab = gpu_levels(full, n, thr)
        cut = d_from_oracle(n, SimpleNamespace(m=r["m"], sl_left=r["sl_left"], sl_right=r["sl_right"],
                                               sl_size=r["sl_size"]), r["dd_level"], r["dd_top"])
        assert cut == d_from_labels(lab), k


def test_tiny_workload_paper_thresholds():
    w = synth.plain_tiny()
    check(w.src, w.dst, w.t, w.num_vertices, PAPER, "tiny, 2^0 .. 2^28")
    check(w.src, w.dst, w.t, w.num_vertices, PAPER, "tiny causal, 2^0 .. 2^28", causal=True)


@pytest.mark.timeout(600)
def test_rmat_hawkes_scaled_paper_thresholds():
    src, dst, t = synth.rmat_hawkes(2_000_000, 17, seed=11)
    check(src, dst, t, 1 << 17, PAPER, "rmat 2M, 2^0 .. 2^28")


def test_each_level_alone():
    """One level per call puts all of a level's rows into one union launch (many concurrent hooks and finds),
    then one compression: labels must still be exact smallest members, not intermediate ancestors."""
    ce = _ce()
    src, dst, t = synth.rmat_hawkes(400_000, 14, seed=13)
    res = gpu_forest(src, dst, t, 1 << 14)
    n = len(t)
    thr = [1, 30, 300, 3000, 30000, 300000, 3000000]
    ref = oracle_levels(src, dst, t, thr)
    for i, w in enumerate(thr):
        note("single level %d n=%d" % (w, n))
        got = ce.level_components(res.msf_tail, res.msf_head, res.msf_w, n, [w]).cpu().numpy()[0]
        assert np.array_equal(got, ref[i]), (w, int((got != ref[i]).sum()))


def test_errors_and_reuse():
    ce = _ce()
    w = synth.plain_tiny()
    res = gpu_forest(w.src, w.dst, w.t, w.num_vertices)
    n = len(w.t)
    note("errors n=%d" % n)
    with pytest.raises(ce.ClusterError) as ei:
        ce.level_components(res.msf_tail, res.msf_head, res.msf_w, n - 1000, [5])
    assert ei.value.status == ce.CE_ERANGE
    shuffled = res.msf_w.flip(0).contiguous()
    with pytest.raises(ce.ClusterError) as ei:
        ce.level_components(res.msf_tail, res.msf_head, shuffled, n, [5])
    assert ei.value.status == ce.CE_EINVAL
    with pytest.raises(ce.ClusterError):
        ce.level_components(res.msf_tail, res.msf_head, res.msf_w, n, [5, 5])
    # a preallocated buffer, reused with fewer levels
    buf = torch.full((3 * n,), -7, dtype=torch.int32, device="cuda:0")
    a = ce.level_components(res.msf_tail, res.msf_head, res.msf_w, n, [10, 100, 1000], labels=buf).cpu().numpy()
    b = ce.level_components(res.msf_tail, res.msf_head, res.msf_w, n, [100], labels=buf).cpu().numpy()
    assert np.array_equal(b[0], a[1])
    ref = oracle_levels(w.src, w.dst, w.t, [10, 100, 1000])
    assert np.array_equal(a, ref)
    # no rows: every record alone
    e = torch.empty(0, dtype=torch.int32, device="cuda:0")
    lab = ce.level_components(e, e, torch.empty(0, dtype=torch.int64, device="cuda:0"), 5, [0, 3]).cpu().numpy()
    assert lab.tolist() == [list(range(5))] * 2
