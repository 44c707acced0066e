"""Pins of the oracle's CAUSAL mode (the increment-weighted line graph of
Def. 1, skeleton by Alg. 2 windows), CPU only.

They tie the oracle to the paper's examples and to libraries, not to itself:
the causal rules of the paper's figure (sink, source, wrong order, tip-to-tail),
Table 2's email chain, Thm 2 per vertex (Alg. 2's rows are a minimum spanning
tree of the node-local line graph, checked against scipy), Thm 3 (equal
weight-filtered components of skeleton and line graph, scipy; MSF weight,
networkx), the unique key-minimal forest by exhaustive enumeration, and the
skeleton bound of Alg. 3.
"""
import itertools

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle
from conftest import load_golden


def arcs_as_set(a):
    return set(zip(a["tail"].tolist(), a["head"].tolist(), a["w"].tolist()))


def comps_at(n, rows, omega):
    """Connected components of the records using rows with w <= omega (App. A uses <=)."""
    keep = rows["w"] <= omega
    g = sp.coo_matrix((np.ones(int(keep.sum())), (rows["tail"][keep], rows["head"][keep])), shape=(n, n))
    k, lab = connected_components(g, directed=False)
    return k, lab


def same_partition(a, b):
    return len(set(zip(a.tolist(), b.tolist()))) == len(set(a.tolist())) == len(set(b.tolist()))


def test_figure_rules_sink_source_order_and_increment():
    # sink: two records into vertex 1 are not arcs of each other
    s, d, t = np.array([0, 2], np.int32), np.array([1, 1], np.int32), np.array([0, 5], np.int64)
    assert len(oracle.causal_line_graph(s, d, t)) == 0
    # source: two records out of vertex 1
    s, d = np.array([1, 1], np.int32), np.array([0, 2], np.int32)
    assert len(oracle.causal_line_graph(s, d, t)) == 0
    # tip-to-tail in the wrong order: 1->2 at t=5 then 0->1 at t=9 (the second cannot cause the first)
    s, d, t = np.array([1, 0], np.int32), np.array([2, 1], np.int32), np.array([5, 9], np.int64)
    assert len(oracle.causal_line_graph(s, d, t)) == 0
    # tip-to-tail in order: 0->1 at 5, 1->2 at 9: one arc, weight 4 (the increment)
    t = np.array([9, 5], np.int64)
    assert arcs_as_set(oracle.causal_line_graph(s, d, t)) == {(1, 0, 4)}
    # equal times satisfy the non-strict causality rule
    t = np.array([7, 7], np.int64)
    assert arcs_as_set(oracle.causal_line_graph(s, d, t)) == {(1, 0, 0)}
    # a pair in both directions at equal times: two antiparallel arcs
    s, d, t = np.array([0, 1], np.int32), np.array([1, 0], np.int32), np.array([3, 3], np.int64)
    assert arcs_as_set(oracle.causal_line_graph(s, d, t)) == {(0, 1, 0), (1, 0, 0)}


def test_table2_chain_is_causal_and_gives_the_same_forest():
    s, d, t = load_golden("table2_chain.txt")
    V = int(max(s.max(), d.max()) + 1)
    arcs = oracle.causal_line_graph(s, d, t, V)
    assert arcs_as_set(arcs) == {(0, 1, 1708), (1, 2, 1977), (2, 3, 291), (3, 4, 651)}
    for tier in (0, 1):
        r = oracle.cluster(s, d, t, 2, V, tier=tier, causal=True)
        assert r.m == 4 and int(r.msf_w.sum()) == 4627
        assert list(r.msf_w) == [291, 651, 1708, 1977]
        assert list(r.sl_w) == [291, 651, 1708, 1977]


def test_window_rule_hand_example():
    """Vertex 9 sees, in time order: in a (t=1), in b (t=2), out x (t=3), out y (t=5), in c (t=6), out z (t=8).
    Alg. 2: x links to the window {a, b}; y to the carried {b}; z to {b, c} (b carried, c new)."""
    # records: a=0: 1->9 @1, b=1: 2->9 @2, x=2: 9->3 @3, y=3: 9->4 @5, c=4: 5->9 @6, z=5: 9->6 @8
    s = np.array([1, 2, 9, 9, 5, 9], np.int32)
    d = np.array([9, 9, 3, 4, 9, 6], np.int32)
    t = np.array([1, 2, 3, 5, 6, 8], np.int64)
    sk = oracle.causal_skeleton(s, d, t, 10)
    assert arcs_as_set(sk) == {(0, 2, 2), (1, 2, 1), (1, 3, 3), (1, 5, 6), (4, 5, 2)}
    full = oracle.causal_line_graph(s, d, t, 10)
    assert len(full) == 7  # every in-edge with every later out-edge: a and b with x, y, z; c with z
    assert len(sk) <= 6 - 1


def test_equal_times_put_in_edges_first():
    """At equal times an in-edge precedes an out-edge (the ordering the proof's perturbation gives), so
    an out-edge at the same second still links to it."""
    s = np.array([9, 1], np.int32)   # record 0 leaves 9, record 1 arrives at 9, both at t = 4
    d = np.array([2, 9], np.int32)
    t = np.array([4, 4], np.int64)
    assert arcs_as_set(oracle.causal_skeleton(s, d, t, 10)) == {(1, 0, 0)}


def _random_graph(rng, n, V, tmax):
    s = rng.integers(0, V, n).astype(np.int32)
    d = rng.integers(0, V, n).astype(np.int32)
    bad = s == d
    d[bad] = (s[bad] + 1 + rng.integers(0, V - 1, bad.sum())) % V
    return s, d, rng.integers(0, tmax, n).astype(np.int64)


def test_thm2_alg2_is_a_local_mst_scipy():
    """Per vertex, the Alg. 2 rows form a spanning forest of the node-local line graph with the minimum
    total weight (scipy), as Thm 2 states."""
    rng = np.random.default_rng(5)
    for trial in range(300):
        n = int(rng.integers(2, 30))
        V = int(rng.integers(2, 5))
        s, d, t = _random_graph(rng, n, V, int(rng.choice([3, 20, 1000])))
        for x in range(V):
            ins = [r for r in range(n) if d[r] == x]
            outs = [q for q in range(n) if s[q] == x]
            local = [(r, q, int(t[q] - t[r])) for r in ins for q in outs if t[r] <= t[q]]
            # restrict the skeleton to rows made at x: tail arrives at x, head leaves x
            sk = [(a, b, w) for a, b, w in zip(*[oracle.causal_skeleton(s, d, t, V)[f].tolist()
                                                  for f in ("tail", "head", "w")]) if d[a] == x and s[b] == x]
            nodes = sorted(set(ins) | set(outs))
            if not nodes:
                continue
            idx = {v: i for i, v in enumerate(nodes)}
            g = nx.Graph()
            g.add_nodes_from(range(len(nodes)))
            for a, b, w in local:
                if not g.has_edge(idx[a], idx[b]) or g[idx[a]][idx[b]]["weight"] > w:
                    g.add_edge(idx[a], idx[b], weight=w)
            mst_w = sum(e[2]["weight"] for e in nx.minimum_spanning_edges(g, data=True))
            f = nx.Graph()
            f.add_nodes_from(range(len(nodes)))
            f.add_edges_from((idx[a], idx[b]) for a, b, _ in sk)
            assert nx.is_forest(f), trial
            assert nx.number_connected_components(f) == nx.number_connected_components(g), trial
            assert sum(w for _, _, w in sk) == mst_w, (trial, x)


def test_thm3_equal_filtered_components_and_msf_weight():
    """Skeleton and full causal line graph have the same components at every threshold (<=), the same MSF
    weight (scipy), and the skeleton obeys the bound of Alg. 3 (sum over vertices of |E_i| - 1)."""
    rng = np.random.default_rng(8)
    for trial in range(200):
        n = int(rng.integers(2, 60))
        V = int(rng.integers(2, 9))
        s, d, t = _random_graph(rng, n, V, int(rng.choice([4, 30, 5000])))
        full = oracle.causal_line_graph(s, d, t, V)
        sk = oracle.causal_skeleton(s, d, t, V)
        deg = np.bincount(s, minlength=V) + np.bincount(d, minlength=V)
        assert len(sk) <= int(np.maximum(deg - 1, 0).sum())
        assert arcs_as_set(sk) <= arcs_as_set(full)
        for omega in sorted(set(full["w"].tolist()) | {0}):
            ka, la = comps_at(n, full, omega)
            kb, lb = comps_at(n, sk, omega)
            assert ka == kb and same_partition(la, lb), (trial, omega)
        a = oracle.cluster(s, d, t, 2, V, tier=0, causal=True)
        b = oracle.cluster(s, d, t, 2, V, tier=1, causal=True)
        assert a.m == b.m and int(a.msf_w.sum()) == int(b.msf_w.sum())
        if len(full):
            g = nx.Graph()
            g.add_nodes_from(range(n))
            for x in full:
                u, v, w = int(x["tail"]), int(x["head"]), int(x["w"])
                if not g.has_edge(u, v) or g[u][v]["weight"] > w:
                    g.add_edge(u, v, weight=w)
            assert int(a.msf_w.sum()) == sum(e[2]["weight"] for e in nx.minimum_spanning_edges(g, data=True))


def _key(e):
    return (int(e["w"]), int(e["head"]), -int(e["tail"]))


def test_exhaustive_small_graphs_tiers_agree_and_forest_is_key_minimal():
    """Every multigraph with V = 3, n <= 3, t in {0,1,2}: the Alg. 2 skeleton gives byte-identical results to
    the full causal line graph, and the MSF is the key-minimal spanning forest over all spanning forests."""
    pairs = [(a, b) for a in range(3) for b in range(3) if a != b]
    done = 0
    for n in (1, 2, 3):
        for es in itertools.product(pairs, repeat=n):
            for ts in itertools.product(range(3), repeat=n):
                s = np.array([e[0] for e in es], np.int32)
                d = np.array([e[1] for e in es], np.int32)
                t = np.array(ts, np.int64)
                a = oracle.cluster(s, d, t, 2, 3, tier=0, causal=True)
                b = oracle.cluster(s, d, t, 2, 3, tier=1, causal=True)
                for f in a._fields:
                    x, y = getattr(a, f), getattr(b, f)
                    assert np.array_equal(np.asarray(x), np.asarray(y)), (es, ts, f)
                full = oracle.causal_line_graph(s, d, t, 3)
                if 0 < len(full) <= 10:
                    mine = sorted(_key(e) for e in zip_rows(a))
                    g = nx.MultiGraph()
                    g.add_nodes_from(range(n))
                    idx = list(range(len(full)))
                    k_best = None
                    ncomp = None
                    for r in range(len(full) + 1):
                        for sub in itertools.combinations(idx, r):
                            h = nx.MultiGraph()
                            h.add_nodes_from(range(n))
                            h.add_edges_from((int(full[i]["tail"]), int(full[i]["head"])) for i in sub)
                            if not nx.is_forest(nx.Graph(h)) or h.number_of_edges() != nx.Graph(h).number_of_edges():
                                continue
                            c = nx.number_connected_components(h)
                            keys = sorted(_key(full[i]) for i in sub)
                            if ncomp is None or c < ncomp or (c == ncomp and keys < k_best):
                                ncomp, k_best = c, keys
                    assert mine == k_best, (es, ts)
                done += 1
    assert done == 6 * 3 + 36 * 9 + 216 * 27


def zip_rows(r):
    out = np.empty(r.m, dtype=oracle.LG_EDGE)
    out["tail"], out["head"], out["w"] = r.msf_tail, r.msf_head, r.msf_w
    return out


@pytest.mark.slow
def test_exhaustive_four_records_sampled():
    pairs = [(a, b) for a in range(3) for b in range(3) if a != b]
    rng = np.random.default_rng(2)
    for _ in range(3000):
        es = [pairs[i] for i in rng.integers(0, len(pairs), 4)]
        ts = rng.integers(0, 3, 4)
        s = np.array([e[0] for e in es], np.int32)
        d = np.array([e[1] for e in es], np.int32)
        t = np.array(ts, np.int64)
        a = oracle.cluster(s, d, t, 2, 3, tier=0, causal=True)
        b = oracle.cluster(s, d, t, 2, 3, tier=1, causal=True)
        for f in a._fields:
            assert np.array_equal(np.asarray(getattr(a, f)), np.asarray(getattr(b, f))), (es, ts, f)


def test_random_tie_heavy_tiers_agree():
    rng = np.random.default_rng(13)
    for trial in range(300):
        n = int(rng.integers(1, 80))
        V = int(rng.integers(2, 10))
        s, d, t = _random_graph(rng, n, V, int(rng.choice([2, 5, 100])))
        for M in (2, 3):
            a = oracle.cluster(s, d, t, M, V, tier=0, causal=True)
            b = oracle.cluster(s, d, t, M, V, tier=1, causal=True)
            for f in a._fields:
                assert np.array_equal(np.asarray(getattr(a, f)), np.asarray(getattr(b, f))), (trial, M, f)
