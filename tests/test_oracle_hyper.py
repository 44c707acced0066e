"""Pins of the oracle's dynamic-hypergraph mode (Sec. 5.3), CPU only.

* A hypergraph whose hyperedges are pairs {i, j} is a graph: every output equals
  the graph oracle's (whose own pins are independent of this code).
* Exhaustive: every hypergraph with V = 3, n <= 3 hyperedges (each any subset of
  {0,1,2}, the empty one included) and t in {0,1,2} gives byte-identical results
  from the definition tier (all meeting pairs) and the skeleton tier (per-vertex
  time-sorted paths), and the forest weight is the minimum over all spanning
  forests of the line graph built here from set intersections.
* Random hypergraphs: the two tiers agree on every field (with and without a
  time cutoff); the forest weight equals networkx's MST of the line graph built
  in Python from set intersections; the skeleton and the full line graph have
  the same weight-filtered components at every threshold (Thm 3 for
  hypergraphs); the skeleton has exactly sum_i (d_i - 1) rows, at most the input
  size (the bound of Sec. 5.3).
* A vertex listed twice in one hyperedge counts once; empty hyperedges are
  isolated nodes; a hand-worked example; argument errors.
"""
import itertools

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle

FIELDS = ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster", "pt_lambda",
          "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected", "labels")


def same(a, b):
    assert (a.status, a.m, a.n_clusters, a.n_labels) == (b.status, b.m, b.n_clusters, b.n_labels)
    for f in FIELDS:
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


def csr(sets):
    off = np.zeros(len(sets) + 1, np.int64)
    for r, S in enumerate(sets):
        off[r + 1] = off[r] + len(S)
    mem = np.array([v for S in sets for v in S], np.int32)
    return mem, off


def random_hyper(rng, n, V, tmax, dmax=6, dup=True):
    sets = []
    for _ in range(n):
        k = int(rng.integers(0, dmax + 1))
        S = [int(x) for x in rng.integers(0, V, k)]
        if dup and S and rng.random() < 0.2:
            S.append(S[0])  # a vertex listed twice
        sets.append(S)
    t = rng.integers(0, tmax, n).astype(np.int64)
    return sets, t


def py_line_graph(sets, t):
    """Line-graph edges from set intersections: (a, b, |t_a - t_b|) for a < b."""
    out = []
    ss = [set(S) for S in sets]
    for a in range(len(sets)):
        for b in range(a + 1, len(sets)):
            if ss[a] & ss[b]:
                out.append((a, b, abs(int(t[a]) - int(t[b]))))
    return out


def test_pairs_reduce_to_the_graph_oracle():
    rng = np.random.default_rng(61)
    for trial in range(200):
        n = int(rng.integers(1, 80))
        V = int(rng.integers(2, 12))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V - 1, n).astype(np.int32)
        d[d >= s] += 1
        t = rng.integers(0, int(rng.choice([5, 100, 10 ** 5])), n).astype(np.int64)
        mem, off = csr([[int(a), int(b)] for a, b in zip(s, d)])
        M = int(rng.choice([2, 3, 5]))
        for tier in (0, 1):
            same(oracle.cluster_hyper(mem, off, t, M, V, tier=tier), oracle.cluster(s, d, t, M, V, tier=tier))


def test_exhaustive_tiny_hypergraphs():
    subsets = [list(c) for k in range(4) for c in itertools.combinations(range(3), k)]  # 8, the empty set first
    checked = 0
    for n in range(1, 4):
        for sets in itertools.product(subsets, repeat=n):
            for t in itertools.product(range(3), repeat=n):
                t = np.array(t, np.int64)
                mem, off = csr(sets)
                a = oracle.cluster_hyper(mem, off, t, 2, 3, tier=0)
                b = oracle.cluster_hyper(mem, off, t, 2, 3, tier=1)
                same(a, b)
                # the forest weight is the minimum over all spanning forests
                edges = py_line_graph(sets, t)
                best = None
                for k in range(len(edges) + 1):
                    for sub in itertools.combinations(edges, k):
                        g = nx.Graph()
                        g.add_nodes_from(range(n))
                        g.add_edges_from((x, y) for x, y, _ in sub)
                        if len(sub) != n - nx.number_connected_components(g) or not nx.is_forest(g):
                            continue
                        if nx.number_connected_components(g) != _components(n, edges):
                            continue
                        w = sum(z for _, _, z in sub)
                        best = w if best is None else min(best, w)
                assert int(a.msf_w.sum()) == (best or 0)
                checked += 1
    assert checked == 24 + 24 ** 2 + 24 ** 3


def _components(n, edges):
    g = nx.Graph()
    g.add_nodes_from(range(n))
    g.add_edges_from((x, y) for x, y, _ in edges)
    return nx.number_connected_components(g)


def test_random_hypergraphs_tiers_networkx_and_thresholds():
    rng = np.random.default_rng(67)
    for trial in range(120):
        n = int(rng.integers(1, 90))
        V = int(rng.integers(1, 15))
        sets, t = random_hyper(rng, n, V, int(rng.choice([4, 60, 10 ** 4])))
        mem, off = csr(sets)
        M = int(rng.choice([2, 3, 4]))
        a = oracle.cluster_hyper(mem, off, t, M, V, tier=0)
        b = oracle.cluster_hyper(mem, off, t, M, V, tier=1)
        same(a, b)
        cut = int(rng.choice([0, 3, 50]))
        same(oracle.cluster_hyper(mem, off, t, M, V, tier=0, max_dt=cut),
             oracle.cluster_hyper(mem, off, t, M, V, tier=1, max_dt=cut))
        edges = py_line_graph(sets, t)
        g = nx.Graph()
        g.add_nodes_from(range(n))
        for x, y, w in edges:
            g.add_edge(x, y, weight=w)
        mst = nx.minimum_spanning_tree(g)
        assert int(b.msf_w.sum()) == int(sum(d["weight"] for _, _, d in mst.edges(data=True)))
        assert b.m == n - nx.number_connected_components(g)
        # Thm 3 for hypergraphs: equal weight-filtered components of skeleton and full line graph
        sk = oracle.hyper_skeleton(mem, off, t, V)
        full = np.array(edges, dtype=[("tail", "<i8"), ("head", "<i8"), ("w", "<i8")]) if edges else None
        for thr in sorted({0, 1, 5, 60, 1 << 20} | {int(w) for w in sk["w"][:5]}):
            ks = sk["w"] <= thr
            g1 = sp.coo_matrix((np.ones(int(ks.sum())), (sk["tail"][ks], sk["head"][ks])), shape=(n, n))
            _, l1 = connected_components(g1, directed=False)
            if full is not None:
                kf = full["w"] <= thr
                g2 = sp.coo_matrix((np.ones(int(kf.sum())), (full["tail"][kf], full["head"][kf])), shape=(n, n))
            else:
                g2 = sp.coo_matrix((n, n))
            _, l2 = connected_components(g2, directed=False)
            # same partition: the label maps are bijective
            pairs = set(zip(l1.tolist(), l2.tolist()))
            assert len(pairs) == len(set(l1.tolist())) == len(set(l2.tolist())), (trial, thr)
        # the bound of Sec. 5.3
        deg = np.zeros(max(V, 1), np.int64)
        for S in sets:
            for v in set(S):
                deg[v] += 1
        assert len(sk) == int(np.sum(np.maximum(deg - 1, 0))) <= len(mem)


def test_repeated_members_and_empty_hyperedges():
    rng = np.random.default_rng(71)
    for trial in range(60):
        sets, t = random_hyper(rng, int(rng.integers(1, 60)), 8, 100, dup=False)
        mem, off = csr(sets)
        base = oracle.cluster_hyper(mem, off, t, 3, 8)
        doubled = [S + S[: len(S) // 2] for S in sets]
        mem2, off2 = csr(doubled)
        same(oracle.cluster_hyper(mem2, off2, t, 3, 8), base)
        # an empty hyperedge is a node without neighbours: it never appears in a row
        for r, S in enumerate(sets):
            if not S:
                assert r not in set(base.msf_tail.tolist()) | set(base.msf_head.tolist())


def test_hand_worked_example():
    """{0,1,2}@0, {2,3}@10, {3,4,5}@15, {6}@5, {}@7: rows (1->2, w 5) then (0->1, w 10); 3 and 4 isolated."""
    mem, off = csr([[0, 1, 2], [2, 3], [3, 4, 5], [6], []])
    t = np.array([0, 10, 15, 5, 7], np.int64)
    for tier in (0, 1):
        r = oracle.cluster_hyper(mem, off, t, 2, 7, tier=tier)
        assert r.m == 2
        assert list(r.msf_tail) == [1, 0] and list(r.msf_head) == [2, 1] and list(r.msf_w) == [5, 10]
        assert list(r.sl_left) == [1, 0] and list(r.sl_right) == [2, 5] and list(r.sl_size) == [2, 3]
    # with M = 2 the only big component continues ROOT and both splits shed: all noise
    assert list(r.labels) == [-1] * 5
    # hyperedges 1 and 2 share vertex 3 only; 0 and 1 share vertex 2 only
    sk = oracle.hyper_skeleton(mem, off, t, 7)
    assert sorted((int(e["tail"]), int(e["head"]), int(e["w"])) for e in sk) == [(0, 1, 10), (1, 2, 5)]


def test_argument_errors():
    t = np.array([0, 1], np.int64)
    mem = np.array([0, 1, 1], np.int32)
    assert oracle.hyper_validate(mem, np.array([0, 2, 3]), t, 2) == oracle.OK
    assert oracle.hyper_validate(mem, np.array([1, 2, 3]), t, 2) == oracle.EINVAL
    assert oracle.hyper_validate(mem, np.array([0, 3, 2]), t, 2) == oracle.EINVAL
    assert oracle.hyper_validate(np.array([0, 1, 2], np.int32), np.array([0, 2, 3]), t, 2) == oracle.ERANGE
    assert oracle.hyper_validate(np.array([0, -1, 1], np.int32), np.array([0, 2, 3]), t, 2) == oracle.ERANGE
    r = oracle.cluster_hyper(mem, np.array([0, 3, 2]), t, 2, 2)
    assert r.status == oracle.EINVAL


def test_discrete_on_hypergraphs_is_per_level_components():
    from test_oracle_discrete import d_from_components, d_from_oracle
    rng = np.random.default_rng(73)
    for trial in range(60):
        n = int(rng.integers(2, 50))
        sets, t = random_hyper(rng, n, 6, int(rng.choice([10, 500])))
        mem, off = csr(sets)
        thr = np.unique(rng.integers(0, 300, int(rng.integers(1, 6))))
        r, dl, dt = oracle.cluster_hyper_discrete(mem, off, t, 2, thr, 6)
        assert r.status == 0
        edges = oracle.hyper_line_graph(mem, off, t, 6)
        assert d_from_oracle(n, r, dl, dt) == d_from_components(n, edges, thr), trial
