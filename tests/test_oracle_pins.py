"""Pins of the CPU oracle to things other than itself (no GPU needed).

Each test checks the oracle against what the paper or the mathematics fixes:
printed worked examples, exhaustive enumeration on tiny inputs, closed forms,
third-party library routines (networkx, scipy, scikit-learn), and invariants of
the paper's theorems. The helpers below are written independently of the
oracle's C code.
"""
import itertools
import os

import networkx as nx
import numpy as np
import pytest
import scipy.cluster.hierarchy as sch
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, minimum_spanning_tree

import oracle
from conftest import load_golden

LAM_ONE = 1 << 63


def lam(w):
    """Fixed-point lambda of the reading: floor(2^63 / max(2w, 1))."""
    return LAM_ONE // max(2 * int(w), 1)


# ----------------------------------------------------------------- helpers
def lg_pairs_py(src, dst, t):
    """Undirected line graph by brute force over all record pairs (Sec. 1.2.2):
    records a<b are adjacent iff they share a vertex; weight |t_a - t_b|."""
    n = len(src)
    out = []
    for a in range(n):
        ea = {int(src[a]), int(dst[a])}
        for b in range(a + 1, n):
            if ea & {int(src[b]), int(dst[b])}:
                out.append((a, b, abs(int(t[a]) - int(t[b]))))
    return out


def key_of(a, b, t):
    """Canonical key of the reading: (w, head, -tail), head = later record by (t, id)."""
    ta, tb = (int(t[a]), a), (int(t[b]), b)
    tail, head = (a, b) if ta < tb else (b, a)
    return (abs(int(t[a]) - int(t[b])), head, -tail)


def components_count(n, edges):
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    c = n
    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
            c -= 1
    return c


def is_acyclic(n, edges):
    return components_count(n, edges) == n - len(edges)


def msf_as_pairs(r):
    return sorted((int(a), int(b)) if a < b else (int(b), int(a)) for a, b in zip(r.msf_tail, r.msf_head))


def assert_same_result(a, b):
    assert a.status == b.status
    for f in oracle.Result._fields:
        x, y = getattr(a, f), getattr(b, f)
        if isinstance(x, np.ndarray):
            assert np.array_equal(x, y), f
        else:
            assert x == y, f


def minimax_matrix(n, pairs):
    """Single-linkage (minimax path) distances via scipy's MST of the full line graph.
    Weights are shifted by +1 because scipy treats explicit zeros as absent."""
    if not pairs:
        return None
    r = np.array([p[0] for p in pairs])
    c = np.array([p[1] for p in pairs])
    w = np.array([p[2] for p in pairs], dtype=np.float64) + 1.0
    T = minimum_spanning_tree(sp.coo_matrix((w, (r, c)), shape=(n, n))).tocoo()
    adj = [[] for _ in range(n)]
    for a, b, ww in zip(T.row, T.col, T.data):
        adj[a].append((b, ww - 1.0))
        adj[b].append((a, ww - 1.0))
    D = np.full((n, n), np.inf)
    for s in range(n):
        D[s, s] = 0.0
        stack = [(s, 0.0)]
        seen = {s}
        while stack:
            x, mx = stack.pop()
            for y, ww in adj[x]:
                if y not in seen:
                    seen.add(y)
                    D[s, y] = max(mx, ww)
                    stack.append((y, max(mx, ww)))
    return D


# ------------------------------------------------------- printed examples
def test_table2_chain_msf_and_dendrogram():
    """Table 2 (Sec. 4.1): the five-email chain. Gaps 1708, 1977, 291, 651 s
    (hand-computed from the printed times); MSF weight 4627."""
    src, dst, t = load_golden("table2_chain.txt")
    for tier in (0, 1):
        r = oracle.cluster(src, dst, t, 2, tier=tier)
        assert r.status == 0 and r.m == 4
        assert list(r.msf_w) == [291, 651, 1708, 1977]
        assert int(r.msf_w.sum()) == 4627
        # merge order: (3,4) at 291; +record 4 (node with 2) at 651; (0,1) at 1708; both at 1977
        assert list(r.sl_w) == [291, 651, 1708, 1977]
        assert [(int(a), int(b)) for a, b in zip(r.sl_left, r.sl_right)] == [(2, 3), (4, 5), (0, 1), (6, 7)]
        assert list(r.sl_size) == [2, 3, 2, 5]
    # reading: a standalone component is never labelled on its own (allow_single_cluster off)
    r = oracle.cluster(src, dst, t, 5, tier=0)
    assert (r.labels == -1).all() and r.n_labels == 0
    # the path has 2n - V' = 10 - 6 = 4 skeleton rows
    assert oracle.skeleton(src, dst, t).size == 4


def test_table3_long_cluster_tiers_agree_and_weight():
    """Table 3 (Sec. 4.1): eleven emails among three people; all records share
    vertices, so the line graph is connected; MSF weight equals networkx's MST."""
    src, dst, t = load_golden("table3_long.txt")
    a = oracle.cluster(src, dst, t, 3, tier=0)
    b = oracle.cluster(src, dst, t, 3, tier=1)
    assert_same_result(a, b)
    assert a.m == 10
    G = nx.Graph()
    G.add_nodes_from(range(11))
    for x, y, w in lg_pairs_py(src, dst, t):
        G.add_edge(x, y, weight=w)
    assert int(a.msf_w.sum()) == int(nx.minimum_spanning_tree(G).size(weight="weight"))
    # the first record is ten days before the rest: it joins last, at the largest weight
    assert int(a.sl_w[-1]) == int(t[1] - t[0]) and int(a.sl_size[-1]) == 11


# --------------------------------------------------- exhaustive enumeration
def _check_exhaustive(src, dst, t):
    n = len(src)
    pairs = lg_pairs_py(src, dst, t)
    a = oracle.cluster(src, dst, t, 2, num_vertices=3, tier=0)
    b = oracle.cluster(src, dst, t, 2, num_vertices=3, tier=1)
    assert_same_result(a, b)
    # spanning forests: acyclic edge sets with n - c edges
    c = components_count(n, [(x, y) for x, y, _ in pairs])
    k = n - c
    keys = {(x, y): key_of(x, y, t) for x, y, _ in pairs}
    best = None
    minw = None
    for sub in itertools.combinations([(x, y) for x, y, _ in pairs], k):
        if not is_acyclic(n, sub):
            continue
        ks = sorted(keys[e] for e in sub)
        if best is None or ks < best[0]:
            best = (ks, sorted(sub))
        w = sum(kk[0] for kk in ks)
        minw = w if minw is None else min(minw, w)
    assert a.m == k
    got = msf_as_pairs(a)
    assert got == best[1]
    assert int(a.msf_w.sum()) == (minw if minw is not None else 0)


def _all_graphs(nmax, times=(0, 1, 2), V=3):
    types = [(s, d, tt) for s in range(V) for d in range(V) if s != d for tt in times]
    for n in range(1, nmax + 1):
        for recs in itertools.product(types, repeat=n):
            yield recs


def test_exhaustive_graph_space_up_to_three_records():
    """Every multigraph with V=3, n<=3, t in {0,1,2}: Tier A (definition) and
    Tier B (skeleton) agree byte for byte, and the MSF is the key-minimal
    spanning forest found by enumerating all spanning forests."""
    cnt = 0
    for recs in _all_graphs(3):
        a = np.array(recs, dtype=np.int64)
        _check_exhaustive(a[:, 0].astype(np.int32), a[:, 1].astype(np.int32), a[:, 2])
        cnt += 1
    assert cnt == 18 + 18 ** 2 + 18 ** 3


def test_exhaustive_graph_space_four_records_sampled():
    """n=4 records: a fixed random sample of 3000 of the 18^4 graphs."""
    rng = np.random.default_rng(12345)
    types = [(s, d, tt) for s in range(3) for d in range(3) if s != d for tt in (0, 1, 2)]
    for _ in range(3000):
        recs = [types[i] for i in rng.integers(0, len(types), 4)]
        a = np.array(recs, dtype=np.int64)
        _check_exhaustive(a[:, 0].astype(np.int32), a[:, 1].astype(np.int32), a[:, 2])


@pytest.mark.slow
def test_exhaustive_graph_space_four_records_full():
    """All 18^4 multigraphs with V=3, n=4, t in {0,1,2} (about 25 s)."""
    for recs in itertools.product([(s, d, tt) for s in range(3) for d in range(3) if s != d for tt in (0, 1, 2)],
                                  repeat=4):
        a = np.array(recs, dtype=np.int64)
        _check_exhaustive(a[:, 0].astype(np.int32), a[:, 1].astype(np.int32), a[:, 2])


def test_spanning_forest_enumeration_up_to_twelve_lg_edges():
    """Random graphs whose full line graph has <= 12 edges: the oracle's MSF is
    the unique key-minimal spanning forest among all of them."""
    rng = np.random.default_rng(7)
    done = 0
    while done < 150:
        n = int(rng.integers(2, 8))
        V = int(rng.integers(3, 7))
        src = rng.integers(0, V, n).astype(np.int32)
        dst = rng.integers(0, V, n).astype(np.int32)
        bad = src == dst
        dst[bad] = (src[bad] + 1) % V
        t = rng.integers(0, 4, n).astype(np.int64)
        pairs = lg_pairs_py(src, dst, t)
        if len(pairs) > 12 or not pairs:
            continue
        r = oracle.cluster(src, dst, t, 2, num_vertices=V, tier=0)
        c = components_count(n, [(x, y) for x, y, _ in pairs])
        keys = {(x, y): key_of(x, y, t) for x, y, _ in pairs}
        forests = [sorted(s) for s in itertools.combinations(keys, n - c) if is_acyclic(n, s)]
        best = min(forests, key=lambda f: sorted(keys[e] for e in f))
        # matroid greedy: the MSF's i-th smallest key is <= that of every spanning forest
        mine = sorted(keys[e] for e in msf_as_pairs(r))
        for f in forests:
            other = sorted(keys[e] for e in f)
            assert all(x <= y for x, y in zip(mine, other))
        assert msf_as_pairs(r) == best
        done += 1


# ------------------------------------------------- library cross-checks
def _random_tie_heavy(rng, n, V, tmax):
    src = rng.integers(0, V, n).astype(np.int32)
    dst = rng.integers(0, V, n).astype(np.int32)
    bad = src == dst
    dst[bad] = (src[bad] + 1 + rng.integers(0, V - 1, bad.sum())) % V
    t = rng.integers(0, tmax, n).astype(np.int64)
    return src, dst, t


def test_random_tie_heavy_tiers_agree_and_theorem_invariants():
    """Thm 1/3 (App. A): the skeleton has the same weighted connectivity as the
    full line graph: equal MSF weight, equal comps(., omega) for every omega
    (with <=, App. A), and exactly 2n - V' skeleton rows (Sec. 2 bound)."""
    rng = np.random.default_rng(2024)
    for it in range(300):
        n = int(rng.integers(1, 31))
        V = int(rng.integers(2, 7))
        src, dst, t = _random_tie_heavy(rng, n, V, int(rng.integers(1, 6)))
        M = int(rng.integers(2, 5))
        b = oracle.cluster(src, dst, t, M, num_vertices=V, tier=1)
        assert_same_result(oracle.cluster(src, dst, t, M, num_vertices=V, tier=0), b)
        full = oracle.full_line_graph(src, dst, t, V)
        sk = oracle.skeleton(src, dst, t, V)
        deg = np.bincount(np.concatenate([src, dst]), minlength=V)
        assert sk.size == 2 * n - int((deg > 0).sum())
        # every skeleton row is a line-graph edge
        fullset = {(int(e["tail"]), int(e["head"])) for e in full}
        assert all((int(e["tail"]), int(e["head"])) in fullset for e in sk)
        # networkx MST weight of the full line graph
        G = nx.Graph()
        G.add_nodes_from(range(n))
        for x, y, w in lg_pairs_py(src, dst, t):
            G.add_edge(x, y, weight=w)
        assert int(b.msf_w.sum()) == int(nx.minimum_spanning_tree(G).size(weight="weight"))
        # comps(L*, omega) == comps(L, omega) for every distinct omega
        for om in sorted(set(int(x) for x in full["w"])):
            def labels_of(E):
                sel = E[E["w"] <= om]
                M = sp.coo_matrix((np.ones(sel.size), (sel["tail"], sel["head"])), shape=(n, n))
                return connected_components(M, directed=False)[1]
            la, lb = labels_of(full), labels_of(sk)
            # same partition
            assert len(set(zip(la, lb))) == len(set(la)) == len(set(lb))


def test_scipy_msf_weight_shifted():
    """scipy's MST of the full line graph (weights +1 since scipy drops zeros)."""
    rng = np.random.default_rng(99)
    for _ in range(60):
        n = int(rng.integers(2, 60))
        V = int(rng.integers(2, 12))
        src, dst, t = _random_tie_heavy(rng, n, V, 50)
        r = oracle.cluster(src, dst, t, 2, num_vertices=V, tier=1)
        pairs = lg_pairs_py(src, dst, t)
        if not pairs:
            assert r.m == 0
            continue
        rr = np.array([p[0] for p in pairs]); cc = np.array([p[1] for p in pairs])
        ww = np.array([p[2] for p in pairs], dtype=np.float64) + 1.0
        T = minimum_spanning_tree(sp.coo_matrix((ww, (rr, cc)), shape=(n, n)))
        assert int(round(T.sum())) - T.nnz == int(r.msf_w.sum())
        assert T.nnz == r.m


def test_star_graph_closed_form_and_scipy_linkage():
    """All records share one hub: the line graph is a clique on the times, the
    skeleton is the sorted path, MSF weight = t_max - t_min, and the dendrogram
    equals scipy's single linkage on the 1-D times (tie-free gaps)."""
    rng = np.random.default_rng(5)
    done = 0
    while done < 40:
        n = int(rng.integers(2, 40))
        # distinct, tie-free gaps: sums of distinct powers of two as offsets
        t = np.sort(rng.choice(10 ** 6, n, replace=False)).astype(np.int64)
        gaps = np.diff(t)
        if len(set(gaps.tolist())) != len(gaps):
            continue
        perm = rng.permutation(n)
        t = t[perm]
        src = np.zeros(n, np.int32)
        dst = np.arange(1, n + 1, dtype=np.int32)
        r = oracle.cluster(src, dst, t, 2, tier=1)
        assert int(r.msf_w.sum()) == int(t.max() - t.min())
        Z = sch.linkage(t.astype(np.float64)[:, None], method="single")
        assert np.array_equal(Z[:, 2].astype(np.int64), r.sl_w)
        assert np.array_equal(Z[:, 3].astype(np.int64), r.sl_size.astype(np.int64))
        assert np.array_equal(np.minimum(Z[:, 0], Z[:, 1]).astype(np.int64), r.sl_left.astype(np.int64))
        assert np.array_equal(np.maximum(Z[:, 0], Z[:, 1]).astype(np.int64), r.sl_right.astype(np.int64))
        done += 1


def test_general_dendrogram_matches_scipy_on_minimax_distances():
    """Tie-free random graphs: single linkage on the minimax-path distances of the
    full line graph (scipy) reproduces the dendrogram rows exactly."""
    rng = np.random.default_rng(11)
    done = 0
    while done < 60:
        n = int(rng.integers(3, 40))
        V = int(rng.integers(2, 10))
        src, dst, _ = _random_tie_heavy(rng, n, V, 2)
        t = rng.choice(10 ** 9, n, replace=False).astype(np.int64)
        pairs = lg_pairs_py(src, dst, t)
        ws = [p[2] for p in pairs]
        if len(set(ws)) != len(ws) or 0 in ws:
            continue
        if components_count(n, [(x, y) for x, y, _ in pairs]) != 1:
            continue
        r = oracle.cluster(src, dst, t, 2, num_vertices=V, tier=0)
        D = minimax_matrix(n, pairs)
        from scipy.spatial.distance import squareform
        Z = sch.linkage(squareform(D, checks=False), method="single")
        assert np.array_equal(Z[:, 2].astype(np.int64), r.sl_w)
        assert np.array_equal(Z[:, 3].astype(np.int64), r.sl_size.astype(np.int64))
        assert np.array_equal(np.minimum(Z[:, 0], Z[:, 1]).astype(np.int64), r.sl_left.astype(np.int64))
        assert np.array_equal(np.maximum(Z[:, 0], Z[:, 1]).astype(np.int64), r.sl_right.astype(np.int64))
        done += 1


def _partition(labels):
    groups = {}
    for i, l in enumerate(labels):
        if l >= 0:
            groups.setdefault(int(l), []).append(i)
    return sorted(tuple(g) for g in groups.values())


def test_condensed_labels_match_sklearn_hdbscan():
    """HDBSCAN (Campello 2013, to which Alg. 1 defers) as implemented by
    scikit-learn, on the minimax distances with min_samples=1 (raw distances):
    the label partition equals the oracle's on tie-free connected inputs."""
    from sklearn.cluster import HDBSCAN
    rng = np.random.default_rng(3)
    done = 0
    while done < 120:
        n = int(rng.integers(6, 60))
        V = int(rng.integers(2, 8))
        src, dst, _ = _random_tie_heavy(rng, n, V, 2)
        # bursty, tie-free times
        t = (rng.integers(0, 4, n) * 10 ** 7 + rng.choice(10 ** 6, n, replace=False)).astype(np.int64)
        pairs = lg_pairs_py(src, dst, t)
        ws = [p[2] for p in pairs]
        if len(set(ws)) != len(ws) or 0 in ws:
            continue
        if components_count(n, [(x, y) for x, y, _ in pairs]) != 1:
            continue
        M = int(rng.integers(2, 7))
        r = oracle.cluster(src, dst, t, M, num_vertices=V, tier=1)
        D = minimax_matrix(n, pairs)
        sk = HDBSCAN(min_cluster_size=M, min_samples=1, metric="precomputed", allow_single_cluster=False,
                     copy=True).fit(D)
        assert _partition(sk.labels_) == _partition(r.labels), (n, M)
        done += 1


# ------------------------------------------------------ hand fixtures
def test_two_bursts_star_hand_computed():
    """Star of 4 records at times 0,1,10,11, M=2 (worked by hand from the
    readings): clusters {0,1} and {2,3} are born at lambda(9) inside ROOT; each
    sheds its two points at lambda(1)."""
    src = np.zeros(4, np.int32)
    dst = np.array([1, 2, 3, 4], np.int32)
    t = np.array([0, 1, 10, 11], np.int64)
    r = oracle.cluster(src, dst, t, 2, tier=1)
    assert r.m == 3 and list(r.sl_w) == [1, 1, 9]
    assert [(int(a), int(b)) for a, b in zip(r.sl_left, r.sl_right)] == [(0, 1), (2, 3), (4, 5)]
    assert list(r.cl_id) == [4, 5, 7] and r.n_clusters == 3
    assert list(r.cl_parent[:2]) == [7, 7]
    L9, L1 = lam(9), lam(1)
    assert L9 == (1 << 62) // 9 and L1 == 1 << 62
    assert list(r.cl_lambda_birth) == [L9, L9, 0]
    assert oracle.stability(r, 0) == 2 * (L1 - L9)
    assert oracle.stability(r, 1) == 2 * (L1 - L9)
    assert oracle.stability(r, 2) == 4 * L9
    assert list(r.cl_selected) == [1, 1, 0]
    assert list(r.labels) == [0, 0, 1, 1]
    assert list(r.pt_cluster) == [4, 4, 5, 5] and list(r.pt_lambda) == [L1] * 4


def test_eom_tie_keeps_parent_hand_computed():
    """Excess of mass with an exact tie (worked by hand): star with times
    0,2 | 5,7 | 13,14, M=2. Clusters P={0,2,5,7} and Q={13,14} are born at
    lambda(6); P splits at gap 3 into A={0,2}, B={5,7}, whose points leave at
    lambda(2). S(P) = 4(L3 - L6) and S(A) + S(B) = 4(L2 - L3); with the floor
    definition 2*L3 = L2 + L6 exactly, so the tie keeps the parent P."""
    t = np.array([0, 2, 5, 7, 13, 14], np.int64)
    r = oracle.cluster(np.zeros(6, np.int32), np.arange(1, 7, dtype=np.int32), t, 2, tier=1)
    L2, L3, L6 = lam(2), lam(3), lam(6)
    assert 2 * L3 == L2 + L6
    row = {int(c): i for i, c in enumerate(r.cl_id)}
    # dendrogram: (4,5)@1 -> 6, (0,1)@2 -> 7, (2,3)@2 -> 8, (7,8)@3 -> 9, (9,6)@6 -> 10
    assert [(int(a), int(b)) for a, b in zip(r.sl_left, r.sl_right)] == [(4, 5), (0, 1), (2, 3), (7, 8), (6, 9)]
    A, B, P, Q = row[7], row[8], row[9], row[6]
    assert oracle.stability(r, P) == 4 * (L3 - L6)
    assert oracle.stability(r, A) + oracle.stability(r, B) == 4 * (L2 - L3) == oracle.stability(r, P)
    assert r.cl_selected[P] == 1 and r.cl_selected[Q] == 1
    assert r.cl_selected[A] == 0 and r.cl_selected[B] == 0
    assert list(r.labels) == [0, 0, 0, 0, 1, 1]


def test_two_bursts_of_six_two_clusters():
    """Two bursts of six records 1e5 s apart around one vertex, M=5: two labels."""
    t = np.array([0, 5, 9, 20, 22, 30, 100000, 100004, 100011, 100013, 100021, 100030], np.int64)
    src = np.zeros(12, np.int32)
    dst = np.arange(1, 13, dtype=np.int32)
    r = oracle.cluster(src, dst, t, 5, tier=1)
    assert r.n_labels == 2
    assert list(r.labels) == [0] * 6 + [1] * 6


def test_all_equal_timestamps_and_matching_and_forest():
    # all-equal timestamps on a star: every weight 0, merges in canonical-key order
    n = 7
    r = oracle.cluster(np.zeros(n, np.int32), np.arange(1, n + 1, dtype=np.int32), np.full(n, 5, np.int64), 3, tier=0)
    assert r.m == n - 1 and (r.sl_w == 0).all()
    assert list(r.msf_head) == list(range(1, n))            # heads ascending
    assert list(r.msf_tail) == list(range(0, n - 1))         # each joins its predecessor
    # matching graph: no two records share a vertex -> empty line graph, all noise
    src = np.arange(0, 20, 2, dtype=np.int32)
    dst = src + 1
    r = oracle.cluster(src, dst, np.arange(10, dtype=np.int64), 2, tier=0)
    assert r.m == 0 and (r.labels == -1).all() and r.n_clusters == 1
    assert (r.pt_cluster == 10).all() and (r.pt_lambda == 0).all()
    # forest of 3 star components of sizes 6, 6, 2, far apart in vertex space, M=3
    src = np.array([0] * 6 + [10] * 6 + [20] * 2, np.int32)
    dst = np.array(list(range(1, 7)) + list(range(11, 17)) + [21, 22], np.int32)
    t = np.array([0, 1, 2, 3, 4, 5, 0, 2, 4, 6, 8, 10, 0, 1], np.int64)
    r = oracle.cluster(src, dst, t, 3, tier=0)
    assert r.m == 14 - 3
    # two big components each start a cluster at lambda 0 under ROOT; the pair is ROOT noise
    assert int(r.cl_parent[0]) == int(r.cl_id[-1]) and int(r.cl_lambda_birth[0]) == 0
    assert set(r.labels[:6].tolist()) == {0} and set(r.labels[6:12].tolist()) == {1}
    assert (r.labels[12:] == -1).all() and (r.pt_lambda[12:] == 0).all()


def test_error_paths_and_degenerate_sizes():
    z = np.zeros(0)
    r = oracle.cluster(z.astype(np.int32), z.astype(np.int32), z.astype(np.int64), 5, num_vertices=1)
    assert r.status == 0 and r.m == 0 and r.n_clusters == 1
    r = oracle.cluster(np.array([0], np.int32), np.array([1], np.int32), np.array([3], np.int64), 5)
    assert r.status == 0 and r.m == 0 and list(r.labels) == [-1]
    assert oracle.cluster(np.array([1], np.int32), np.array([1], np.int32), np.array([3], np.int64), 5).status == oracle.ESELFLOOP
    assert oracle.cluster(np.array([0], np.int32), np.array([9], np.int32), np.array([3], np.int64), 5,
                          num_vertices=4).status == oracle.ERANGE
    assert oracle.cluster(np.array([0, 1], np.int32), np.array([1, 2], np.int32),
                          np.array([0, 1 << 62], np.int64), 5).status == oracle.ERANGE
    assert oracle.cluster(np.array([0], np.int32), np.array([1], np.int32), np.array([3], np.int64), 1).status == oracle.EINVAL


# ------------------------------------------------ invariants at the tiny workload
def test_condensed_invariants_on_tiny_workload():
    """The 200k-edge Chung-Lu/burst workload: every point leaves exactly one
    cluster, chosen clusters are an antichain, every label class has >= M
    members and is connected in the skeleton (Sec. 4: clusters are connected)."""
    import synth
    w = synth.plain_tiny()
    r = oracle.cluster(w.src, w.dst, w.t, w.min_cluster_size, w.num_vertices, tier=1)
    n, M = w.n, w.min_cluster_size
    assert r.status == 0
    ids = set(int(x) for x in r.cl_id)
    assert all(int(c) in ids for c in r.pt_cluster)
    row = {int(c): i for i, c in enumerate(r.cl_id)}
    chosen = [i for i in range(r.n_clusters) if r.cl_selected[i]]
    for i in chosen:
        a = int(r.cl_parent[i])
        while a != 0xFFFFFFFF:
            assert not r.cl_selected[row[a]]
            a = int(r.cl_parent[row[a]])
    counts = np.bincount(r.labels[r.labels >= 0], minlength=r.n_labels)
    assert (counts >= M).all() and counts.size == r.n_labels == len(chosen)
    # label classes connected in the skeleton restricted to the class
    sk = oracle.skeleton(w.src, w.dst, w.t, w.num_vertices)
    la = r.labels
    keep = (la[sk["tail"]] == la[sk["head"]]) & (la[sk["tail"]] >= 0)
    A = sp.coo_matrix((np.ones(int(keep.sum())), (sk["tail"][keep], sk["head"][keep])), shape=(n, n))
    _, comp = connected_components(A, directed=False)
    lab_pts = np.nonzero(la >= 0)[0]
    assert len(set(zip(la[lab_pts].tolist(), comp[lab_pts].tolist()))) == r.n_labels
    # labels numbered by ascending minimum member id
    first = [int(np.nonzero(la == k)[0][0]) for k in range(r.n_labels)]
    assert first == sorted(first)
    # Tier A agrees with Tier B on a 3000-edge prefix (full line graph fits)
    s, d, tt = w.src[:3000], w.dst[:3000], w.t[:3000]
    assert_same_result(oracle.cluster(s, d, tt, M, w.num_vertices, tier=0),
                       oracle.cluster(s, d, tt, M, w.num_vertices, tier=1))


def test_joined_below_is_the_cycle_property():
    """The forest checker: on the MSF every non-row line-graph edge is joined below and no row is; replacing a
    row by a heavier edge across the same cut is caught."""
    rng = np.random.default_rng(41)
    swaps = 0
    for trial in range(60):
        n = int(rng.integers(2, 40))
        s, d, t = _random_tie_heavy(rng, n, int(rng.integers(2, 8)), int(rng.choice([3, 50])))
        edges = oracle.full_line_graph(s, d, t)
        mt, mh, mw = oracle.kruskal(n, edges, t)
        if len(edges) == 0:
            continue
        got = oracle.joined_below(n, mt, mh, mw, edges["tail"], edges["head"], edges["w"])
        rows = set(zip(mt.tolist(), mh.tolist()))
        is_row = np.array([(a, b) in rows for a, b in zip(edges["tail"].tolist(), edges["head"].tolist())])
        assert np.array_equal(got, ~is_row), trial
        # swap: drop row k, add the cheapest non-row edge that reconnects its two sides (if any); the dropped row
        # is then not joined below while it is no row any more
        if len(mt) == 0:
            continue
        k = int(rng.integers(0, len(mt)))
        keep = [i for i in range(len(mt)) if i != k]
        g = nx.Graph()
        g.add_nodes_from(range(n))
        g.add_edges_from((int(mt[i]), int(mh[i])) for i in keep)
        comp = nx.node_connected_component(g, int(mt[k]))
        across = [e for e in edges if (int(e["tail"]) in comp) != (int(e["head"]) in comp)
                  and (int(e["tail"]), int(e["head"])) != (int(mt[k]), int(mh[k]))]
        if not across:
            continue
        alt = min(across, key=lambda e: (int(e["w"]), int(e["head"]), -int(e["tail"])))
        ft = np.append(mt[keep], alt["tail"]).astype(np.uint32)
        fh = np.append(mh[keep], alt["head"]).astype(np.uint32)
        fw = np.append(mw[keep], alt["w"]).astype(np.int64)
        order = sorted(range(len(ft)), key=lambda i: (int(fw[i]), int(fh[i]), -int(ft[i])))
        ft, fh, fw = ft[order], fh[order], fw[order]
        bad = oracle.joined_below(n, ft, fh, fw, mt[k:k + 1], mh[k:k + 1], mw[k:k + 1])
        assert not bad[0], trial
        swaps += 1
    assert swaps >= 10


def test_condense_wrapper_equals_full_pipeline():
    """oracle.condense(oracle.dendrogram(MSF)) reproduces oracle.cluster on a mid-sized sample."""
    import synth
    w = synth.plain_tiny()
    r = oracle.cluster(w.src, w.dst, w.t, w.min_cluster_size, w.num_vertices, tier=1)
    L, R, W, S = oracle.dendrogram(w.n, r.msf_tail, r.msf_head, r.msf_w)
    assert np.array_equal(L, r.sl_left) and np.array_equal(R, r.sl_right) and np.array_equal(S, r.sl_size)
    c = oracle.condense(w.n, L, R, W, S, w.min_cluster_size)
    for f in ("pt_cluster", "pt_lambda", "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi",
              "cl_stab_lo", "cl_selected", "labels"):
        assert np.array_equal(getattr(c, f), getattr(r, f)), f
    assert c.n_labels == r.n_labels
    # a forest with a cycle is rejected
    with pytest.raises(RuntimeError):
        oracle.dendrogram(3, np.array([0, 1, 0], np.uint32), np.array([1, 2, 2], np.uint32),
                          np.array([1, 1, 2], np.int64))


def test_time_filtered_line_graph():
    """Time-filtered line graph (Sec. 5.1): only edges with w <= max_dt. Definition and skeleton tiers agree for
    every cutoff (Thm 3 at that threshold), and the forest is exactly the unfiltered forest's rows with
    w <= max_dt (Kruskal takes edges in key order, so the filter cuts a prefix); networkx MSF weight of the
    filtered full line graph agrees."""
    rng = np.random.default_rng(17)
    for trial in range(120):
        n = int(rng.integers(2, 50))
        V = int(rng.integers(2, 8))
        s, d, t = _random_tie_heavy(rng, n, V, int(rng.choice([5, 60, 3000])))
        for causal in (False, True):
            full = oracle.cluster(s, d, t, 2, V, tier=1, causal=causal)
            edges = oracle.causal_line_graph(s, d, t, V) if causal else oracle.full_line_graph(s, d, t, V)
            for cut in sorted(set([0, 1, 7] + [int(x) for x in rng.choice(full.msf_w, min(3, full.m))] if full.m
                                  else [0, 3])):
                a = oracle.cluster(s, d, t, 2, V, tier=0, causal=causal, max_dt=cut)
                b = oracle.cluster(s, d, t, 2, V, tier=1, causal=causal, max_dt=cut)
                assert_same_result(a, b)
                keep = full.msf_w <= cut
                assert np.array_equal(a.msf_w, full.msf_w[keep]) and np.array_equal(a.msf_tail, full.msf_tail[keep])
                g = nx.Graph()
                g.add_nodes_from(range(n))
                for e in edges[edges["w"] <= cut]:
                    u, v, w = int(e["tail"]), int(e["head"]), int(e["w"])
                    if not g.has_edge(u, v) or g[u][v]["weight"] > w:
                        g.add_edge(u, v, weight=w)
                assert int(a.msf_w.sum()) == sum(x[2]["weight"] for x in nx.minimum_spanning_edges(g, data=True))
                assert a.m == n - nx.number_connected_components(g)
