"""Pins of the oracle's discrete dendrogram (Alg. 5) and of condensing on it,
CPU only.

* D against its definition: per-level connected components of the line graph
  keeping edges with w <= omega_i (scipy), for random graphs and threshold sets,
  in both line-graph modes.
* Condensing with several children per node reduces to the binary condensing
  when every level holds exactly one merge (thresholds = the distinct weights of
  a tie-free input).
* A hand-computed three-way split: three bursts joined at one level become three
  sibling clusters (no intermediate cluster), with exact stabilities.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle

LAM = lambda w: (1 << 63) // max(2 * int(w), 1)


def d_from_components(n, edges, thresholds):
    """Definition: D-nodes are components that first appear at a level, keyed (level, min member, size), each
    with the key of the D-node it first becomes part of."""
    nodes = {}
    labs = []
    for i, w in enumerate(thresholds):
        keep = edges["w"] <= w
        g = sp.coo_matrix((np.ones(int(keep.sum())), (edges["tail"][keep], edges["head"][keep])), shape=(n, n))
        _, lab = connected_components(g, directed=False)
        labs.append(lab)
    sizes = [np.bincount(lab) for lab in labs]
    mins = []
    for lab in labs:
        mn = np.full(lab.max() + 1, n, np.int64)
        np.minimum.at(mn, lab, np.arange(n))
        mins.append(mn)
    for i in range(len(thresholds)):
        lab, sz, mn = labs[i], sizes[i], mins[i]
        for c in range(len(sz)):
            if sz[c] < 2:
                continue
            members_min = int(mn[c])
            # a D-node unless the same component existed one level lower
            if i > 0:
                lower = labs[i - 1][members_min]
                if sizes[i - 1][lower] == sz[c]:
                    continue
            nodes[(i, members_min, int(sz[c]))] = None
    # parents: the D-node at the next level where the component grows
    for (i, mm, szc) in list(nodes):
        par = None
        for j in range(i + 1, len(thresholds)):
            c = labs[j][mm]
            if sizes[j][c] != szc:
                par = (j, int(mins[j][c]), int(sizes[j][c]))
                break
        nodes[(i, mm, szc)] = par
    return nodes


def d_from_oracle(n, r, dd_level, dd_top):
    m = r.m
    rowpar = np.full(m, -1, np.int64)
    for k in range(m):
        for c in (int(r.sl_left[k]), int(r.sl_right[k])):
            if c >= n:
                rowpar[c - n] = k
    # min member of every row's subtree (children precede parents)
    mn = np.zeros(m, np.int64)
    for k in range(m):
        a, b = int(r.sl_left[k]), int(r.sl_right[k])
        mn[k] = min(a if a < n else mn[a - n], b if b < n else mn[b - n])
    nodes = {}
    for k in range(m):
        if int(dd_top[k]) != n + k:
            continue
        key = (int(dd_level[k]), int(mn[k]), int(r.sl_size[k]))
        p = rowpar[k]
        if p < 0:
            nodes[key] = None
        else:
            top = int(dd_top[p]) - n
            nodes[key] = (int(dd_level[top]), int(mn[top]), int(r.sl_size[top]))
    return nodes


def _random_graph(rng, n, V, tmax):
    s = rng.integers(0, V, n).astype(np.int32)
    d = rng.integers(0, V, n).astype(np.int32)
    bad = s == d
    d[bad] = (s[bad] + 1 + rng.integers(0, V - 1, bad.sum())) % V
    return s, d, rng.integers(0, tmax, n).astype(np.int64)


def test_discrete_dendrogram_is_per_level_components():
    rng = np.random.default_rng(23)
    for trial in range(150):
        n = int(rng.integers(2, 70))
        V = int(rng.integers(2, 10))
        s, d, t = _random_graph(rng, n, V, int(rng.choice([8, 100, 4000])))
        for causal in (False, True):
            thr = np.unique(rng.integers(0, int(rng.choice([4, 50, 5000])), int(rng.integers(1, 8))))
            if trial % 3 == 0:
                thr = np.array([1 << k for k in range(13)], np.int64)
            r, dl, dt = oracle.cluster_discrete(s, d, t, 2, thr, V, causal=causal)
            assert r.status == 0
            edges = oracle.causal_line_graph(s, d, t, V) if causal else oracle.full_line_graph(s, d, t, V)
            assert d_from_oracle(n, r, dl, dt) == d_from_components(n, edges, thr), (trial, causal, thr)


def test_multiway_condensing_reduces_to_binary_with_one_merge_per_level():
    rng = np.random.default_rng(29)
    checked = 0
    for trial in range(200):
        n = int(rng.integers(3, 60))
        V = int(rng.integers(2, 8))
        s, d, t = _random_graph(rng, n, V, 10 ** 6)
        r = oracle.cluster(s, d, t, 3, V)
        if r.m == 0 or len(np.unique(r.msf_w)) != r.m:
            continue  # needs a tie-free forest
        for M in (2, 3, 4):
            b = oracle.cluster(s, d, t, M, V)
            rd, dl, dt = oracle.cluster_discrete(s, d, t, M, np.unique(r.msf_w), V)
            assert np.array_equal(dt, np.arange(r.m) + n)  # every row is its own D-node
            for f in ("pt_cluster", "pt_lambda", "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi",
                      "cl_stab_lo", "cl_selected", "labels"):
                assert np.array_equal(getattr(rd, f), getattr(b, f)), (trial, M, f)
        checked += 1
    assert checked >= 50


def test_three_bursts_joined_at_one_level_hand_computed():
    """Star around vertex 0; bursts A (t 0..4), B (100..104), C (200..204); M = 3; thresholds [1, 128].
    Level 0 (w <= 1) forms the three bursts, level 1 joins all 15 records at once. ROOT continues into the
    single component; at its D-node three big children start three sibling clusters at lambda(128); inside
    each burst every record is a small child and leaves at lambda(1)."""
    s = np.zeros(15, np.int32)
    d = np.arange(1, 16, dtype=np.int32)
    t = np.array([0, 1, 2, 3, 4, 100, 101, 102, 103, 104, 200, 201, 202, 203, 204], np.int64)
    r, dl, dt = oracle.cluster_discrete(s, d, t, 3, [1, 128], 16)
    assert r.n_clusters == 4 and r.n_labels == 3
    L1, L128 = LAM(1), LAM(128)
    assert list(r.cl_lambda_birth[:3]) == [L128] * 3 and list(r.cl_size[:3]) == [5, 5, 5]
    stab = [(int(h) << 64) | int(lo) for h, lo in zip(r.cl_stab_hi, r.cl_stab_lo)]
    assert stab[:3] == [5 * (L1 - L128)] * 3 and stab[3] == 15 * L128  # ROOT: 15 records born at 0
    assert list(r.cl_selected) == [1, 1, 1, 0]
    assert list(r.labels) == [0] * 5 + [1] * 5 + [2] * 5
    assert all(int(x) == L1 for x in r.pt_lambda)
    # the exact dendrogram's binary condensing has an extra cluster (the first two bursts joined at 96)
    b = oracle.cluster(s, d, t, 3, 16)
    assert b.n_clusters == 5


def test_rows_above_the_last_threshold_are_left_out():
    s = np.zeros(6, np.int32)
    d = np.arange(1, 7, dtype=np.int32)
    t = np.array([0, 1, 2, 1000, 1001, 1002], np.int64)
    r, dl, dt = oracle.cluster_discrete(s, d, t, 3, [1, 2, 4], 7)
    assert r.m == 4 and r.n_clusters == 3  # two components of 3: both start clusters at lambda 0
    assert list(r.cl_lambda_birth[:2]) == [0, 0]
    with pytest.raises(RuntimeError):
        oracle.condense_discrete(6, r.sl_left, r.sl_right, np.array([1, 1, 1, 9]), r.sl_size, 3, [1, 2, 4])
