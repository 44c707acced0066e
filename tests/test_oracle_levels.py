"""Pins of the oracle's per-level connected components (Alg. 5 computed as the
paper does it: one connected-components pass per threshold), CPU only.

* A hand-computed star: four records on one vertex at times 0, 1, 10, 11.
* scipy's connected_components on the full line graph restricted to w <= the
  threshold, for random graphs and threshold sets, in both line-graph modes.
* The skeleton and the forest give the same labels as the full line graph
  (Thm 3 at every threshold), which is what lets the GPU path run on the MSF.
* Invariants: a label is its component's smallest member, and every level
  refines the next.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle


def scipy_labels(n, edges, w):
    keep = edges["w"] <= w
    g = sp.coo_matrix((np.ones(int(keep.sum())), (edges["tail"][keep], edges["head"][keep])), shape=(n, n))
    _, lab = connected_components(g, directed=False)
    low = np.full(lab.max() + 1, n, np.int64)
    np.minimum.at(low, lab, np.arange(n))
    return low[lab].astype(np.int32)


def _random_graph(rng, n, V, tmax):
    s = rng.integers(0, V, n).astype(np.int32)
    d = rng.integers(0, V, n).astype(np.int32)
    bad = s == d
    d[bad] = (s[bad] + 1 + rng.integers(0, V - 1, bad.sum())) % V
    return s, d, rng.integers(0, tmax, n).astype(np.int64)


def test_hand_star():
    # all four records share vertex 0: pairs at |dt| = 1 (0,1), 1 (2,3), 9 (1,2), 10, 10, 11
    src = np.zeros(4, np.int32)
    dst = np.arange(1, 5, dtype=np.int32)
    t = np.array([0, 1, 10, 11], np.int64)
    lg = oracle.full_line_graph(src, dst, t)
    lab = oracle.level_components(4, lg["tail"], lg["head"], lg["w"], [0, 1, 5, 9, 100])
    assert lab.tolist() == [[0, 1, 2, 3], [0, 0, 2, 2], [0, 0, 2, 2], [0, 0, 0, 0], [0, 0, 0, 0]]


@pytest.mark.parametrize("causal", [False, True])
def test_random_graphs_against_scipy_and_across_edge_sets(causal):
    rng = np.random.default_rng(211 if causal else 209)
    for trial in range(40):
        n = int(rng.integers(2, 160))
        V = int(rng.integers(2, 25))
        src, dst, t = _random_graph(rng, n, V, int(rng.choice([5, 60, 5000])))
        thr = np.unique(rng.integers(0, 6000, int(rng.integers(1, 9))))
        full = (oracle.causal_line_graph if causal else oracle.full_line_graph)(src, dst, t)
        lab = oracle.level_components(n, full["tail"], full["head"], full["w"], thr)
        for i, w in enumerate(thr):
            assert np.array_equal(lab[i], scipy_labels(n, full, int(w))), (causal, trial, i)
        sk = (oracle.causal_skeleton if causal else oracle.skeleton)(src, dst, t)
        assert np.array_equal(oracle.level_components(n, sk["tail"], sk["head"], sk["w"], thr), lab), (causal, trial)
        r = oracle.cluster(src, dst, t, 2, V, tier=1, causal=causal)
        lab_f = oracle.level_components(n, r.msf_tail, r.msf_head, r.msf_w, thr)
        assert np.array_equal(lab_f, lab), (causal, trial)
        # invariants: smallest member, refinement
        ids = np.arange(n)
        assert np.all(lab <= ids)
        for i in range(len(thr)):
            assert np.array_equal(lab[i][lab[i]], lab[i])
            if i + 1 < len(thr):
                assert np.array_equal(lab[i + 1][lab[i]], lab[i + 1])


def test_no_edges_and_no_levels():
    assert oracle.level_components(3, [], [], [], [0, 7]).tolist() == [[0, 1, 2], [0, 1, 2]]
    assert oracle.level_components(3, [0], [1], [4], []).shape == (0, 3)
    assert oracle.level_components(0, [], [], [], [1]).shape == (1, 0)


def test_argument_errors():
    for thr in ([3, 3], [5, 2], [-1, 4]):
        with pytest.raises(ValueError):
            oracle.level_components(3, [0], [1], [4], thr)
    with pytest.raises(ValueError):
        oracle.level_components(3, [0], [3], [4], [5])
