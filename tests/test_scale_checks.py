"""The large-size checker accepts the oracle's own result and rejects planted
mistakes (CPU only)."""
import numpy as np
import pytest

import oracle
import synth
from scale_checks import check_result

FIELDS = ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster", "pt_lambda",
          "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected", "labels")


@pytest.fixture(scope="module")
def tiny():
    w = synth.plain_tiny()
    r = oracle.cluster(w.src, w.dst, w.t, w.min_cluster_size, w.num_vertices, tier=1)
    got = {"m": r.m, "n_clusters": r.n_clusters, "n_labels": r.n_labels}
    for f in FIELDS:
        got[f] = np.array(getattr(r, f))
    return w, got


def run(w, got):
    check_result(w.src, w.dst, w.t, w.num_vertices, w.min_cluster_size, got, n_vertices=3000, per_vertex=200,
                 log=lambda s: None)


def test_accepts_the_oracle_result(tiny):
    run(*tiny)


def test_rejects_a_non_minimal_forest(tiny):
    """Swap one MSF row for a heavier skeleton edge across the same cut: still a spanning forest of the same size,
    so only the cycle property can catch it."""
    w, got = tiny
    src, dst, t = w.src, w.dst, w.t
    sk = oracle.skeleton(src, dst, t, w.num_vertices)
    mt, mh, mw = got["msf_tail"], got["msf_head"], got["msf_w"]
    rows = set(zip(mt.tolist(), mh.tolist()))
    import networkx as nx
    rng = np.random.default_rng(3)
    g = nx.Graph()
    g.add_nodes_from(range(w.n))
    g.add_edges_from(zip(mt.tolist(), mh.tolist()))
    for _ in range(50):
        k = int(rng.integers(0, len(mt)))
        g.remove_edge(int(mt[k]), int(mh[k]))
        comp = nx.node_connected_component(g, int(mt[k]))
        g.add_edge(int(mt[k]), int(mh[k]))
        inside = np.zeros(w.n, bool)
        inside[list(comp)] = True
        across = sk[(inside[sk["tail"]] != inside[sk["head"]])]
        across = across[[(a, b) not in rows for a, b in zip(across["tail"].tolist(), across["head"].tolist())]]
        if len(across):
            break
    else:
        pytest.skip("no replacement edge found")
    alt = across[np.lexsort((-across["tail"].astype(np.int64), across["head"], across["w"]))[0]]
    ft = np.append(np.delete(mt, k), alt["tail"]).astype(np.uint32)
    fh = np.append(np.delete(mh, k), alt["head"]).astype(np.uint32)
    fw = np.append(np.delete(mw, k), alt["w"]).astype(np.int64)
    o = np.lexsort((-ft.astype(np.int64), fh, fw))
    bad = dict(got)
    bad["msf_tail"], bad["msf_head"], bad["msf_w"] = ft[o], fh[o], fw[o]
    L, R, LW, S = oracle.dendrogram(w.n, bad["msf_tail"], bad["msf_head"], bad["msf_w"])
    c = oracle.condense(w.n, L, R, LW, S, w.min_cluster_size)
    bad.update(sl_left=L, sl_right=R, sl_w=LW, sl_size=S, n_clusters=len(c.cl_id), n_labels=c.n_labels)
    for f in ("pt_cluster", "pt_lambda", "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi",
              "cl_stab_lo", "cl_selected", "labels"):
        bad[f] = getattr(c, f)
    with pytest.raises(AssertionError, match="cycle property"):
        check_result(src, dst, t, w.num_vertices, w.min_cluster_size, bad, n_vertices=10000, per_vertex=100000,
                     log=lambda s: None)


@pytest.mark.parametrize("field,idx", [("labels", 17), ("cl_stab_lo", 3), ("sl_size", 100), ("msf_w", 5)])
def test_rejects_planted_output_errors(tiny, field, idx):
    w, got = tiny
    bad = dict(got)
    a = bad[field].copy()
    a[idx] = a[idx] + 1
    bad[field] = a
    with pytest.raises((AssertionError, RuntimeError)):
        run(w, bad)


def test_rejects_a_missing_row(tiny):
    w, got = tiny
    bad = dict(got)
    for f in ("msf_tail", "msf_head", "msf_w"):
        bad[f] = got[f][:-1]
    bad["m"] = got["m"] - 1
    with pytest.raises(AssertionError, match="forest size"):
        run(w, bad)
