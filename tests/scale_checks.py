"""Checks of a full result at sizes where the oracle's skeleton and Kruskal are
too slow: the MSF by properties that pin it, everything downstream of the MSF
exactly by the oracle's own union-find and condensing run on the given rows.

  * every MSF row is a line-graph edge (its records share a vertex) with
    w = t_head - t_tail and tail before head in record order;
  * rows are in strictly ascending canonical key (w, head, 2^32-1-tail);
  * the rows form a forest (the oracle's union-find rejects a cycle) with as
    many components as the line graph, i.e. the connected components of the
    vertex graph over vertices that have an edge (scipy);
  * cycle property: sampled line-graph edges (pairs of records of sampled
    vertices, the largest hub included) that are not rows are joined by rows
    of smaller key, and none is a cheaper edge across a cut;
  * dendrogram rows, condensed tree, stabilities, selection and labels equal
    the oracle's, computed from the given MSF rows.
"""
import numpy as np

import oracle

FIELDS_AFTER_MSF = ("pt_cluster", "pt_lambda", "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi",
                    "cl_stab_lo", "cl_selected", "labels")


def key_lt(w1, h1, t1, w2, h2, t2):
    """(w, head, 2^32-1-tail) lexicographic: first < second."""
    return (w1 < w2) | ((w1 == w2) & ((h1 < h2) | ((h1 == h2) & (t1 > t2))))


def sample_line_graph_edges(src, dst, t, V, n_vertices, per_vertex, seed):
    """Random pairs of records that share a sampled vertex (the largest hub always included)."""
    rng = np.random.default_rng(seed)
    deg = np.bincount(src, minlength=V) + np.bincount(dst, minlength=V)
    cand = np.nonzero(deg > 1)[0]
    hub = int(np.argmax(deg))
    verts = np.unique(np.concatenate([[hub], rng.choice(cand, min(n_vertices, cand.size), replace=False)]))
    mask = np.zeros(V, bool)
    mask[verts] = True
    ids = np.nonzero(mask[src] | mask[dst])[0]
    ends = np.concatenate([src[ids], dst[ids]])
    recs = np.concatenate([ids, ids])
    keep = mask[ends]
    ends, recs = ends[keep], recs[keep]
    order = np.argsort(ends, kind="stable")
    ends, recs = ends[order], recs[order]
    starts = np.searchsorted(ends, verts)
    stops = np.searchsorted(ends, verts, side="right")
    pa, pb = [], []
    for a, b in zip(starts, stops):
        k = b - a
        if k < 2:
            continue
        q = min(per_vertex, k * (k - 1) // 2)
        i = rng.integers(a, b, q)
        j = rng.integers(a, b, q)
        ok = recs[i] != recs[j]
        pa.append(recs[i][ok])
        pb.append(recs[j][ok])
    pa, pb = np.concatenate(pa), np.concatenate(pb)
    first = (t[pa] < t[pb]) | ((t[pa] == t[pb]) & (pa < pb))
    tail, head = np.where(first, pa, pb), np.where(first, pb, pa)
    return tail, head, t[head] - t[tail]


def check_msf_and_dendrogram(data, got, n_vertices=4000, per_vertex=64, seed=7, log=print):
    """data: {"src", "dst", "t", "V"}; got: the result as host arrays. Consumes data's arrays."""
    src, dst, t, V = data["src"], data["dst"], data["t"], data["V"]
    n = len(src)
    m = got["m"]
    tail = got["msf_tail"].astype(np.int64)
    head = got["msf_head"].astype(np.int64)
    mw = got["msf_w"]
    assert len(tail) == m
    if m:
        assert tail.min() >= 0 and head.max() < n
        share = ((src[tail] == src[head]) | (src[tail] == dst[head]) | (dst[tail] == src[head]) |
                 (dst[tail] == dst[head]))
        assert share.all(), "an MSF row joins records that share no vertex"
        del share
        log("rows join records that share a vertex")
        assert np.array_equal(mw, t[head] - t[tail]), "MSF weight"
        assert np.all((t[tail] < t[head]) | ((t[tail] == t[head]) & (tail < head))), "row orientation"
        assert np.all(key_lt(mw[:-1], head[:-1], tail[:-1], mw[1:], head[1:], tail[1:])), "row order"
    log("rows checked")

    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    deg = np.bincount(src, minlength=V) + np.bincount(dst, minlength=V)
    g = coo_matrix((np.ones(n, np.int8), (src, dst)), shape=(V, V)).tocsr()
    log("vertex graph built")
    _, lab = connected_components(g, directed=False)
    del g
    c_line = len(np.unique(lab[deg > 0]))
    del lab, deg
    assert m == n - c_line, "forest size %d, line graph needs %d rows" % (m, n - c_line)
    log("components %d" % c_line)

    qt, qh, qw = sample_line_graph_edges(src, dst, t, V, n_vertices, per_vertex, seed)
    log("sampled %d line-graph edges" % len(qt))
    data.clear()
    del src, dst, t

    L, R, LW, S = oracle.dendrogram(n, got["msf_tail"], got["msf_head"], mw)  # raises on a cycle
    for f, ref in (("sl_left", L), ("sl_right", R), ("sl_w", LW), ("sl_size", S)):
        assert np.array_equal(got[f], ref), f
    del L, R, LW, S
    log("dendrogram equal")

    joined = oracle.joined_below(n, got["msf_tail"], got["msf_head"], mw, qt, qh, qw)
    log("joined-below query done")
    # a sampled pair not joined below must itself be a row (a row joined below would have closed a cycle,
    # which the union-find above rejects)
    U = np.unique(qh[~joined].astype(np.int64) * np.int64(n) + qt[~joined].astype(np.int64))
    found = np.zeros(len(U), bool)
    if len(U):
        for a in range(0, m, 1 << 26):
            rk = head[a:a + (1 << 26)] * np.int64(n) + tail[a:a + (1 << 26)]
            pos = np.minimum(np.searchsorted(U, rk), len(U) - 1)
            hit = U[pos] == rk
            found[pos[hit]] = True
    assert found.all(), "cycle property fails for %d sampled edges" % int((~found).sum())
    log("cycle property on %d sampled line-graph edges (%d of them rows)" % (len(qt), len(U)))


def check_condensed(n, M, got, log=print):
    """Condensed tree, stabilities, selection and labels: the oracle's condensing on the result's own
    dendrogram rows (checked equal to the oracle's union-find by check_msf_and_dendrogram)."""
    c = oracle.condense(n, got["sl_left"], got["sl_right"], got["sl_w"], got["sl_size"], M)
    assert (got["n_clusters"], got["n_labels"]) == (len(c.cl_id), c.n_labels)
    for f in FIELDS_AFTER_MSF:
        assert np.array_equal(got[f], getattr(c, f)), f
    log("condensed tree and labels equal")


def check_result(src, dst, t, V, M, got, n_vertices=4000, per_vertex=64, seed=7, log=print):
    n = len(src)
    check_msf_and_dendrogram({"src": src, "dst": dst, "t": t, "V": V}, got, n_vertices, per_vertex, seed, log)
    check_condensed(n, M, got, log)
