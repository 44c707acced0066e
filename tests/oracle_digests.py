"""Oracle digests of whole workloads, computed in worker processes (host only: no GPU, no torch).

A worker regenerates one graph of the batching workload, or one request of the serving stream, from its
seed (the generators are counter-based, so a graph is the same however it is produced), clusters it with
the oracle (skeleton tier) and returns a digest of every output field. The GPU side digests its own outputs
the same way, so a test compares whole workloads with the oracle without moving outputs between processes.
"""
import hashlib

import numpy as np

FIELDS = ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster", "pt_lambda",
          "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected", "labels")


def digest_fields(get, m, n_clusters, n_labels):
    """blake2b over every field's values as int64 (bit patterns of unsigned values kept) and the counts."""
    h = hashlib.blake2b(digest_size=20)
    h.update(np.array([m, n_clusters, n_labels], np.int64).tobytes())
    for f in FIELDS:
        x = np.asarray(get(f))
        h.update(np.int64(x.size).tobytes())
        h.update(x.astype(np.int64).tobytes())
    return h.hexdigest()


def batch_graph_digest(args):
    """(g, n_g, seed, M) -> (g, digest of the oracle's outputs for graph g of the batching workload)."""
    g, n_g, seed, M = args
    import oracle
    import synth
    s, d, t, V = synth.batch_graph(g, n_g, seed)
    r = oracle.cluster(s, d, t, M, V, tier=1)
    if r.status != 0:
        return g, "status %d" % r.status
    return g, digest_fields(lambda f: getattr(r, f), r.m, r.n_clusters, r.n_labels)


def request_digest(args):
    """(r, n_r, seed, M) -> (r, digest of the oracle's outputs for request r of the serving stream)."""
    r, n_r, seed, M = args
    import oracle
    import synth
    s, d, t, V = synth.request_graph(r, n_r, seed)
    res = oracle.cluster(s, d, t, M, V, tier=1)
    if res.status != 0:
        return r, "status %d" % res.status
    return r, digest_fields(lambda f: getattr(res, f), res.m, res.n_clusters, res.n_labels)
