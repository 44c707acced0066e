"""Determinism: the outputs depend only on the input, not on scheduling, atomics' order or tuning.

A 2M-record R-MAT graph (Hawkes times over 90 days) is clustered ten times with the default plan, then with
other dendrogram level plans (CE_KRT_LEVEL_BITS 2 and 9; the default takes 4), with the Boruvka filter split
forced from the first round and turned off (CE_SPLIT_MIN_EDGES 1 and 0), and on a second stream while the
first stream runs another call; every run must be byte-identical to the first and to the oracle.
"""
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster", "pt_lambda",
          "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected", "labels")


def _same(a, b, what):
    assert (a["m"], a["n_clusters"], a["n_labels"]) == (b["m"], b["n_clusters"], b["n_labels"]), what
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), (what, f)


@pytest.mark.timeout(300)
def test_ten_repeats_and_plans():
    import paper_2311_10337_amd as ce
    n, scale, M = 2_000_000, 17, 10
    src, dst, t = synth.rmat_hawkes(n, scale, seed=21)
    V = 1 << scale
    dev = torch.device("cuda:0")
    s_d, d_d, t_d = (torch.from_numpy(a).to(dev) for a in (src, dst, t))
    ws = torch.empty(ce.workspace_bytes(n, V, M), dtype=torch.uint8, device=dev)

    def run():
        return ce.to_numpy(ce.cluster_edges(s_d, d_d, t_d, M, V, workspace=ws))

    first = run()
    ref = oracle.cluster(src, dst, t, M, V, tier=1)
    assert ref.status == 0
    _same(first, {**{f: getattr(ref, f) for f in FIELDS}, "m": ref.m, "n_clusters": ref.n_clusters,
                  "n_labels": ref.n_labels}, "oracle")
    for k in range(9):
        _same(run(), first, "repeat %d" % (k + 1))
    saved = {k: os.environ.get(k) for k in ("CE_KRT_LEVEL_BITS", "CE_SPLIT_MIN_EDGES")}
    try:
        for key, val in (("CE_KRT_LEVEL_BITS", "2"), ("CE_KRT_LEVEL_BITS", "9"), ("CE_SPLIT_MIN_EDGES", "1"),
                         ("CE_SPLIT_MIN_EDGES", "0")):
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
            os.environ[key] = val
            _same(run(), first, "%s=%s" % (key, val))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    # the same call on a second stream, enqueued while another call runs on the first
    other = torch.cuda.Stream(device=dev)
    ws2 = torch.empty_like(ws)
    a_out = ce.Outputs(n, M, dev)
    b_out = ce.Outputs(n, M, dev)
    torch.cuda.synchronize()
    ra = ce.cluster_edges(s_d, d_d, t_d, M, V, outputs=a_out, workspace=ws)
    with torch.cuda.stream(other):
        rb = ce.cluster_edges(s_d, d_d, t_d, M, V, outputs=b_out, workspace=ws2, stream=other)
    torch.cuda.synchronize()
    _same(ce.to_numpy(ra), first, "first stream")
    _same(ce.to_numpy(rb), first, "second stream")
