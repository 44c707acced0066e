"""Full-oracle parity on the paths that set the 2^30-record workload apart, at a size the oracle finishes
in about a minute: an R-MAT graph of 5e7 records whose largest vertex has a planted degree of about 1e7,
Hawkes times over 365 days (25-bit time span), and the exact dendrogram built with three level plans: the
default one (two global levels of 9 and 8 bits here; 11 and 10 at 2^30 records), three levels of 6, 6 and 5
bits, and five levels of 4, 4, 3, 3 and 3 bits (CE_KRT_LEVEL_BITS, read on every call). Every output field
is compared with the oracle's (skeleton tier).
"""
import os
import time

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster", "pt_lambda",
          "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected", "labels")


@pytest.fixture
def live(capsys):
    def note(msg):
        with capsys.disabled():
            print("[gpu-hub] %s %s" % (time.strftime("%H:%M:%S"), msg), flush=True)
    return note


@pytest.mark.timeout(600)
def test_planted_hub_year_span_level_plans(live):
    import paper_2311_10337_amd as ce
    n, scale, M = 50_000_000, 22, 25
    src, dst, t = synth.rmat_hawkes(n, scale, seed=12, T=365 * synth.DAY, hub_extra=11_000_000)
    V = 1 << scale
    deg = np.bincount(src, minlength=V) + np.bincount(dst, minlength=V)
    assert deg.max() >= 10_000_000, deg.max()
    assert int(t.max() - t.min()).bit_length() == 25
    live("generated n=%d, hub degree %d" % (n, deg.max()))
    dev = torch.device("cuda:0")
    s_d, d_d, t_d = (torch.from_numpy(a).to(dev) for a in (src, dst, t))
    outs = ce.Outputs(n, M, dev)
    ws = torch.empty(ce.workspace_bytes(n, V, M), dtype=torch.uint8, device=dev)
    got = {}
    old = os.environ.get("CE_KRT_LEVEL_BITS")
    try:
        for bits in ("6", "4", None):
            if bits:
                os.environ["CE_KRT_LEVEL_BITS"] = bits
            else:
                os.environ.pop("CE_KRT_LEVEL_BITS", None)
            got[bits] = ce.to_numpy(ce.cluster_edges(s_d, d_d, t_d, M, V, outputs=outs, workspace=ws))
            live("gpu done with level bits %s: m=%d" % (bits or "default", got[bits]["m"]))
    finally:
        if old is None:
            os.environ.pop("CE_KRT_LEVEL_BITS", None)
        else:
            os.environ["CE_KRT_LEVEL_BITS"] = old
    del s_d, d_d, t_d, outs, ws
    torch.cuda.empty_cache()
    ref = oracle.cluster(src, dst, t, M, V, tier=1)
    live("oracle done: m=%d clusters=%d labels=%d" % (ref.m, ref.n_clusters, ref.n_labels))
    assert ref.status == 0
    for bits, g in got.items():
        assert (g["m"], g["n_clusters"], g["n_labels"]) == (ref.m, ref.n_clusters, ref.n_labels), bits
        for f in FIELDS:
            assert np.array_equal(g[f], getattr(ref, f)), (bits, f)
