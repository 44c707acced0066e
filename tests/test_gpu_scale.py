"""Parity at the 2^30-record single-graph workload (R-MAT scale 26, planted hub,
365-day Hawkes times, M = 25), in the launch configuration bench.py times.

The full oracle would need hours of one host core here, so the MSF is checked
by the properties that pin it, the dendrogram exactly by the oracle's
union-find on the GPU's MSF rows, and the condensed tree, stabilities,
selection and labels exactly by the oracle's condensing on the GPU's
dendrogram rows (tests/scale_checks.py).

The condensed half (about three minutes, 70 GB of host memory) runs with
every GPU test run. The MSF and dendrogram half needs about thirteen minutes
and 200 GB of host memory; it runs only with CE_SCALE_TEST=1, in a process
of its own (-k msf), so that the oracle's progress lines (CE_ORACLE_PROGRESS,
read once per process) are on.
"""
import os
import sys
import time

import pytest

import synth
from scale_checks import check_condensed, check_msf_and_dendrogram

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu]
long_check = pytest.mark.skipif(os.environ.get("CE_SCALE_TEST") != "1",
                                reason="2^30-record MSF check: set CE_SCALE_TEST=1 (13 minutes, 200 GB host)")


_capsys = None


def _say(msg):
    print("[gpu-scale] %s %s" % (time.strftime("%H:%M:%S"), msg), flush=True)


def note(msg):
    """Progress lines go straight to the terminal (output capture suspended), so a long check is seen working."""
    if _capsys is not None:
        with _capsys.disabled():
            _say(msg)
    else:
        _say(msg)


@pytest.fixture(autouse=True)
def _live_progress(capsys):
    global _capsys
    _capsys = capsys
    yield
    _capsys = None


def run_scale(keep_inputs):
    import gc
    import paper_2311_10337_amd as ce
    gc.collect()
    torch.cuda.empty_cache()  # the 2^30-record call needs about 250 GB of the 288 GB
    note("start")
    w = synth.plain_scale()
    note("generated n=%d V=%d" % (w.n, w.num_vertices))
    dev = torch.device("cuda:0")
    s_d = torch.from_numpy(w.src).to(dev)
    d_d = torch.from_numpy(w.dst).to(dev)
    t_d = torch.from_numpy(w.t).to(dev)
    res = ce.cluster_edges(s_d, d_d, t_d, w.min_cluster_size, w.num_vertices)
    del s_d, d_d, t_d
    got = ce.to_numpy(res)
    del res
    torch.cuda.empty_cache()
    note("gpu done: m=%d clusters=%d labels=%d" % (got["m"], got["n_clusters"], got["n_labels"]))
    data = {"src": w.src, "dst": w.dst, "t": w.t, "V": w.num_vertices} if keep_inputs else None
    return w.n, w.min_cluster_size, data, got


@long_check
@pytest.mark.timeout(1150)
def test_scale_msf_and_dendrogram(monkeypatch):
    # the oracle's union-find passes over 2^30 rows take minutes each: they report every 2^26 rows on stderr,
    # which reaches the terminal while output capture is suspended
    monkeypatch.setenv("CE_ORACLE_PROGRESS", "1")
    n, M, data, got = run_scale(True)
    for f in ("pt_cluster", "pt_lambda", "labels"):
        del got[f]
    with _capsys.disabled():
        check_msf_and_dendrogram(data, got, log=_say)


@pytest.mark.timeout(600)
def test_scale_condensed():
    n, M, _, got = run_scale(False)
    for f in ("msf_tail", "msf_head", "msf_w"):
        del got[f]
    check_condensed(n, M, got, log=note)
