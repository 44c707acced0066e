"""GPU tests of the serving loop: continuous batching returns, for every request,
exactly the result it gets alone (and the oracle's, where checked), isolates
data errors to their request, and enforces its memory and in-flight limits.
"""
import os
import sys
import time

import numpy as np
import pytest

import oracle
import synth
from conftest import load_golden

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster", "pt_lambda",
          "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected", "labels")


def _ce():
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.fail("libce.so is not built")
    return ce


def note(msg):
    print("[gpu-serve] " + msg, flush=True)
    sys.stdout.flush()


def same(got, ref, label):
    assert (got["m"], got["n_clusters"], got["n_labels"]) == (ref["m"], ref["n_clusters"], ref["n_labels"]), label
    for f in FIELDS:
        if not np.array_equal(got[f], ref[f]):
            raise AssertionError("%s: field %s differs" % (label, f))


def alone(req):
    ce = _ce()
    s, d, t, V, M = req
    dev = torch.device("cuda:0")
    r = ce.cluster_edges(torch.from_numpy(np.ascontiguousarray(s, np.int32)).to(dev),
                         torch.from_numpy(np.ascontiguousarray(d, np.int32)).to(dev),
                         torch.from_numpy(np.ascontiguousarray(t, np.int64)).to(dev), M, V)
    return ce.to_numpy(r)


def oracle_dict(req):
    s, d, t, V, M = req
    r = oracle.cluster(s, d, t, M, V, tier=1)
    assert r.status == 0
    out = {"m": r.m, "n_clusters": r.n_clusters, "n_labels": r.n_labels}
    for f in FIELDS:
        out[f] = getattr(r, f)
    return out


def serve_all(srv, reqs):
    """Submit every request (retrying while the server is full) and collect the results by index."""
    ce = _ce()
    pending, results = {}, {}
    i = 0
    while i < len(reqs) or pending:
        while i < len(reqs):
            s, d, t, V, M = reqs[i]
            try:
                pending[srv.submit(s, d, t, M, V)] = i
                i += 1
            except ce.ServerBusy:
                break
        for tk in list(pending):
            r = srv.poll(tk)
            if r is not None:
                results[pending.pop(tk)] = r
        if pending and i >= len(reqs):
            tk = next(iter(pending))
            results[pending.pop(tk)] = srv.poll(tk, wait=True)
    return [results[k] for k in range(len(reqs))]


def request_mix():
    reqs = []
    sizes = np.minimum(synth.request_sizes(20000, seed=4)[:36], 300_000)
    for r in range(36):
        s, d, t, V = synth.request_graph(r, int(sizes[r]), seed=4)
        reqs.append((s, d, t, V, 10))
    for name, M in (("table2_chain.txt", 2), ("table3_long.txt", 3)):
        s, d, t = load_golden(name)
        reqs.insert(len(reqs) // 2, (s, d, t, int(max(s.max(), d.max()) + 1), M))
    e32, e64 = np.zeros(0, np.int32), np.zeros(0, np.int64)
    reqs.insert(5, (e32, e32, e64, 3, 10))
    reqs.insert(9, (np.array([0], np.int32), np.array([1], np.int32), np.array([4], np.int64), 2, 10))
    reqs.insert(12, (np.zeros(6, np.int32), np.arange(1, 7, dtype=np.int32),
                     np.array([0, 2, 5, 7, 13, 14], np.int64), 7, 2))
    return reqs


def test_mixed_equals_alone():
    ce = _ce()
    reqs = request_mix()
    note("%d requests, %d records" % (len(reqs), sum(len(r[0]) for r in reqs)))
    refs = [alone(r) for r in reqs]
    # small requests also against the oracle
    for k, r in enumerate(reqs):
        if len(r[0]) <= 20_000:
            same(refs[k], oracle_dict(r), "alone request %d vs oracle" % k)
    with ce.Server(8 << 30, workers=3, max_inflight=64, max_batch_records=400_000) as srv:
        got = serve_all(srv, reqs)
        st = srv.stats()
    note("stats %s" % st)
    for k, g in enumerate(got):
        assert g.status == ce.CE_OK, (k, g.error)
        same(ce.to_numpy(g.result), refs[k], "mixed request %d" % k)
        assert 0 <= g.queue_s <= g.latency_s
    assert st["requests_done"] == len(reqs)
    assert st["batches"] < len(reqs), "requests were not batched"
    assert st["max_batch_requests"] >= 2
    assert st["max_concurrent_batches"] >= 2, "batches did not overlap"
    # the same requests through the server one at a time
    with ce.Server(8 << 30, workers=1, max_inflight=4) as srv:
        for k in range(0, len(reqs), 7):
            s, d, t, V, M = reqs[k]
            tk = srv.submit(s, d, t, M, V)
            g = srv.poll(tk, wait=True)
            assert g.status == ce.CE_OK
            same(ce.to_numpy(g.result), refs[k], "served alone request %d" % k)


def test_data_error_stays_with_its_request():
    ce = _ce()
    reqs = request_mix()[:12]
    s, d, t, V, M = reqs[3]
    d = d.copy()
    d[len(d) // 2] = s[len(d) // 2]  # a self loop
    reqs[3] = (s, d, t, V, M)
    s, d, t, V, M = reqs[7]
    s = s.copy()
    s[0] = V  # outside [0, V)
    reqs[7] = (s, d, t, V, M)
    with ce.Server(4 << 30, workers=2, max_inflight=64) as srv:
        got = serve_all(srv, reqs)
    assert got[3].status == ce.CE_ESELFLOOP and got[3].result is None
    assert got[7].status == ce.CE_ERANGE
    for k, g in enumerate(got):
        if k not in (3, 7):
            assert g.status == ce.CE_OK, (k, g.error)
            same(ce.to_numpy(g.result), alone(reqs[k]), "request %d next to failing ones" % k)


def test_admission_limits():
    ce = _ce()
    reqs = request_mix()[:10]
    big = max(len(r[0]) for r in reqs)
    need = ce.server_request_bytes(big, 1 << 16, 10)
    # a budget that holds about one of the largest requests at a time: still every result is right
    with ce.Server(int(need * 1.6), workers=2, max_inflight=3, input_fraction_pct=40) as srv:
        got = serve_all(srv, reqs)
        st = srv.stats()
        assert st["work_peak_bytes"] <= st["work_capacity_bytes"]
        assert st["input_peak_bytes"] <= st["input_capacity_bytes"]
        # in-flight limit
        tickets = []
        with pytest.raises(ce.ServerBusy):
            for _ in range(4):
                s, d, t, V, M = reqs[0]
                tickets.append(srv.submit(s, d, t, M, V))
        for tk in tickets:
            assert srv.poll(tk, wait=True).status == ce.CE_OK
        # a request that can never fit
        s, d, t, V = synth.request_graph(0, 3_000_000, seed=4)
        with pytest.raises(ce.ClusterError) as ei:
            srv.submit(s, d, t, 10, V)
        assert ei.value.status == ce.CE_ENOMEM
    for k, g in enumerate(got):
        assert g.status == ce.CE_OK
        same(ce.to_numpy(g.result), alone(reqs[k]), "tight-budget request %d" % k)


def test_open_loop_arrivals_small():
    """A short open-loop replay: arrivals at their scheduled times, every result checked."""
    ce = _ce()
    sizes = np.minimum(synth.request_sizes(20000, seed=4)[:60], 200_000)
    arr = synth.request_arrivals(20000, seed=4)[:60]
    reqs = [synth.request_graph(r, int(sizes[r]), seed=4) for r in range(60)]
    reqs = [(s, d, t, V, 10) for (s, d, t, V) in reqs]
    lat = []
    with ce.Server(8 << 30, workers=2, max_inflight=64) as srv:
        t0 = time.perf_counter()
        pending = {}
        results = {}
        for k in range(60):
            while time.perf_counter() - t0 < arr[k] - arr[0]:
                for tk in list(pending):
                    r = srv.poll(tk)
                    if r is not None:
                        results[pending.pop(tk)] = r
                time.sleep(0.0005)
            s, d, t, V, M = reqs[k]
            pending[srv.submit(s, d, t, M, V)] = k
        for tk, k in list(pending.items()):
            results[k] = srv.poll(tk, wait=True)
    for k in range(60):
        assert results[k].status == ce.CE_OK
        lat.append(results[k].latency_s)
        if k % 6 == 0:
            same(ce.to_numpy(results[k].result), alone(reqs[k]), "open-loop request %d" % k)
    note("latency p50 %.2f ms p99 %.2f ms" % (1e3 * np.percentile(lat, 50), 1e3 * np.percentile(lat, 99)))


@pytest.fixture
def live(capsys):
    """Progress lines that reach the terminal while the test runs (long tests print as they go)."""
    def say(msg):
        with capsys.disabled():
            print("[gpu-serve] %s %s" % (time.strftime("%H:%M:%S"), msg), flush=True)
    return say


@pytest.mark.timeout(900)
def test_stream_prefix_against_the_oracle(live):
    """The first 1 000 requests of the serving stream (about 2.1e8 records, sizes up to the stream's 5e6)
    served with continuous batching, up to 256 in flight: every request's outputs equal the oracle's on that
    request alone (digests of every field; afterwards the oracle runs in 16 host processes that regenerate
    each request from its seed)."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor, ThreadPoolExecutor, as_completed
    import oracle_digests
    ce = _ce()
    count, M, seed = 1000, 10, 4
    sizes = synth.request_sizes(20000, seed=seed)[:count]
    live("stream prefix: %d requests, %d records, largest %d" % (count, int(sizes.sum()), int(sizes.max())))
    with ThreadPoolExecutor(max_workers=16) as ex:
        reqs = list(ex.map(lambda r: synth.request_graph(r, int(sizes[r]), seed), range(count)))
    live("generated")
    got = {}
    with ce.Server(32 << 30, workers=3, max_inflight=256) as srv:
        pending = {}
        k = 0
        while k < count or pending:
            while k < count and len(pending) < 256:
                s, d, t, V = reqs[k]
                try:
                    pending[srv.submit(s, d, t, M, V)] = k
                except ce.ServerBusy:
                    break
                k += 1
            done = False
            for tk in list(pending):
                r = srv.poll(tk)
                if r is not None:
                    kk = pending.pop(tk)
                    assert r.status == ce.CE_OK, (kk, r.error)
                    h = ce.to_numpy(r.result)
                    got[kk] = oracle_digests.digest_fields(lambda f: h[f], h["m"], h["n_clusters"], h["n_labels"])
                    done = True
                    if len(got) % 200 == 0:
                        live("served and digested %d" % len(got))
            if not done:
                time.sleep(0.0005)
    del reqs
    live("oracle on every request in 16 processes")
    ref = {}
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1),
                             mp_context=multiprocessing.get_context("spawn")) as ex:
        futs = [ex.submit(oracle_digests.request_digest, (int(r), int(sizes[r]), seed, M))
                for r in np.argsort(-sizes)]  # largest first, so the pool drains evenly
        for fut in as_completed(futs):
            r, dg = fut.result()
            ref[r] = dg
            if len(ref) % 50 == 0:
                live("oracle %d" % len(ref))
    bad = [r for r in range(count) if ref[r] != got[r]]
    assert not bad, "requests differing from the oracle: %s" % bad[:10]
    live("all %d requests equal the oracle" % count)
