"""The asynchronous boundary: enqueue-only calls, a device header read by ce_result_status, and HIP-graph
capture and replay of a whole call.

* Two calls enqueued on two streams with no host synchronisation in between both equal the oracle.
* Data errors (self loop, id out of range, a time span wider than the declared time_bits, bad device
  offsets) are reported in the device header, and no output is written.
* A batch with device offsets equals the synchronous batch call graph by graph.
* The 4096-graph batch (about 2.4e8 records) captured in a HIP graph and replayed equals the uncaptured call
  on every output; replays are checked with the program's own eager work and synchronisations between them.
* A captured single-graph call replayed on new contents of the same input buffers equals the uncaptured
  call on those contents and the oracle.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster", "pt_lambda",
          "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected", "labels")


def _oracle(s, d, t, V, M):
    r = oracle.cluster(s, d, t, M, V, tier=1)
    assert r.status == 0
    return r


def _same_as_oracle(got, ref, label):
    assert (got["m"], got["n_clusters"], got["n_labels"]) == (ref.m, ref.n_clusters, ref.n_labels), label
    for f in FIELDS:
        assert np.array_equal(got[f], getattr(ref, f)), (label, f)


def _dev(*arrays):
    dev = torch.device("cuda:0")
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrays]


def test_two_streams_no_host_sync():
    import paper_2311_10337_amd as ce
    dev = torch.device("cuda:0")
    ga = synth.plain_tiny(seed=31, n=150_000, V=7000)
    gb = synth.rmat_hawkes(400_000, 14, seed=32)
    cases = [(ga.src, ga.dst, ga.t, ga.num_vertices, 5), (gb[0], gb[1], gb[2], 1 << 14, 10)]
    streams = [torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)]
    state = []
    for (s, d, t, V, M), st in zip(cases, streams):
        n = len(s)
        ins = _dev(s, d, t)
        outs = ce.Outputs(n, M, dev)
        ws = torch.empty(ce.workspace_bytes(n, V, M), dtype=torch.uint8, device=dev)
        hdr = torch.zeros(ce.hdr_words(1), dtype=torch.int64, device=dev)
        state.append((ins, outs, ws, hdr, n, st))
    torch.cuda.synchronize()
    for (ins, outs, ws, hdr, n, st), (s, d, t, V, M) in zip(state, cases):
        ce.cluster_edges_async(*ins, M, V, outs, ws, hdr, time_bits=40, stream=st)
    # both calls are in flight; no host wait between the two enqueues
    for (ins, outs, ws, hdr, n, st), (s, d, t, V, M) in zip(state, cases):
        got = ce.to_numpy(ce.async_result(outs, n, hdr, stream=st))
        _same_as_oracle(got, _oracle(s, d, t, V, M), "stream call n=%d" % n)


def test_data_errors_in_the_header():
    import paper_2311_10337_amd as ce
    dev = torch.device("cuda:0")
    s = np.array([0, 1, 2, 3], np.int32)
    d = np.array([1, 2, 3, 0], np.int32)
    t = np.array([0, 5, 9, 14], np.int64)
    outs = ce.Outputs(4, 2, dev)
    ws = torch.empty(ce.workspace_bytes(4, 4, 2), dtype=torch.uint8, device=dev)
    hdr = torch.zeros(ce.hdr_words(1), dtype=torch.int64, device=dev)
    sentinel = torch.full_like(outs.t["labels"], 77)
    for label, (ss, dd, tt, bits, want) in {
            "self loop": (np.array([0, 1, 3, 3], np.int32), d, t, 8, ce.CE_ESELFLOOP),
            "id out of range": (s, np.array([1, 2, 9, 0], np.int32), t, 8, ce.CE_ERANGE),
            "span wider than time_bits": (s, d, np.array([0, 5, 9, 300], np.int64), 8, ce.CE_ERANGE)}.items():
        outs.t["labels"].copy_(sentinel)
        ce.cluster_edges_async(*_dev(ss, dd, tt), 2, 4, outs, ws, hdr, time_bits=bits)
        with pytest.raises(ce.ClusterError) as e:
            ce.result_status(hdr, 1)
        assert e.value.status == want, label
        assert torch.equal(outs.t["labels"], sentinel), label  # nothing written
    # the same records within the declared span
    ce.cluster_edges_async(*_dev(s, d, t), 2, 4, outs, ws, hdr, time_bits=8)
    _same_as_oracle(ce.to_numpy(ce.async_result(outs, 4, hdr)), _oracle(s, d, t, 4, 2), "cycle")
    # host-checked arguments: a declared width beyond the time domain, no workspace, causal mode
    import ctypes
    lib = ce.load_library()
    p = ce.make_params(2, 4, time_bits=63)
    args = [ctypes.c_void_p(x.data_ptr()) for x in _dev(s, d, t)]
    assert lib.ce_cluster_edges_async(*args, 4, ctypes.byref(p), ctypes.byref(outs.struct),
                                      ctypes.c_void_p(hdr.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                      None) == ce.CE_EINVAL
    p = ce.make_params(2, 4, time_bits=8)
    assert lib.ce_cluster_edges_async(*args, 4, ctypes.byref(p), ctypes.byref(outs.struct),
                                      ctypes.c_void_p(hdr.data_ptr()), None, 0, None) == ce.CE_EINVAL
    p = ce.make_params(2, 4, causal=True, time_bits=8)
    assert lib.ce_cluster_edges_async(*args, 4, ctypes.byref(p), ctypes.byref(outs.struct),
                                      ctypes.c_void_p(hdr.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                      None) == ce.CE_EINVAL


def _batch_inputs(G, seed):
    sizes = synth.batch_sizes(G, seed)
    return synth.batch_workload(G, seed=seed, sizes=sizes)


def test_batch_device_offsets_equal_the_batch_call():
    import paper_2311_10337_amd as ce
    dev = torch.device("cuda:0")
    src, dst, t, eoff, voff = _batch_inputs(96, 41)
    n, G, M = int(eoff[-1]), 96, 5
    ins = _dev(src, dst, t)
    ref = ce.cluster_batch(*ins, eoff, voff, M)
    outs = ce.batch_outputs(eoff, M, dev)
    ws = torch.empty(ce.batch_workspace_bytes_for(n, G, M), dtype=torch.uint8, device=dev)
    hdr = torch.zeros(ce.hdr_words(G), dtype=torch.int64, device=dev)
    eo, vo = _dev(eoff, voff)
    ce.cluster_batch_async(*ins, eo, vo, int(voff[-1]), M, outs, ws, hdr, time_bits=32)
    got = ce.async_batch_result(outs, eoff, hdr)
    for a, b in ((got.m, ref.m), (got.n_clusters, ref.n_clusters), (got.n_labels, ref.n_labels),
                 (got.row_offsets, ref.row_offsets), (got.cluster_offsets, ref.cluster_offsets)):
        assert np.array_equal(a, b)
    for g in range(G):
        x, y = got.graph(g), ref.graph(g)
        for f in FIELDS:
            assert np.array_equal(x[f], y[f]), (g, f)
    # offsets that do not start at 0 are an argument error found on the device
    bad = eo.clone()
    bad[0] = 1
    ce.cluster_batch_async(*ins, bad, vo, int(voff[-1]), M, outs, ws, hdr, time_bits=32)
    with pytest.raises(ce.ClusterError) as e:
        ce.result_status(hdr, G)
    assert e.value.status == ce.CE_EINVAL


def _snapshot(outs, counts):
    rows, recs, cls = counts
    return {f: outs.t[f][:(recs if f in ("pt_cluster", "pt_lambda", "labels") else cls if f.startswith("cl_")
                           else rows)].clone() for f in FIELDS}


@pytest.mark.timeout(600)
def test_captured_4096_graph_batch_replays_equal():
    import paper_2311_10337_amd as ce
    dev = torch.device("cuda:0")
    src, dst, t, eoff, voff = synth.batch_workload(4096, seed=3)
    n, G, M = int(eoff[-1]), 4096, 5
    ins = _dev(src, dst, t)
    eo, vo = _dev(eoff, voff)
    outs = ce.batch_outputs(eoff, M, dev)
    ws = torch.empty(ce.batch_workspace_bytes_for(n, G, M), dtype=torch.uint8, device=dev)
    hdr = torch.zeros(ce.hdr_words(G), dtype=torch.int64, device=dev)
    # uncaptured
    ce.cluster_batch_async(*ins, eo, vo, int(voff[-1]), M, outs, ws, hdr, time_bits=32)
    ref = ce.async_batch_result(outs, eoff, hdr)
    counts = (int(ref.row_offsets[-1]), n, int(ref.cluster_offsets[-1]))
    want = _snapshot(outs, counts)
    want_hdr = hdr.clone()
    # captured once, replayed three times with eager work and synchronisations in between
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            ce.cluster_batch_async(*ins, eo, vo, int(voff[-1]), M, outs, ws, hdr, time_bits=32,
                                   stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    for k in range(3):
        for f in FIELDS:
            outs.t[f].fill_(2 if f == "cl_selected" else -1)
        hdr.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(hdr, want_hdr), "replay %d header" % k
        got = _snapshot(outs, counts)
        for f in FIELDS:
            assert torch.equal(got[f], want[f]), ("replay %d" % k, f)
        ws.fill_(0xA5)  # the next replay starts from a scrambled workspace


def test_captured_call_on_new_inputs():
    import paper_2311_10337_amd as ce
    dev = torch.device("cuda:0")
    n, V, M = 120_000, 6000, 5
    first = synth.plain_tiny(seed=51, n=n, V=V)
    ins = _dev(first.src, first.dst, first.t)
    outs = ce.Outputs(n, M, dev)
    ws = torch.empty(ce.workspace_bytes(n, V, M), dtype=torch.uint8, device=dev)
    hdr = torch.zeros(ce.hdr_words(1), dtype=torch.int64, device=dev)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            ce.cluster_edges_async(*ins, M, V, outs, ws, hdr, time_bits=24, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    for seed in (52, 53, 51):
        g = synth.plain_tiny(seed=seed, n=n, V=V)
        for dst_t, a in zip(ins, (g.src, g.dst, g.t)):
            dst_t.copy_(torch.from_numpy(a))
        torch.cuda.synchronize()
        graph.replay()
        got = ce.to_numpy(ce.async_result(outs, n, hdr))
        _same_as_oracle(got, _oracle(g.src, g.dst, g.t, V, M), "replay on seed %d" % seed)


def test_async_calls_are_not_timed():
    """Kernel timing (ce_timing_enable) covers synchronous calls only: an asynchronous call, also one captured
    in a HIP graph, records no events and gives the same outputs."""
    import paper_2311_10337_amd as ce
    dev = torch.device("cuda:0")
    n, V, M = 60_000, 3000, 5
    g = synth.plain_tiny(seed=61, n=n, V=V)
    ins = _dev(g.src, g.dst, g.t)
    outs = ce.Outputs(n, M, dev)
    ws = torch.empty(ce.workspace_bytes(n, V, M), dtype=torch.uint8, device=dev)
    hdr = torch.zeros(ce.hdr_words(1), dtype=torch.int64, device=dev)
    ref = _oracle(g.src, g.dst, g.t, V, M)
    ce.timing_enable("k_")
    try:
        ce.cluster_edges_async(*ins, M, V, outs, ws, hdr, time_bits=24)
        _same_as_oracle(ce.to_numpy(ce.async_result(outs, n, hdr)), ref, "timed async call")
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                ce.cluster_edges_async(*ins, M, V, outs, ws, hdr, time_bits=24, stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
        outs.t["labels"].fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        _same_as_oracle(ce.to_numpy(ce.async_result(outs, n, hdr)), ref, "captured call with timing on")
        ms, launches = ce.timing_read()
        assert launches == 0
        ce.cluster_edges(*ins, M, V, outputs=outs, workspace=ws)  # a synchronous call is timed
        ms, launches = ce.timing_read()
        assert launches > 100 and ms > 0
    finally:
        ce.timing_enable(None)
