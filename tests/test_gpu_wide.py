"""GPU parity over the whole time domain (Sec. 1.2.1 puts no bound on integer
times; spans up to 2^62 - 1 are accepted, as by the oracle).

When bits(span) + bits(n-1) + 1 exceeds the 63-bit key word, the key's weight
field holds the rank of the weight among the skeleton's distinct weights
(weight ranks): the order is the same, and the weights are read back from the
times. These tests drive inputs whose plain keys need 64 to 85 bits through
every mode (single graphs, asynchronous calls, batches, causal, hypergraphs,
the max_dt cutoff and the discrete dendrogram) and compare every output field
with the oracle; CE_WEIGHT_RANKS=1 forces the ranked layout on ordinary
inputs, and the span limit itself is checked on both sides.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster", "pt_lambda",
          "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected", "labels")
SPAN_LIMIT = 1 << 62


def _ce():
    import paper_2311_10337_amd as ce
    if not os.path.exists(ce.LIB_PATH):
        pytest.fail("libce.so is not built")
    return ce


def note(msg):
    print("[gpu-wide] " + msg, flush=True)
    sys.stdout.flush()


def dev(*arrays):
    d = torch.device("cuda:0")
    return [torch.from_numpy(np.ascontiguousarray(a)).to(d) for a in arrays]


def key_bits(t, n):
    span = int(t.max()) - int(t.min()) if n else 0
    return span.bit_length() + max(n - 1, 0).bit_length() + 1


def as_dict(r):
    out = {"m": r.m, "n_clusters": r.n_clusters, "n_labels": r.n_labels}
    for f in FIELDS:
        out[f] = getattr(r, f)
    return out


def same(got, ref, label):
    assert (got["m"], got["n_clusters"], got["n_labels"]) == (ref["m"], ref["n_clusters"], ref["n_labels"]), label
    for f in FIELDS:
        if not np.array_equal(got[f], ref[f]):
            raise AssertionError("%s: field %s differs" % (label, f))


def year_in_microseconds(n, V, seed):
    """Chung-Lu bursts over 365 days, times in microseconds (each second's records spread over it)."""
    s, d, t = synth.chung_lu_bursts(n, V, seed, T=365 * synth.DAY)
    rng = np.random.default_rng(seed + 1000)
    return s, d, t * 1_000_000 + rng.integers(0, 1_000_000, n)


def full_range(n, V, seed):
    """Chung-Lu endpoints, times uniform over [-2^61, 2^61): spans just below 2^62."""
    s, d, _ = synth.chung_lu_bursts(n, V, seed)
    rng = np.random.default_rng(seed + 2000)
    return s, d, rng.integers(-(1 << 61), (1 << 61) - 1, n, dtype=np.int64)


def coarse_wide(n, V, seed):
    """Times on a coarse grid of multiples of 2^41 below 2^61: wide keys with many equal weights (ties)."""
    s, d, _ = synth.chung_lu_bursts(n, V, seed)
    rng = np.random.default_rng(seed + 3000)
    return s, d, rng.integers(0, 1 << 20, n, dtype=np.int64) << 41


def ref_plain(s, d, t, V, M, causal=False, max_dt=-1):
    r = oracle.cluster(s, d, t, M, V, tier=1, causal=causal, max_dt=max_dt)
    assert r.status == 0
    return as_dict(r)


CASES = [("year-us", year_in_microseconds, 1_000_000, 50_000),
         ("full-range", full_range, 500_000, 20_000),
         ("coarse", coarse_wide, 300_000, 10_000),
         ("full-range-4M", full_range, 1 << 22, 1 << 17)]


@pytest.mark.timeout(600)
def test_wide_single_graphs():
    ce = _ce()
    for label, gen, n, V in CASES:
        s, d, t = gen(n, V, 7)
        kb = key_bits(t, n)
        assert kb > 63
        note("%s n=%d key bits %d" % (label, n, kb))
        got = ce.to_numpy(ce.cluster_edges(*dev(s, d, t), 5, V))
        same(got, ref_plain(s, d, t, V, 5), label)
        assert got["msf_w"].max() > (1 << 40)


def test_span_limits():
    ce = _ce()
    # the record's own key would need exactly 64 bits: n = 4, span 2^61 - 1
    s = np.array([0, 1, 2, 0], np.int32)
    d = np.array([1, 2, 0, 2], np.int32)
    t = np.array([0, 1 << 60, (1 << 61) - 1, 5], np.int64)
    assert key_bits(t, 4) == 64
    for causal in (False, True):
        got = ce.to_numpy(ce.cluster_edges(*dev(s, d, t), 2, 3, causal=causal))
        same(got, ref_plain(s, d, t, 3, 2, causal=causal), "64-bit key causal=%s" % causal)
    # the largest span accepted, then the first one refused, on both sides
    for span, ok in (((1 << 62) - 1, True), (1 << 62, False)):
        tt = np.array([-7, -7 + span // 3, -7 + span, 11], np.int64)
        r = oracle.cluster(s, d, tt, 2, 3, tier=1)
        if ok:
            assert r.status == 0
            same(ce.to_numpy(ce.cluster_edges(*dev(s, d, tt), 2, 3)), as_dict(r), "span 2^62-1")
        else:
            assert r.status == oracle.ERANGE
            with pytest.raises(ce.ClusterError) as e:
                ce.cluster_edges(*dev(s, d, tt), 2, 3)
            assert e.value.status == ce.CE_ERANGE


def test_wide_async_undeclared_span():
    ce = _ce()
    d0 = torch.device("cuda:0")
    for label, gen, n, V in CASES[:3]:
        s, d, t = gen(n, V, 11)
        ref = ref_plain(s, d, t, V, 5)
        outs = ce.Outputs(n, 5, d0)
        ws = torch.empty(ce.workspace_bytes(n, V, 5), dtype=torch.uint8, device=d0)
        hdr = torch.zeros(ce.hdr_words(1), dtype=torch.int64, device=d0)
        for tb in (0, 62):  # 0: no declared width (the ranked layout covers every span below 2^62)
            ce.cluster_edges_async(*dev(s, d, t), 5, V, outs, ws, hdr, time_bits=tb)
            same(ce.to_numpy(ce.async_result(outs, n, hdr)), ref, "%s async time_bits=%d" % (label, tb))


def _wide_batch(G, seed):
    rng = np.random.default_rng(seed)
    graphs = []
    for g in range(G):
        n = int(rng.choice([0, 1, 5, 300, 4000, 30000]))
        V = int(rng.integers(2, 400))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V - 1, n).astype(np.int32)
        d[d >= s] += 1
        kind = g % 3
        if kind == 0:
            t = rng.integers(-(1 << 61), (1 << 61) - 1, n, dtype=np.int64)
        elif kind == 1:
            t = rng.integers(0, 64, n, dtype=np.int64) << 55
        else:
            t = rng.integers(0, 365 * 86400 * 1_000_000, n, dtype=np.int64)
        graphs.append((s, d, t, V))
    eoff = np.cumsum([0] + [len(x[0]) for x in graphs]).astype(np.int64)
    voff = np.cumsum([0] + [x[3] for x in graphs]).astype(np.int64)
    cat = lambda k, dt: np.concatenate([np.asarray(x[k], dt) for x in graphs])
    return graphs, cat(0, np.int32), cat(1, np.int32), cat(2, np.int64), eoff, voff


def test_wide_batches_sync_and_async():
    ce = _ce()
    d0 = torch.device("cuda:0")
    graphs, src, dst, t, eoff, voff = _wide_batch(48, 5)
    G, n = len(graphs), int(eoff[-1])
    ins = dev(src, dst, t)
    br = ce.cluster_batch(*ins, eoff, voff, 3)
    outs = ce.batch_outputs(eoff, 3, d0)
    ws = torch.empty(ce.batch_workspace_bytes_for(n, G, 3), dtype=torch.uint8, device=d0)
    hdr = torch.zeros(ce.hdr_words(G), dtype=torch.int64, device=d0)
    eo, vo = dev(eoff, voff)
    ce.cluster_batch_async(*ins, eo, vo, int(voff[-1]), 3, outs, ws, hdr, time_bits=0)
    ar = ce.async_batch_result(outs, eoff, hdr)
    for g, (s, d, tt, V) in enumerate(graphs):
        ref = ref_plain(s, d, tt, V, 3)
        same(br.graph(g), ref, "batch graph %d" % g)
        same(ar.graph(g), ref, "async batch graph %d" % g)


def test_wide_causal():
    ce = _ce()
    for label, gen, n, V in CASES[:3]:
        s, d, t = gen(n // 2, V, 13)
        note("causal %s n=%d" % (label, n // 2))
        got = ce.to_numpy(ce.cluster_edges(*dev(s, d, t), 5, V, causal=True))
        same(got, ref_plain(s, d, t, V, 5, causal=True), "causal " + label)


def test_wide_hypergraphs():
    ce = _ce()
    mem, off, t = synth.hyper_bursts(200_000, 10_000, 17, T=365 * synth.DAY)
    rng = np.random.default_rng(17)
    for label, tt in (("year-us", t * 1_000_000 + rng.integers(0, 1_000_000, len(t))),
                      ("full-range", rng.integers(-(1 << 61), (1 << 61) - 1, len(t), dtype=np.int64))):
        r = oracle.cluster_hyper(mem, off, tt, 5, 10_000, tier=1)
        assert r.status == 0
        got = ce.to_numpy(ce.cluster_hyperedges(*dev(mem, off, tt), 5, 10_000))
        same(got, as_dict(r), "hyper " + label)


def test_wide_cutoff_and_discrete_levels():
    ce = _ce()
    s, d, t = year_in_microseconds(300_000, 20_000, 19)
    for cut in (0, 1_000_000, 3_600_000_000, (1 << 62)):
        got = ce.to_numpy(ce.cluster_edges(*dev(s, d, t), 5, 20_000, max_dt=cut))
        same(got, ref_plain(s, d, t, 20_000, 5, max_dt=cut), "cutoff %d" % cut)
    thr = [1_000_000 * 4 ** k for k in range(12)]
    r, dl, dt = oracle.cluster_discrete(s, d, t, 5, thr, 20_000)
    got = ce.to_numpy(ce.cluster_edges(*dev(s, d, t), 5, 20_000, thresholds=thr))
    same(got, as_dict(r), "discrete levels")


def test_forced_ranks_on_ordinary_inputs():
    ce = _ce()
    w = synth.plain_tiny(seed=23)
    hw = synth.hyper_tiny(seed=24, n=100_000)
    os.environ["CE_WEIGHT_RANKS"] = "1"
    try:
        for causal in (False, True):
            got = ce.to_numpy(ce.cluster_edges(*dev(w.src, w.dst, w.t), 5, w.num_vertices, causal=causal))
            same(got, ref_plain(w.src, w.dst, w.t, w.num_vertices, 5, causal=causal), "forced causal=%s" % causal)
        r = oracle.cluster_hyper(hw.members, hw.offsets, hw.t, 5, hw.num_vertices, tier=1)
        got = ce.to_numpy(ce.cluster_hyperedges(*dev(hw.members, hw.offsets, hw.t), 5, hw.num_vertices))
        same(got, as_dict(r), "forced hyper")
    finally:
        del os.environ["CE_WEIGHT_RANKS"]
