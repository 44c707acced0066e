"""GPU parity: the HIP path through the C ABI equals the CPU oracle element by element.

All outputs are integers (no floating point anywhere on the path), so the bar
is bit-exact equality on every field: MSF rows, dendrogram rows, per-record
exits, cluster rows with exact u128 stabilities, selection flags and labels.
"""
import os
import sys

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
    print("[gpu-parity] " + msg, flush=True)
    sys.stdout.flush()


def run_gpu(src, dst, t, V, M):
    ce = _ce()
    dev = torch.device("cuda:0")
    s = torch.from_numpy(np.ascontiguousarray(src, np.int32)).to(dev)
    d = torch.from_numpy(np.ascontiguousarray(dst, np.int32)).to(dev)
    tt = torch.from_numpy(np.ascontiguousarray(t, np.int64)).to(dev)
    return ce.to_numpy(ce.cluster_edges(s, d, tt, M, V))


def assert_parity(src, dst, t, V, M, label=""):
    note("case %s n=%d V=%d M=%d" % (label, len(src), V, M))
    ref = oracle.cluster(src, dst, t, M, V, tier=1)
    assert ref.status == 0
    got = run_gpu(src, dst, t, V, M)
    assert got["m"] == ref.m and got["n_clusters"] == ref.n_clusters and got["n_labels"] == ref.n_labels, label
    for f in FIELDS:
        a, b = got[f], getattr(ref, f)
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0][:10] if a.shape == b.shape else "shape %s vs %s" % (a.shape, b.shape)
            raise AssertionError("%s: field %s differs at %s" % (label, f, bad))
    return got


def test_golden_tables():
    for name, M in (("table2_chain.txt", 2), ("table2_chain.txt", 5), ("table3_long.txt", 3)):
        s, d, t = load_golden(name)
        V = int(max(s.max(), d.max()) + 1)
        assert_parity(s, d, t, V, M, name)


def test_hand_fixtures():
    # two bursts on a star; exact EOM tie; all-equal times; matching graph; forest of three stars
    cases = [
        (np.zeros(4, np.int32), np.arange(1, 5, dtype=np.int32), np.array([0, 1, 10, 11], np.int64), 2),
        (np.zeros(6, np.int32), np.arange(1, 7, dtype=np.int32), np.array([0, 2, 5, 7, 13, 14], np.int64), 2),
        (np.zeros(7, np.int32), np.arange(1, 8, dtype=np.int32), np.full(7, 5, np.int64), 3),
        (np.arange(0, 20, 2, dtype=np.int32), np.arange(1, 21, 2, dtype=np.int32), np.arange(10, dtype=np.int64), 2),
        (np.array([0] * 6 + [10] * 6 + [20] * 2, np.int32), np.array(list(range(1, 7)) + list(range(11, 17)) + [21, 22],
                                                                     np.int32),
         np.array([0, 1, 2, 3, 4, 5, 0, 2, 4, 6, 8, 10, 0, 1], np.int64), 3),
    ]
    for i, (s, d, t, M) in enumerate(cases):
        assert_parity(s, d, t, int(max(s.max(), d.max()) + 1), M, "hand%d" % i)


def test_degenerate_sizes():
    ce = _ce()
    z32, z64 = np.zeros(0, np.int32), np.zeros(0, np.int64)
    got = run_gpu(z32, z32, z64, 4, 5)
    assert got["m"] == 0 and got["n_clusters"] == 1 and got["n_labels"] == 0
    assert list(got["cl_id"]) == [0] and list(got["cl_parent"]) == [ce.NONE32]
    assert_parity(np.array([0], np.int32), np.array([1], np.int32), np.array([7], np.int64), 2, 2, "n1")
    assert_parity(np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([7, 9], np.int64), 3, 2, "n2")


def test_random_tie_heavy_small():
    rng = np.random.default_rng(77)
    for it in range(150):
        n = int(rng.integers(2, 300))
        V = int(rng.integers(2, 40))
        src = rng.integers(0, V, n).astype(np.int32)
        dst = rng.integers(0, V, n).astype(np.int32)
        bad = src == dst
        dst[bad] = (src[bad] + 1) % V
        t = rng.integers(0, int(rng.integers(1, 200)), n).astype(np.int64) - int(rng.integers(0, 1000))
        assert_parity(src, dst, t, V, int(rng.integers(2, 8)), "rand%d" % it)


def test_ragged_sizes_across_tiles():
    """Sizes around the radix tile (2048 keys), the LDS dendrogram interval
    (512 rows) and the global level boundaries, with ragged tails."""
    for i, n in enumerate([511, 512, 513, 1023, 2047, 2048, 2049, 4097, 33000, 70001]):
        w = synth.chung_lu_bursts(n, max(2, n // 20), seed=100 + i)
        assert_parity(w[0], w[1], w[2], max(2, n // 20), 5, "ragged%d" % n)


def test_min_cluster_sizes_around_the_exit_paths():
    """Exits come from a top-down pass over small subtrees for M <= 64 and from a walk up from each record
    above that; both sides of the switch, on the tiny workload and on random graphs."""
    w = synth.plain_tiny()
    for M in (63, 64, 65, 200, 5000):
        assert_parity(w.src, w.dst, w.t, w.num_vertices, M, "tiny M=%d" % M)
    rng = np.random.default_rng(79)
    for it in range(20):
        n = int(rng.integers(100, 3000))
        V = int(rng.integers(2, 30))
        src = rng.integers(0, V, n).astype(np.int32)
        dst = rng.integers(0, V - 1, n).astype(np.int32)
        dst[dst >= src] += 1
        t = rng.integers(0, 500, n).astype(np.int64)
        assert_parity(src, dst, t, V, int(rng.choice([64, 65, 90, 300])), "bigM%d" % it)


def test_error_paths():
    ce = _ce()
    dev = torch.device("cuda:0")
    mk = lambda a, dt: torch.tensor(a, dtype=dt, device=dev)
    with pytest.raises(ce.ClusterError) as e:
        ce.cluster_edges(mk([0, 1], torch.int32), mk([1, 1], torch.int32), mk([0, 1], torch.int64), 2, 3)
    assert e.value.status == ce.CE_ESELFLOOP
    with pytest.raises(ce.ClusterError) as e:
        ce.cluster_edges(mk([0, 5], torch.int32), mk([1, 1], torch.int32), mk([0, 1], torch.int64), 2, 3)
    assert e.value.status == ce.CE_ERANGE
    with pytest.raises(ce.ClusterError) as e:
        ce.cluster_edges(mk([0, 1], torch.int32), mk([1, 2], torch.int32), mk([0, 1], torch.int64), 1, 3)
    assert e.value.status == ce.CE_EINVAL
    with pytest.raises(ce.ClusterError) as e:  # a span of 2^63 - 1: at least 2^62 is refused
        ce.cluster_edges(mk([0, 1, 2], torch.int32), mk([1, 2, 3], torch.int32),
                         mk([-(1 << 62), 0, (1 << 62) - 1], torch.int64), 2, 4)
    assert e.value.status == ce.CE_ERANGE


def test_tiny_workload_full():
    """Chung-Lu (exponent 2.1) endpoints, Poisson-burst times over 30 days:
    10k vertices, 200k records, M=5 -- every output element vs the oracle."""
    w = synth.plain_tiny()
    assert_parity(w.src, w.dst, w.t, w.num_vertices, w.min_cluster_size, "tiny")


def test_rmat_hawkes_scaled():
    """R-MAT (.57,.19,.19,.05) endpoints with per-pair Hawkes times over 90 days,
    scaled down to 2M records on 2^17 vertices (hubs ~1e4), M=10."""
    s, d, t = synth.rmat_hawkes(2_000_000, 17, seed=11)
    assert_parity(s, d, t, 1 << 17, 10, "rmat2M")


def test_determinism_repeated_runs():
    w = synth.plain_tiny(seed=5, n=100_000, V=5000)
    a = run_gpu(w.src, w.dst, w.t, w.num_vertices, 5)
    for _ in range(3):
        b = run_gpu(w.src, w.dst, w.t, w.num_vertices, 5)
        for f in FIELDS:
            assert np.array_equal(a[f], b[f]), f


@pytest.mark.timeout(1200)
def test_mid_workload_full_size():
    """The benchmark's workload at full size (R-MAT scale 20, 50M records,
    per-pair Hawkes times over 90 days, M=10), in the configuration bench.py
    times (preallocated workspace and outputs): every output element vs the
    oracle (about two minutes of single-threaded oracle time)."""
    ce = _ce()
    w = synth.plain_mid()
    dev = torch.device("cuda:0")
    src, dst, tt = (torch.from_numpy(a).to(dev) for a in (w.src, w.dst, w.t))
    outs = ce.Outputs(w.n, w.min_cluster_size, dev)
    ws = torch.empty(ce.workspace_bytes(w.n, w.num_vertices, w.min_cluster_size), dtype=torch.uint8, device=dev)
    note("mid full size: GPU run")
    got = ce.to_numpy(ce.cluster_edges(src, dst, tt, w.min_cluster_size, w.num_vertices, outputs=outs, workspace=ws))
    del src, dst, tt, outs, ws
    note("mid full size: oracle run (m=%d)" % got["m"])
    ref = oracle.cluster(w.src, w.dst, w.t, w.min_cluster_size, w.num_vertices, tier=1)
    note("mid full size: comparing")
    assert got["m"] == ref.m and got["n_clusters"] == ref.n_clusters and got["n_labels"] == ref.n_labels
    for f in FIELDS:
        assert np.array_equal(got[f], getattr(ref, f)), f
