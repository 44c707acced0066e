"""GPU parity with Borůvka's filter split forced on small graphs.

The split (light edges first, heavy edges contracted once afterwards) runs by
default only from 2^20 live edges on, which the full-size and scaled workloads
reach. CE_SPLIT_MIN_EDGES lowers that bar, so here it runs on graphs the
oracle finishes in a moment, in every mode and in a batch, at several
thresholds (so it starts after different rounds), and must leave every
output bit-exact.
"""
import os

import numpy as np
import pytest

import synth
import test_gpu_batch as batch
import test_gpu_causal as causal
import test_gpu_hyper as hyper
import test_gpu_parity as undirected

pytestmark = pytest.mark.gpu


@pytest.fixture
def split_at():
    old = os.environ.get("CE_SPLIT_MIN_EDGES")

    def set_(v):
        os.environ["CE_SPLIT_MIN_EDGES"] = str(v)

    yield set_
    if old is None:
        os.environ.pop("CE_SPLIT_MIN_EDGES", None)
    else:
        os.environ["CE_SPLIT_MIN_EDGES"] = old


def test_undirected(split_at):
    rng = np.random.default_rng(101)
    for k in range(12):
        n = int(rng.integers(600, 30000))
        V = int(rng.integers(20, 2000))
        src, dst, t = synth.chung_lu_bursts(n, V, int(rng.integers(1, 1 << 30)))
        for thr in (1, 2000):
            split_at(thr)
            undirected.assert_parity(src, dst, t, V, int(rng.choice([2, 5, 10])), "split%d thr=%d" % (k, thr))


def test_tiny_workload_and_ties(split_at):
    w = synth.plain_tiny()
    split_at(64)
    undirected.assert_parity(w.src, w.dst, w.t, w.num_vertices, w.min_cluster_size, "tiny thr=64")
    # few distinct times: many equal weights, keys ordered by ids
    rng = np.random.default_rng(7)
    n, V = 20000, 300
    src = rng.integers(0, V, n).astype(np.int32)
    dst = ((src + rng.integers(1, V, n)) % V).astype(np.int32)
    t = rng.integers(0, 4, n).astype(np.int64)
    undirected.assert_parity(src, dst, t, V, 5, "ties thr=64")


def test_causal(split_at):
    rng = np.random.default_rng(103)
    for k in range(6):
        n = int(rng.integers(600, 20000))
        V = int(rng.integers(20, 1000))
        src, dst, t = synth.chung_lu_bursts(n, V, int(rng.integers(1, 1 << 30)))
        for thr in (1, 500):
            split_at(thr)
            causal.assert_parity(src, dst, t, V, 5, "causal split%d thr=%d" % (k, thr))


def test_hypergraph(split_at):
    rng = np.random.default_rng(107)
    for k in range(6):
        n = int(rng.integers(600, 8000))
        V = int(rng.integers(20, 400))
        mem, off = hyper.csr(hyper.random_sets(rng, n, V, 6))
        t = rng.integers(0, 100000, n).astype(np.int64)
        for thr in (1, 500):
            split_at(thr)
            hyper.check(mem, off, t, V, 4, "hyper split%d thr=%d" % (k, thr))


def test_batch(split_at):
    rng = np.random.default_rng(109)
    graphs = []
    for g in range(24):
        n = int(rng.integers(1, 6000))
        s, d, t, V = synth.batch_graph(g, n, seed=11)
        graphs.append((s, d, t, V))
    for thr in (1, 3000):
        split_at(thr)
        batch.check_batch_vs_oracle(graphs, 5, "batch thr=%d" % thr)


def test_switched_off(split_at):
    w = synth.plain_tiny()
    split_at(0)
    undirected.assert_parity(w.src, w.dst, w.t, w.num_vertices, w.min_cluster_size, "tiny, split off")
