"""The seeded input generators follow their stated recipes (host only).

Each check compares a generated sample with what the recipe's own parameters predict, with a slack of about
four standard errors where the quantity is random:

* Chung-Lu endpoints (exponent 2.1): the k-th largest expected degree falls as k^(-1/(gamma-1)), and the hub's
  degree is 2n w_0 / sum(w); the times come in bursts (per-vertex gaps far below those of uniform times);
* R-MAT (a, b, c) = (0.57, 0.19, 0.19): the largest source and destination degrees are n (a+b)^scale and
  n (a+c)^scale; a planted hub gains about as many records as were redirected to it; per-pair Hawkes times
  are spaced on the process's own time scales;
* lognormal sizes: median, spread (from the 16th and 84th percentiles, which the clipping does not reach) and
  the clipped fractions at both bounds;
* Poisson arrivals at 200 requests/s: mean gap 5 ms, coefficient of variation 1;
* every generator: no self loops, ids and times in range, the same arrays for the same seed, other arrays for
  another seed; a batch graph or a request is the same alone as inside its workload.
"""
import math

import numpy as np

import synth

DAY = 86400


def _basic(s, d, t, V, T):
    assert s.dtype == np.int32 and d.dtype == np.int32 and t.dtype == np.int64
    assert not np.any(s == d), "self loop"
    assert s.min() >= 0 and d.min() >= 0 and max(s.max(), d.max()) < V
    assert t.min() >= 0 and t.max() < T


def _rank_slope(deg, lo, hi):
    ds = np.sort(deg)[::-1].astype(np.float64)
    k = np.arange(lo, hi + 1)
    return np.polyfit(np.log(k), np.log(ds[k - 1]), 1)[0]


def _vertex_gaps(s, d, t):
    ends = np.concatenate([s, d])
    tt = np.concatenate([t, t])
    o = np.lexsort((tt, ends))
    e2, t2 = ends[o], tt[o]
    same = e2[1:] == e2[:-1]
    return (t2[1:] - t2[:-1])[same]


def test_chung_lu_bursts_tiny_recipe():
    w = synth.plain_tiny()
    assert (w.n, w.num_vertices, w.min_cluster_size) == (200_000, 10_000, 5)
    _basic(w.src, w.dst, w.t, w.num_vertices, 30 * DAY)
    deg = np.bincount(w.src, minlength=w.num_vertices) + np.bincount(w.dst, minlength=w.num_vertices)
    gamma = 2.1
    assert abs(_rank_slope(deg, 1, 100) - (-1.0 / (gamma - 1.0))) < 0.1
    wt = (np.arange(w.num_vertices) + 1.0) ** (-1.0 / (gamma - 1.0))
    hub = 2 * w.n * wt[0] / wt.sum()
    assert abs(deg.max() - hub) < 0.1 * hub, (deg.max(), hub)
    # bursts: consecutive records of a vertex are minutes apart, where uniform times would be hours apart
    gaps = _vertex_gaps(w.src, w.dst, w.t)
    assert np.median(gaps) < 600
    tu = np.random.default_rng(0).integers(0, 30 * DAY, w.n)
    assert np.median(_vertex_gaps(w.src, w.dst, tu)) > 3000


def test_rmat_degrees_hawkes_times_and_hub():
    n, scale = 2_000_000, 17
    a, b, c = 0.57, 0.19, 0.19
    V = 1 << scale
    s, d, t = synth.rmat_hawkes(n, scale, 1)
    _basic(s, d, t, V, 90 * DAY)
    out_top, in_top = np.bincount(s, minlength=V).max(), np.bincount(d, minlength=V).max()
    assert abs(out_top - n * (a + b) ** scale) < 0.05 * n * (a + b) ** scale
    assert abs(in_top - n * (a + c) ** scale) < 0.05 * n * (a + c) ** scale
    # per pair: the k earliest events of a Hawkes process (immigrants every 100 s, stationary rate 1/30 s,
    # offspring delays of mean 300 s)
    key = s.astype(np.int64) * V + d
    o = np.lexsort((t, key))
    k2, t2 = key[o], t[o]
    same = k2[1:] == k2[:-1]
    assert same.sum() > n // 20
    g = np.median((t2[1:] - t2[:-1])[same])
    assert 7.5 <= g <= 300, g
    # a planted hub: the redirected endpoints land on the largest vertex, never as a self loop
    extra = 500_000
    s2, d2, t2 = synth.rmat_hawkes(n, scale, 1, hub_extra=extra)
    _basic(s2, d2, t2, V, 90 * DAY)
    deg = np.bincount(s, minlength=V) + np.bincount(d, minlength=V)
    deg2 = np.bincount(s2, minlength=V) + np.bincount(d2, minlength=V)
    assert int(np.argmax(deg2)) == int(np.argmax(deg))
    assert deg.max() + 0.8 * extra <= deg2.max() <= deg.max() + extra


def _lognormal_checks(x, median, sigma, lo, hi):
    from scipy.stats import norm
    N = len(x)
    assert x.min() >= lo and x.max() <= hi
    se = 1.2533 * sigma / math.sqrt(N)  # standard error of the log of a sample median
    assert abs(math.log(np.median(x) / median)) < 4 * se
    q16, q84 = np.percentile(x, [15.865, 84.135])
    assert abs(0.5 * math.log(q84 / q16) - sigma) < 0.05 * sigma
    for bound, p in ((hi, norm.sf(math.log(hi / median) / sigma)), (lo, norm.cdf(math.log(lo / median) / sigma))):
        got = int(np.sum(x == bound))
        assert abs(got - N * p) <= 4 * math.sqrt(N * p * (1 - p)) + 1, (bound, got, N * p)


def test_batch_and_request_sizes():
    _lognormal_checks(synth.batch_sizes(4096, 3), 20000.0, 1.5, 500, 2_000_000)
    _lognormal_checks(synth.request_sizes(20000, 4), 70711.0, 1.42, 1000, 5_000_000)


def test_poisson_arrivals():
    a = synth.request_arrivals(20000, 200.0, 4)
    gaps = np.diff(np.concatenate([[0.0], a]))
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 0.005) < 4 * 0.005 / math.sqrt(len(gaps))
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05


def test_batch_graph_alone_equals_its_slice():
    G, seed = 16, 3
    src, dst, t, eoff, voff = synth.batch_workload(G, seed)
    sizes = synth.batch_sizes(G, seed)
    assert np.array_equal(np.diff(eoff), sizes)
    for g in (0, 5, 15):
        s, d, tt, V = synth.batch_graph(g, int(sizes[g]), seed)
        assert V == max(2, int(sizes[g]) // 20) == voff[g + 1] - voff[g]
        a, b = eoff[g], eoff[g + 1]
        assert np.array_equal(s, src[a:b]) and np.array_equal(d, dst[a:b]) and np.array_equal(tt, t[a:b])
        _basic(s, d, tt, V, 30 * DAY)


def test_request_graph_recipe_and_out_arrays():
    n = 100_000
    s, d, t, V = synth.request_graph(3, n, 4)
    assert V == 2 ** math.ceil(math.log2(n / 16))
    _basic(s, d, t, V, 90 * DAY)
    out = (np.empty(n, np.int32), np.empty(n, np.int32), np.empty(n, np.int64))
    s2, d2, t2, V2 = synth.request_graph(3, n, 4, out=out)
    assert V2 == V and s2 is out[0]
    assert np.array_equal(s, s2) and np.array_equal(d, d2) and np.array_equal(t, t2)


def test_seeds():
    a = synth.rmat_hawkes(100_000, 12, 7)
    b = synth.rmat_hawkes(100_000, 12, 7)
    c = synth.rmat_hawkes(100_000, 12, 8)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not np.array_equal(a[0], c[0]) and not np.array_equal(a[2], c[2])
    x = synth.chung_lu_bursts(50_000, 2000, 1)
    y = synth.chung_lu_bursts(50_000, 2000, 1)
    z = synth.chung_lu_bursts(50_000, 2000, 2)
    assert all(np.array_equal(p, q) for p, q in zip(x, y))
    assert not np.array_equal(x[2], z[2])
    assert synth.child_seed(3, 0) != synth.child_seed(3, 1) != synth.child_seed(4, 1)


def test_hypergraph_recipe():
    h = synth.hyper_tiny()
    assert (h.n, h.num_vertices, h.min_cluster_size) == (200_000, 10_000, 5)
    k = np.diff(h.offsets)
    assert h.offsets[0] == 0 and h.offsets[-1] == h.nnz
    assert k.min() >= 2 and k.max() <= 65  # sender + 1..64 recipients
    assert np.median(k - 1) == 2  # recipients: lognormal, median 2
    assert h.members.min() >= 0 and h.members.max() < h.num_vertices
    assert h.t.min() >= 0 and h.t.max() < 30 * DAY


def test_mid_workload_sizes():
    w = synth.plain_mid()
    assert (w.n, w.num_vertices, w.min_cluster_size) == (50_000_000, 1 << 20, 10)
    assert w.t.max() < 90 * DAY and w.t.min() >= 0
