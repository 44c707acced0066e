"""A host model of the parallel exact dendrogram, checked against the oracle's union-find pass (Alg. 1 step 3).

The library builds the single-linkage tree from the key-sorted forest without the serial pass: the rows are
split into aligned intervals over a few global levels, each interval into sub-intervals run one after another,
and one union-find indexed by label serves every interval of a level at once, because the labels (the roots
at an interval's start) of different intervals of one length never meet. A hook records the sub-interval it
was made in, so that the relabelling of sub-interval q sees the roots at the start of q while the unions of q
are going on. Below a few rows per interval a local union-find finishes each interval.

This model runs those steps on the host with small intervals (so that inputs of a few hundred rows go through
several global levels), performs the unions of every sub-interval in a random order, with relabels and unions
of different rows interleaved at random (the order a GPU may run them in), and must give exactly the oracle's
children and sizes for every row. It is a check of the algorithm, not of the kernels: those are compared with
the oracle on the GPU.
"""
import numpy as np
import pytest

import oracle
import synth

NONE = -1


class LabelForest:
    """Union-find over labels; an entry is [parent, stamp (sub-interval of the hook, NONE for a root),
    largest row + 1 of the component (0: none yet), size]."""

    def __init__(self):
        self.e = {}

    def reset(self, label, size):
        self.e[label] = [label, NONE, 0, size]

    def find_before(self, x, q):
        """Root of x at the start of sub-interval q: links made during q are not followed."""
        while True:
            p, stamp = self.e[x][0], self.e[x][1]
            if p == x or stamp >= q:
                return x
            x = p

    def find(self, x):
        while self.e[x][0] != x:
            x = self.e[x][0]
        return x

    def union(self, a, b, q):
        """Hook the larger current root under the smaller during q; returns the hooked root (None: joined)."""
        a, b = self.find(a), self.find(b)
        if a == b:
            return None
        hi, lo = max(a, b), min(a, b)
        self.e[hi][0], self.e[hi][1] = lo, q
        return hi


def model_dendrogram(n, tail, head, local_bits, level_bits, rng, forest=LabelForest):
    """Children (node ids: record < n, or n + row) and sizes of every row, computed the parallel way."""
    m = len(tail)
    lu, lv = [int(x) for x in tail], [int(x) for x in head]
    su, sv = [1] * m, [1] * m
    if m == 0:
        return lu, lv, []
    L = max(1, int(m - 1).bit_length())  # rows are j < 2^L
    hi = L - 1
    while hi >= local_bits:
        lo = max(local_bits, hi - level_bits + 1)
        uf = forest()
        for j in range(m):
            uf.reset(lu[j], su[j])
            uf.reset(lv[j], sv[j])
        span, sub = 1 << (hi + 1), 1 << lo
        for q in range(1 << (hi - lo + 1)):
            rows = [j for a in range(0, m, span) for j in range(a + q * sub, min(a + (q + 1) * sub, m))
                    if j < a + span]
            # each row: relabel to the roots at the start of q, then union; rows interleave at random
            todo = [(j, 0) for j in rng.permutation(rows)]
            roots, hooked = {}, {}
            while todo:
                k = int(rng.integers(len(todo)))
                j, stage = todo[k]
                if stage == 0:
                    a, b = uf.find_before(lu[j], q), uf.find_before(lv[j], q)
                    if q:
                        if uf.e[a][2]:
                            lu[j], su[j] = n + uf.e[a][2] - 1, uf.e[a][3]
                        if uf.e[b][2]:
                            lv[j], sv[j] = n + uf.e[b][2] - 1, uf.e[b][3]
                    roots[j] = (a, b)
                    todo[k] = (j, 1)
                else:
                    hooked[j] = uf.union(*roots[j], q)
                    todo.pop(k)
            # then sizes and largest rows move to the final roots (the hooked roots' entries are no longer
            # changed by anyone, so their sizes are those at the start of q)
            adds = []
            for j in rows:
                h = hooked[j]
                if h is not None:
                    adds.append((uf.find(h), uf.e[h][3], j + 1))
            for f, size, top in adds:
                uf.e[f][3] += size
                uf.e[f][2] = max(uf.e[f][2], top)
        hi = lo - 1
    # the local stage: every interval of 2^local_bits rows alone, in row order
    for a in range(0, m, 1 << local_bits):
        parent, size, top = {}, {}, {}

        def root(x):
            while parent[x] != x:
                x = parent[x]
            return x
        for j in range(a, min(a + (1 << local_bits), m)):
            for lab, s in ((lu[j], su[j]), (lv[j], sv[j])):
                if lab not in parent:
                    parent[lab], size[lab], top[lab] = lab, s, None
            ra, rb = root(lu[j]), root(lv[j])
            assert ra != rb, "a forest row joins one component"
            if top[ra] is not None:
                lu[j], su[j] = n + top[ra], size[ra]
            if top[rb] is not None:
                lv[j], sv[j] = n + top[rb], size[rb]
            parent[rb] = ra
            size[ra] += size[rb]
            top[ra] = j
    return lu, lv, [su[j] + sv[j] for j in range(m)]


def _forest(seed, n, V):
    w = synth.plain_tiny(seed=seed, n=n, V=V)
    res = oracle.cluster(w.src, w.dst, w.t, 2, w.num_vertices, tier=1)
    assert res.status == 0
    return n, res


@pytest.mark.parametrize("seed,n,V,local_bits,level_bits", [
    (1, 300, 40, 2, 1), (2, 500, 30, 2, 2), (3, 700, 200, 3, 2), (4, 400, 8, 1, 3), (5, 1000, 60, 2, 4),
    (6, 64, 5, 0, 1), (7, 257, 20, 2, 3)])
def test_model_equals_the_oracle(seed, n, V, local_bits, level_bits):
    n, res = _forest(seed, n, V)
    m = res.m
    L, R, W, S = oracle.dendrogram(n, res.msf_tail, res.msf_head, res.msf_w)
    rng = np.random.default_rng(seed)
    for trial in range(3):  # three random schedules
        lu, lv, size = model_dendrogram(n, res.msf_tail[:m], res.msf_head[:m], local_bits, level_bits, rng)
        got_l = np.minimum(lu, lv)
        got_r = np.maximum(lu, lv)
        assert np.array_equal(got_l, L) and np.array_equal(got_r, R), (seed, trial)
        assert np.array_equal(np.asarray(size, np.int64), np.asarray(S, np.int64)), (seed, trial)


def test_model_catches_a_missing_stamp():
    """With finds that also follow links made during the current sub-interval (no stamps), the relabelling
    sees roots that are too new: the model must then disagree with the oracle on some input."""
    class Unstamped(LabelForest):
        def find_before(self, x, q):
            return self.find(x)

    bad = 0
    for seed in range(1, 6):
        n, res = _forest(seed, 400, 25)
        m = res.m
        L, R, _, S = oracle.dendrogram(n, res.msf_tail, res.msf_head, res.msf_w)
        rng = np.random.default_rng(seed)
        lu, lv, size = model_dendrogram(n, res.msf_tail[:m], res.msf_head[:m], 2, 2, rng, forest=Unstamped)
        bad += int(not (np.array_equal(np.minimum(lu, lv), L) and np.array_equal(np.asarray(size), S)))
    assert bad > 0
