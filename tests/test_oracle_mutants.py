"""Planted mistakes in the oracle (on the CPU): each mutated copy of the oracle's
C source must fail at least one pin in test_oracle_pins.py,
test_oracle_causal.py, test_oracle_discrete.py, test_oracle_hyper.py or
test_oracle_levels.py. This shows the pins
would catch a dropped term, a wrong sign or index, or a transposed operand."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ce_oracle.c")

MUTANTS = [
    ("key tie on tail reversed", "a->tail > b->tail ? -1 : 1", "a->tail < b->tail ? -1 : 1"),
    ("record order ties by descending id", "  return a < b;\n}", "  return a > b;\n}"),
    ("weight sign flipped", "e.w = g_t[e.head] - g_t[e.tail];", "e.w = g_t[e.tail] - g_t[e.head];"),
    ("skeleton drops first pair", "for (int64_t k = off[x] + 1; k < off[x + 1]; k++)",
     "for (int64_t k = off[x] + 2; k < off[x + 1]; k++)"),
    ("dendrogram children transposed", "left[k] = na < nb ? na : nb;", "left[k] = na < nb ? nb : na;"),
    ("dendrogram size off by one", "size[k] = sz[a] + sz[b];", "size[k] = sz[a] + sz[b] - 1;"),
    ("lambda drops the factor 2", "/ (2 * (uint64_t)w);", "/ ((uint64_t)w);"),
    ("stability drops child-cluster term", "stab[P] += (u128)nsize[x] *", "stab[P] += (u128)0 *"),
    ("EOM ties go to children", "else if (childsum[r] > S)", "else if (childsum[r] >= S)"),
    ("big child test strict", "int b1 = nsize[c1] >= (uint64_t)M", "int b1 = nsize[c1] > (uint64_t)M"),
    ("root rule: one big component becomes a cluster", "if (nbig >= 2) {", "if (nbig >= 1) {"),
    ("labels numbered by maximum member", "if (got >= 0 && p < minmem[got]) minmem[got] = p;",
     "if (got >= 0 && (minmem[got] == INT64_MAX || p > minmem[got])) minmem[got] = p;"),
    ("causal: out-edges first at equal times", "if (ia != ib) return ia ? -1 : 1;",
     "if (ia != ib) return ia ? 1 : -1;"),
    ("causal: every earlier arrival joins each departure", "carried = latest; since = k + 1;",
     "carried = -1;"),
    ("causal: nothing carried past a departure", "if (carried >= 0) put_arc(", "if (0) put_arc("),
    ("causal: strict temporal causality", "if (src[q] != x || t[r] > t[q]) continue;",
     "if (src[q] != x || t[r] >= t[q]) continue;"),
    ("causal: head-to-head pairs", "if (src[q] != x || t[r] > t[q]) continue;",
     "if (dst[q] != x || q == r || t[r] > t[q]) continue;"),
    ("causal: arc weight reversed", "out[*cnt].w = t[e] - t[a];", "out[*cnt].w = t[a] - t[e];"),
    ("time filter strict", "if (edges[e].w <= max_dt) edges[k++] = edges[e];",
     "if (edges[e].w < max_dt) edges[k++] = edges[e];"),
    ("discrete levels with strict thresholds", "while (L < q && lw[k] > thr[L]) L++;",
     "while (L < q && lw[k] >= thr[L]) L++;"),
    ("discrete birth with one big child", "if (nb >= 2) { is_cluster[c] = 1;", "if (nb >= 1) { is_cluster[c] = 1;"),
    ("discrete blocks ignore levels", "dd_top[k] = (p != NONE32 && dd_level[p] == dd_level[k]) ? dd_top[p]",
     "dd_top[k] = (p != NONE32) ? dd_top[p]"),
    ("hyper: meeting tested on the first member only", "for (int64_t k = off[b]; k < off[b + 1] && !meet; k++)",
     "for (int64_t k = off[b]; k < off[b] + 1 && k < off[b + 1] && !meet; k++)"),
    ("hyper: incident lists left unsorted",
     'qsort(lst + voff[x], (size_t)d, sizeof(uint32_t), cmp_rec); /* incident hyperedges in time order */',
     "/* unsorted */"),
    ("hyper: star instead of path", "out[cnt] = make_edge(prev, cur);", "out[cnt] = make_edge(lst[voff[x]], cur);"),
    ("level components keep edges strictly below", "if (w[e] > thr[l]) continue;", "if (w[e] >= thr[l]) continue;"),
    ("level components labelled by largest member", "if ((uint32_t)r < low[root]) low[root] = (uint32_t)r;",
     "if (low[root] == UINT32_MAX || (uint32_t)r > low[root]) low[root] = (uint32_t)r;"),
]


PIN_FILES = ["test_oracle_pins.py", "test_oracle_causal.py", "test_oracle_discrete.py", "test_oracle_hyper.py",
             "test_oracle_levels.py"]
# the pin file that covers a mutant's function runs first (pytest -x stops at the first failing pin); every
# file still runs when it passes
FIRST = {"causal": "test_oracle_causal.py", "discrete": "test_oracle_discrete.py", "hyper": "test_oracle_hyper.py",
         "level": "test_oracle_levels.py", "time filter": "test_oracle_pins.py"}


def pin_order(name):
    first = next((f for k, f in FIRST.items() if name.startswith(k)), PIN_FILES[0])
    return [first] + [f for f in PIN_FILES if f != first]


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new, tmp_path):
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation anchor not unique: %s" % name
    mut = tmp_path / "ce_oracle_mut.c"
    mut.write_text(text.replace(old, new))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", "-o", str(lib), str(mut)])
    env = dict(os.environ, CE_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"]
                       + [os.path.join(ROOT, "tests", f) for f in pin_order(name)] + ["-k", "not four_records"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "planted mistake '%s' passed every pin:\n%s" % (name, r.stdout[-2000:])
