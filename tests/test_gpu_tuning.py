"""Launch choices never change an output. Four configurations of ce_tuning
(the built-in rules; a CE_TUNE_FILE line; environment variables; a call's
own ce_tuning), each in a fresh child process, cluster the same 2M-record
R-MAT graph (which takes the filter split by default) and a 64-graph batch;
every output is byte-identical across them, and equal to the oracle. The
autotuner's sweep on a small graph keeps only choices whose outputs are
identical to the built-in ones and writes its line to the tuning file."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FIELDS = ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster", "pt_lambda",
          "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected", "labels")
N, SCALE, G = 2_000_000, 17, 64

CHILD = r"""
import json, os, sys
sys.path.insert(0, sys.argv[1])
import numpy as np, torch
import synth, paper_2311_10337_amd as ce
out_dir, knobs = sys.argv[2], json.loads(sys.argv[3])
dev = torch.device("cuda:0")
to = lambda *xs: [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in xs]
s, d, t = synth.rmat_hawkes(%(N)d, %(SCALE)d, seed=61)
src, dst, tt, eoff, voff = synth.batch_workload(%(G)d, seed=62)
print("[child] inputs ready, knobs %%s" %% knobs, flush=True)
with ce.tuned(knobs or None):
    seen = ce.resolve_tuning(len(t), 1 << %(SCALE)d)
    r = ce.to_numpy(ce.cluster_edges(*to(s, d, t), 5, 1 << %(SCALE)d))
    br = ce.cluster_batch(*to(src, dst, tt), eoff, voff, 5)
res = {("g_" + k): v for k, v in r.items() if isinstance(v, np.ndarray)}
res["g_counts"] = np.array([r["m"], r["n_clusters"], r["n_labels"]])
for k in range(len(eoff) - 1):
    for f, v in br.graph(k).items():
        if v is not None:
            res["b%%d_%%s" %% (k, f)] = np.asarray(v)
np.savez(os.path.join(out_dir, "out.npz"), **res)
print(json.dumps({"resolved": seen}), flush=True)
""" % {"N": N, "SCALE": SCALE, "G": G}


def run_child(tmp, name, env_extra, knobs):
    out = tmp / name
    out.mkdir()
    env = {k: v for k, v in os.environ.items()
           if k not in ("CE_TUNE_FILE", "CE_RADIX_IPT", "CE_LIST_GRID", "CE_KRT_LEVEL_BITS", "CE_SPLIT_MIN_EDGES")}
    env.update(env_extra)
    print("[gpu-tuning] child %s" % name, flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(out), json.dumps(knobs)], env=env,
                       capture_output=True, text=True, timeout=400)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    resolved = json.loads(r.stdout.strip().splitlines()[-1])["resolved"]
    with np.load(out / "out.npz") as z:
        return resolved, {k: z[k] for k in z.files}


@pytest.mark.timeout(1500)
def test_outputs_identical_under_four_tunings(tmp_path):
    f = tmp_path / "choices.tune"
    f.write_text("%d %d 0 4 1024 3 -1\n" % (N.bit_length(), (1 << SCALE).bit_length()))
    configs = [
        ("built-in", {}, {}),
        ("file", {"CE_TUNE_FILE": str(f)}, {}),
        ("environment", {"CE_RADIX_IPT": "16", "CE_LIST_GRID": "16384", "CE_KRT_LEVEL_BITS": "7",
                         "CE_SPLIT_MIN_EDGES": "262144"}, {}),
        ("call", {}, {"radix_keys_per_thread": 8, "list_grid": 2048, "krt_level_bits": 5,
                      "split_min_edges": 1 << 22}),
    ]
    runs = [run_child(tmp_path, name, env, knobs) for name, env, knobs in configs]
    seen = [r[0] for r in runs]
    assert seen[0] == {"radix_keys_per_thread": 8, "list_grid": 4096, "krt_level_bits": 0,
                       "split_min_edges": 1 << 20}
    assert seen[1] == {"radix_keys_per_thread": 4, "list_grid": 1024, "krt_level_bits": 3, "split_min_edges": -1}
    assert seen[2] == {"radix_keys_per_thread": 16, "list_grid": 16384, "krt_level_bits": 7,
                       "split_min_edges": 262144}
    assert seen[3] == configs[3][2]
    base = runs[0][1]
    for (name, _, _), (_, got) in zip(configs[1:], runs[1:]):
        assert set(got) == set(base), name
        for k in base:
            assert np.array_equal(got[k], base[k]), (name, k)
    # the built-in run against the oracle
    s, d, t = synth.rmat_hawkes(N, SCALE, seed=61)
    r = oracle.cluster(s, d, t, 5, 1 << SCALE, tier=1)
    assert r.status == 0
    assert list(base["g_counts"]) == [r.m, r.n_clusters, r.n_labels]
    for fld in FIELDS:
        assert np.array_equal(base["g_" + fld], getattr(r, fld)), fld
    src, dst, tt, eoff, voff = synth.batch_workload(G, seed=62)
    for k in range(G):
        e0, e1 = int(eoff[k]), int(eoff[k + 1])
        rg = oracle.cluster(src[e0:e1], dst[e0:e1], tt[e0:e1], 5, int(voff[k + 1] - voff[k]), tier=1)
        for fld in FIELDS:
            assert np.array_equal(base["b%d_%s" % (k, fld)], getattr(rg, fld)), (k, fld)


@pytest.mark.timeout(600)
def test_sweep_keeps_outputs_and_writes_the_file(tmp_path):
    import paper_2311_10337_amd as ce
    from paper_2311_10337_amd import autotune
    dev = torch.device("cuda:0")
    s, d, t = synth.chung_lu_bursts(300_000, 15_000, 71)
    ins = [torch.from_numpy(x).to(dev) for x in (s, d, t)]
    path = str(tmp_path / "swept.tune")
    small = {"krt_level_bits": (3, 6), "split_min_edges": (-1,), "list_grid": (1024,), "radix_keys_per_thread": (4,)}
    outs = ce.Outputs(len(t), 5, dev)
    ws = torch.empty(ce.workspace_bytes(len(t), 15_000, 5), dtype=torch.uint8, device=dev)
    run = lambda: ce.cluster_edges(*ins, 5, 15_000, outputs=outs, workspace=ws)
    res = autotune.sweep(run, autotune.result_digest, reps=2, candidates=small,
                         log=lambda m: print("[gpu-tuning] " + m, flush=True))
    assert len(res["trials"]) == 1 + 2 + 1 + 1 + 1
    assert res["tuned_ms"] <= res["default_ms"] * 1.0001 or res["knobs"] == {}
    bkt = autotune.bucket(len(t), 15_000, 1)
    autotune.write_entry(bkt, res["knobs"], res["default_ms"], res["tuned_ms"], path)
    assert autotune.knobs_for(len(t), 15_000, None, path) == res["knobs"]
    # the chosen knobs, applied by the library from the file, give the oracle's outputs
    os.environ["CE_TUNE_FILE"] = path
    try:
        got = ce.to_numpy(ce.cluster_edges(*ins, 5, 15_000))
    finally:
        del os.environ["CE_TUNE_FILE"]
    r = oracle.cluster(s, d, t, 5, 15_000, tier=1)
    for fld in FIELDS:
        assert np.array_equal(got[fld], getattr(r, fld)), fld
