"""The committed profile summaries still describe the committed code (host only).

* Every counter summary's machine-readable block parses and carries the hash of the current kernel sources,
  so bench.py reports its traffic instead of null (a kernel change since the counters were taken fails
  here until they are taken again).
* Every bench.py command a summary gives is accepted by bench.py's own argument parser, so the command
  still runs the committed files.
* The largest kernel of each whole-pipeline kernel-stats summary is the kernel bench.py times for its
  roofline by default.
"""
import glob
import json
import os
import shlex

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def _summaries(pattern):
    paths = sorted(glob.glob(os.path.join(PROFILES, pattern)))
    assert paths, pattern
    return paths


def _json_block(text):
    start = text.find("```json")
    assert start >= 0, "no machine-readable block"
    return json.loads(text[start + 7:text.find("```", start + 7)])


def _bench_args(text):
    """The bench.py arguments of every command line in the summary's code blocks."""
    out = []
    in_code = False
    for line in text.splitlines():
        if line.startswith("```"):
            in_code = not in_code
            continue
        if not in_code or "bench.py" not in line:
            continue
        words = shlex.split(line)
        if "bench.py" in words:
            out.append(words[words.index("bench.py") + 1:])
    return out


@pytest.mark.parametrize("path", _summaries("*_pmc.md"), ids=os.path.basename)
def test_counter_summary_matches_the_kernel_sources(path):
    from paper_2311_10337_amd import profiling
    with open(path) as fh:
        blob = _json_block(fh.read())
    assert blob["source_hash"] == profiling.source_hash()
    if blob.get("scope") == "pipeline":
        traffic = profiling.load_pipeline_traffic(path)
    else:
        traffic = profiling.load_traffic(blob["kernel"], path)
    assert traffic and traffic > 0
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        scale = blob[counter]["scale"]
        assert 0.5 < scale < 4.0, (counter, scale)  # the copy calibration is near 1 or 2, never wild


@pytest.mark.parametrize("path", _summaries("*.md"), ids=os.path.basename)
def test_bench_commands_parse(path):
    import bench
    with open(path) as fh:
        cmds = _bench_args(fh.read())
    assert cmds, "no bench.py command in %s" % path
    for args in cmds:
        bench.make_parser().parse_args(args)


@pytest.mark.parametrize("path", _summaries("pipeline_*_kernel_stats.md"), ids=os.path.basename)
def test_largest_kernel_is_the_roofline_kernel(path):
    import bench
    with open(path) as fh:
        rows = [ln for ln in fh.read().splitlines() if ln.startswith("| ") and not ln.startswith("| kernel")]
    first = rows[0].split("|")[1].strip()
    assert first == bench.make_parser().get_default("roofline_kernel")
