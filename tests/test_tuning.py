"""Launch choices on the host (no GPU): the order of their sources (a call's
own ce_tuning, then the environment, then the CE_TUNE_FILE entry of the
call's bucket, then the built-in rules) as ce_resolve_tuning reports it, the
limits the library puts on them, and the autotuner's tuning file written,
read back and matched by bucket."""
import os

import pytest

import paper_2311_10337_amd as ce
from paper_2311_10337_amd import autotune

ENV = ("CE_TUNE_FILE", "CE_RADIX_IPT", "CE_LIST_GRID", "CE_KRT_LEVEL_BITS", "CE_SPLIT_MIN_EDGES")
BUILT_IN = {"radix_keys_per_thread": 8, "list_grid": 4096, "krt_level_bits": 0, "split_min_edges": 1 << 20}


@pytest.fixture
def clean_env(monkeypatch):
    for k in ENV:
        monkeypatch.delenv(k, raising=False)
    if not os.path.exists(ce.LIB_PATH):
        pytest.skip("libce.so is not built")
    return monkeypatch


def test_built_in_choices(clean_env):
    assert ce.resolve_tuning(1 << 30, 1 << 26) == BUILT_IN
    assert ce.resolve_tuning(0, 1) == BUILT_IN


def test_sources_in_order(clean_env, tmp_path):
    f = tmp_path / "t.tune"
    n, V = 57_000, 2850
    # n_bits V_bits maxdeg_bits radix list_grid krt split default_ms tuned_ms
    f.write_text("# comment\n%d %d 9 16 2048 3 -1 1.9 1.7\n20 12 4 4 1024 5 262144 0 0\n" %
                 (n.bit_length(), V.bit_length()))
    clean_env.setenv("CE_TUNE_FILE", str(f))
    assert ce.resolve_tuning(n, V) == {"radix_keys_per_thread": 16, "list_grid": 2048, "krt_level_bits": 3,
                                       "split_min_edges": -1}
    assert ce.resolve_tuning(1 << 19, 4000) == {"radix_keys_per_thread": 4, "list_grid": 1024,
                                                "krt_level_bits": 5, "split_min_edges": 262144}
    assert ce.resolve_tuning(1 << 25, 4000) == BUILT_IN  # no line for this bucket
    clean_env.setenv("CE_KRT_LEVEL_BITS", "6")
    clean_env.setenv("CE_LIST_GRID", "8192")
    got = ce.resolve_tuning(n, V)
    assert got["krt_level_bits"] == 6 and got["list_grid"] == 8192 and got["radix_keys_per_thread"] == 16
    got = ce.resolve_tuning(n, V, {"krt_level_bits": 2, "split_min_edges": 1 << 18})
    assert got == {"radix_keys_per_thread": 16, "list_grid": 8192, "krt_level_bits": 2, "split_min_edges": 1 << 18}
    # the file is read again when it changes
    f.write_text("%d %d 9 4 0 0 0\n" % (n.bit_length(), V.bit_length()))
    os.utime(f, (1, 1))
    clean_env.delenv("CE_KRT_LEVEL_BITS")
    clean_env.delenv("CE_LIST_GRID")
    assert ce.resolve_tuning(n, V) == dict(BUILT_IN, radix_keys_per_thread=4)


def test_limits(clean_env):
    got = ce.resolve_tuning(100, 10, {"radix_keys_per_thread": 5, "list_grid": 7, "krt_level_bits": 99})
    assert got == {"radix_keys_per_thread": 8, "list_grid": 256, "krt_level_bits": 12, "split_min_edges": 1 << 20}
    clean_env.setenv("CE_SPLIT_MIN_EDGES", "0")  # 0 turns the split off
    assert ce.resolve_tuning(100, 10)["split_min_edges"] == -1
    assert ce.resolve_tuning(100, 10, {"list_grid": 1 << 20})["list_grid"] == 65536


def test_unknown_knob_is_refused():
    with pytest.raises(ValueError):
        ce.set_tuning({"tile": 3})


def test_tuning_file_round_trip(tmp_path):
    path = str(tmp_path / "x.tune")
    autotune.write_entry((16, 12, 9), {"krt_level_bits": 3, "list_grid": 1024}, 1.876, 1.77, path)
    autotune.write_entry((26, 20, 19), {}, 95.0, 95.0, path)
    autotune.write_entry((16, 12, 11), {"radix_keys_per_thread": 16}, 2.0, 1.9, path)
    autotune.write_entry((16, 12, 9), {"krt_level_bits": 4}, 1.8, 1.7, path)  # replaces the first line
    e = autotune.read_entries(path)
    assert e[(16, 12, 9)]["knobs"] == {"krt_level_bits": 4}
    assert e[(26, 20, 19)]["knobs"] == {}
    assert autotune.knobs_for(57_000, 2850, 300, path) == {"krt_level_bits": 4}
    assert autotune.knobs_for(57_000, 2850, 2000, path) == {"radix_keys_per_thread": 16}
    assert autotune.knobs_for(57_000, 2850, None, path) == {"krt_level_bits": 4}
    assert autotune.knobs_for(1 << 30, 2850, None, path) is None
    lines = open(path).read().splitlines()
    assert lines[0].startswith("#") and len(lines) == 4


def test_library_reads_the_autotuners_file(clean_env, tmp_path):
    path = str(tmp_path / "y.tune")
    autotune.write_entry(autotune.bucket(200_000, 10_000, 900), {"krt_level_bits": 5, "list_grid": 2048,
                                                                 "split_min_edges": -1}, 3.0, 2.5, path)
    clean_env.setenv("CE_TUNE_FILE", path)
    assert ce.resolve_tuning(200_000, 10_000) == {"radix_keys_per_thread": 8, "list_grid": 2048,
                                                  "krt_level_bits": 5, "split_min_edges": -1}


def test_digest_tells_outputs_apart():
    torch = pytest.importorskip("torch")
    x = torch.arange(1000, dtype=torch.int32)
    y = x.clone()
    y[[10, 11]] = y[[11, 10]]  # two elements swapped
    assert autotune.device_digest([x]) == autotune.device_digest([x.clone()])
    assert autotune.device_digest([x]) != autotune.device_digest([y])
    assert autotune.device_digest([x[:999]]) != autotune.device_digest([x])
