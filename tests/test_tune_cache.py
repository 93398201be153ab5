"""The tuning cache file of the autotuner (host code of libhbj; no GPU needed).

The library keeps autotuned launch choices in one JSON object {"version": 1, "entries": {key: {"variant":
v, "us": [...]}}}, merged with the file and rewritten atomically after each decision. Checked here: what
is stored can be read back by this and by a fresh process, the file is valid JSON with exactly the stored
entries, entries written by another process are kept, an unreadable file counts as empty, bad keys are
rejected, and the path follows the HBJ_TUNE_CACHE rule.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture
def cache(hbj, tmp_path):
    path = tmp_path / "sub" / "tune.json"
    hbj.set_tune_cache_path(str(path))
    yield hbj, path
    hbj.set_tune_cache_path(None)  # back to the session's file


def test_store_lookup_and_file_contents(cache):
    hbj, path = cache
    assert hbj.tune_cache_size() == 0
    assert hbj.tune_cache_lookup("solve|gfx950|c128|128x128|kl128|ku128|p1|n64|r1|wg") is None
    hbj.tune_cache_store("solve|gfx950|c128|128x128|kl128|ku128|p1|n64|r1|wg", 2, [10.5, 9.25, 8.0, 0.0])
    hbj.tune_cache_store("scatter_mm|gfx950|c64|steps|16x16", 7)
    assert hbj.tune_cache_lookup("solve|gfx950|c128|128x128|kl128|ku128|p1|n64|r1|wg") == 2
    assert hbj.tune_cache_lookup("scatter_mm|gfx950|c64|steps|16x16") == 7
    assert path.exists()  # the directory was created
    doc = json.loads(path.read_text())
    assert doc["version"] == 1
    assert doc["entries"] == {
        "solve|gfx950|c128|128x128|kl128|ku128|p1|n64|r1|wg": {"variant": 2, "us": [10.5, 9.25, 8.0, 0.0]},
        "scatter_mm|gfx950|c64|steps|16x16": {"variant": 7, "us": []},
    }
    # overwrite one entry
    hbj.tune_cache_store("scatter_mm|gfx950|c64|steps|16x16", 3, [1.0])
    assert json.loads(path.read_text())["entries"]["scatter_mm|gfx950|c64|steps|16x16"]["variant"] == 3
    # read back after a reload of the same file
    hbj.set_tune_cache_path(str(path))
    assert hbj.tune_cache_size() == 2
    assert hbj.tune_cache_lookup("scatter_mm|gfx950|c64|steps|16x16") == 3


def test_fresh_process_reads_the_file_and_merges(cache):
    hbj, path = cache
    hbj.tune_cache_store("a|1", 1, [1.0, 2.0])
    code = ("import paper_2209_10886_amd as h; import sys; "
            "assert h.tune_cache_path() == sys.argv[1], h.tune_cache_path(); "
            "assert h.tune_cache_lookup('a|1') == 1; h.tune_cache_store('b|2', 0, [3.0]); print('ok')")
    env = dict(os.environ, HBJ_TUNE_CACHE=str(path))
    r = subprocess.run([sys.executable, "-c", code, str(path)], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    # this process stores again: the other process's entry survives the rewrite
    hbj.tune_cache_store("c|3", 2)
    entries = json.loads(path.read_text())["entries"]
    assert set(entries) == {"a|1", "b|2", "c|3"}
    assert entries["b|2"] == {"variant": 0, "us": [3.0]}


@pytest.mark.parametrize("text", ["", "not json", "{\"version\": 2, \"entries\": {}}",
                                  "{\"version\": 1, \"entries\": {\"k\": {\"us\": [1]}}}",
                                  "{\"version\": 1, \"entries\": {\"bad key\": {\"variant\": 1}}}",
                                  "{\"version\": 1, \"entries\": {\"k\": {\"variant\": 1.5}}}",
                                  "{\"version\": 1, \"entries\": {\"k\": {\"variant\": 1}}} trailing"])
def test_unreadable_file_counts_as_empty(cache, text):
    hbj, path = cache
    path.parent.mkdir(parents=True, exist_ok=True)
    path.write_text(text)
    hbj.set_tune_cache_path(str(path))
    assert hbj.tune_cache_size() == 0
    hbj.tune_cache_store("k", 4)
    assert json.loads(path.read_text())["entries"] == {"k": {"variant": 4, "us": []}}


def test_bad_keys_and_sizes_are_rejected(cache):
    hbj, path = cache
    for key in ("", "has space", "quote\"", "x" * 201, "new\nline"):
        with pytest.raises(hbj.HbjError) as e:
            hbj.tune_cache_store(key, 0)
        assert e.value.code == hbj.EINVAL
    with pytest.raises(hbj.HbjError):
        hbj.tune_cache_store("ok", 0, [0.0] * 65)
    assert hbj.tune_cache_size() == 0


def test_no_file_keeps_decisions_in_memory(hbj, tmp_path):
    hbj.set_tune_cache_path("")
    assert hbj.tune_cache_path() == ""
    hbj.tune_cache_store("mem|1", 5)
    assert hbj.tune_cache_lookup("mem|1") == 5
    assert list(tmp_path.iterdir()) == []
    hbj.set_tune_cache_path(None)


def test_unwritable_file_reports_eio(hbj, tmp_path):
    blocker = tmp_path / "file"
    blocker.write_text("x")
    hbj.set_tune_cache_path(str(blocker / "tune.json"))  # a directory component is a file
    with pytest.raises(hbj.HbjError) as e:
        hbj.tune_cache_store("k|1", 1)
    assert e.value.code == hbj.EIO
    assert hbj.tune_cache_lookup("k|1") == 1  # kept in memory
    hbj.set_tune_cache_path(None)


@pytest.mark.parametrize("env,expect", [("", ""), ("off", ""), ("/tmp/x/y.json", "/tmp/x/y.json"), (None, "HOME")])
def test_path_rule(env, expect, tmp_path):
    e = {k: v for k, v in os.environ.items() if k not in ("HBJ_TUNE_CACHE", "XDG_CACHE_HOME")}
    e["HOME"] = str(tmp_path)
    if env is not None:
        e["HBJ_TUNE_CACHE"] = env
    code = "import paper_2209_10886_amd as h; print(h.tune_cache_path())"
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=e, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    want = os.path.join(str(tmp_path), ".cache", "hbj", "tune.json") if expect == "HOME" else expect
    assert r.stdout.strip() == want
    e["XDG_CACHE_HOME"] = str(tmp_path / "xdg")
    if env is None:
        r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=e, capture_output=True, text=True, timeout=120)
        assert r.stdout.strip() == os.path.join(str(tmp_path), "xdg", "hbj", "tune.json")
