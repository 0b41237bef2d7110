"""Host logic of the autotuner's cache (no GPU): keys, size signatures,
lookups of the committed cache for every workload bench.py runs, and the
save/load round trip."""
import json

import numpy as np
import pytest

from paper_1810_11518_amd import autotune, synth


@pytest.fixture(autouse=True)
def _gfx950(monkeypatch):
    # the architecture comes from the device; these checks run without one
    monkeypatch.setattr(autotune, "arch", lambda: "gfx950")


def test_size_signature():
    assert autotune.size_signature([490] * 3, [640] * 3) == "490x640"
    # pixel-count quantiles rounded to powers of two
    Hs, Ws = [100] * 10 + [1000] * 10, [100] * 10 + [1000] * 10
    sig = autotune.size_signature(Hs, Ws)
    lo, mid, hi = (int(x) for x in sig[len("mix:"):].split("/"))
    assert sig.startswith("mix:") and lo == 8192 and hi == 1048576 and lo <= mid <= hi
    for v in (lo, mid, hi):
        assert v & (v - 1) == 0


def test_key_parts():
    Hs, Ws = [490] * 2, [640] * 2
    assert autotune.key(Hs, Ws, 3, (7, 6)) == "gfx950|k3|7x6|490x640"
    assert autotune.key(Hs, Ws, 3, (20, 20), windows=True) == "gfx950|k3|20x20|490x640|win"
    assert autotune.key(Hs, Ws, 2, (7, 6), flags=4) == "gfx950|k2|7x6|490x640|f4"


@pytest.mark.parametrize("name,k,windows", [
    ("batch", 3, None), ("uneven", 3, None), ("large", 2, None), ("large", 3, None),
    ("large", 4, None), ("batch", 3, 10), ("batch", 3, 20), ("batch", 3, 25), ("batch", 3, 50),
    ("batch", 3, 100)])
def test_committed_cache_covers_the_bench_workloads(name, k, windows):
    """bench.py takes its launch shapes from the committed cache: every
    workload it times has an entry (else it would run an untuned default)."""
    Hs, Ws = synth.workload_sizes(name)
    cells = synth.WORKLOADS[name]["cells"] if windows is None else (windows, windows)
    tune = autotune.lookup(Hs, Ws, k, cells, windows=windows is not None)
    assert tune, (name, k, windows)
    assert tune["block_threads"] % 64 == 0 and 64 <= tune["block_threads"] <= 1024
    for c in tune["classes"]:
        assert c["cell_rows_per_item"] >= 1 and c["rows_per_task"] >= 1


def test_headline_tune_is_the_measured_one():
    Hs, Ws = synth.workload_sizes("batch")
    assert autotune.lookup(Hs, Ws, 3, (7, 6)) == {
        "block_threads": 256, "classes": [{"cell_rows_per_item": 2, "rows_per_task": 8}]}


def test_save_and_load_round_trip(tmp_path):
    path = str(tmp_path / "tuned.json")
    assert autotune.lookup([64], [64], 3, (7, 6), path=path) is None
    t1 = {"block_threads": 320, "classes": [{"cell_rows_per_item": 7, "rows_per_task": 8}]}
    t2 = {"block_threads": 128, "classes": [{"cell_rows_per_item": 2, "rows_per_task": 4}]}
    autotune.save([64], [64], 3, (7, 6), t1, 1.23456, path=path, note="a")
    autotune.save([64], [64], 3, (10, 10), t2, 2.0, path=path, windows=True)
    assert autotune.lookup([64], [64], 3, (7, 6), path=path) == t1
    assert autotune.lookup([64], [64], 3, (10, 10), path=path, windows=True) == t2
    # a window key and a cell-grid key of the same size stay apart
    assert autotune.lookup([64], [64], 3, (10, 10), path=path) is None
    with open(path) as f:
        cache = json.load(f)
    assert cache["gfx950|k3|7x6|64x64"] == {"tune": t1, "ms": 1.2346, "note": "a"}
    assert not list(tmp_path.glob("*.tmp*"))  # written through a replaced temporary


def test_default_classes():
    assert autotune.default_classes([490] * 4, [640] * 4, 7) == [
        {"cell_rows_per_item": 1, "rows_per_task": 8}]
    Hs = np.array([50, 100, 200, 400, 800, 1000])
    cls = autotune.default_classes(Hs, Hs, 7)
    assert len(cls) == 3 and "max_pixels" not in cls[-1]
    assert cls[0]["max_pixels"] < cls[1]["max_pixels"]
