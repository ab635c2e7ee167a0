"""Host logic of the sweep-schedule autotuner: selection and the cache file (CPU, no GPU)."""
import json
import os

import pytest

from paper_2402_10488_amd import autotune as at


class _Problem:
    nx, ny, n_dir, B = 128, 128, 64, 256


def _timer(table, calls):
    def t(cands):
        calls.append(list(cands))
        return [table.get(tuple(c), -1.0) for c in cands]
    return t


def test_select_fastest_valid_and_deterministic():
    assert at.select({(1, 4, 1): 2.0, (4, 4, 1): 0.6, (8, 2, 1): 0.7}) == (4, 4, 1)
    assert at.select({(1, 4, 1): -1.0, (2, 4, 2): 1.5}) == (2, 4, 2)
    assert at.select({(8, 1, 1): 0.5, (2, 2, 4): 0.5}) == (2, 2, 4)    # tie: smaller schedule
    assert at.select({(1, 1, 1): -1.0}) is None
    assert at.select({}) is None


def test_tune_times_once_then_reads_the_cache(tmp_path):
    path = str(tmp_path / "t.json")
    calls = []
    times = {(1, 4, 1): 1.2, (4, 4, 1): 0.59, (8, 2, 1): 0.61, (2, 4, 2): 0.8}
    r1 = at.tune(_Problem(), None, "mixed", path=path, timer=_timer(times, calls), device="dev0")
    assert (r1["dg"], r1["wpb"], r1["bands"], r1["cached"]) == (4, 4, 1, False)
    assert len(calls) == 1 and len(calls[0]) == len(at.CANDIDATES)
    assert r1["candidates"]["4,4,1"] == 0.59 and r1["candidates"]["1,1,1"] == -1.0

    def boom(_):
        raise AssertionError("cached entry must not be re-timed")

    r2 = at.tune(_Problem(), None, "mixed", path=path, timer=boom, device="dev0")
    assert (r2["dg"], r2["wpb"], r2["bands"], r2["cached"], r2["ms"]) == (4, 4, 1, True, 0.59)
    # another precision, another device, or a refresh is timed again
    at.tune(_Problem(), None, "fp64", path=path, timer=_timer(times, calls), device="dev0")
    at.tune(_Problem(), None, "mixed", path=path, timer=_timer(times, calls), device="dev1")
    times[(1, 2, 4)] = 0.3
    r3 = at.tune(_Problem(), None, "mixed", path=path, timer=_timer(times, calls), device="dev0",
                 refresh=True)
    assert (r3["dg"], r3["wpb"], r3["bands"]) == (1, 2, 4) and len(calls) == 4
    data = json.load(open(path))
    assert data["version"] == at.VERSION and len(data["entries"]) == 3


def test_unreadable_or_foreign_cache_is_replaced(tmp_path):
    path = str(tmp_path / "t.json")
    with open(path, "w") as f:
        f.write("{not json")
    calls = []
    r = at.tune(_Problem(), None, "mixed", path=path, timer=_timer({(2, 2, 1): 1.0}, calls),
                device="d")
    assert (r["dg"], r["wpb"]) == (2, 2) and len(calls) == 1
    json.dump({"version": at.VERSION + 1, "entries": {r["key"]: {"dg": 8, "wpb": 4, "bands": 1}}},
              open(path, "w"))
    r = at.tune(_Problem(), None, "mixed", path=path, timer=_timer({(1, 2, 2): 1.0}, calls),
                device="d")
    assert (r["dg"], r["wpb"], r["bands"], r["cached"]) == (1, 2, 2, False)


def test_no_runnable_candidate_raises(tmp_path):
    with pytest.raises(RuntimeError):
        at.tune(_Problem(), None, "mixed", path=str(tmp_path / "t.json"),
                timer=lambda c: [-1.0] * len(c), device="d")


def test_cache_path_from_environment(monkeypatch, tmp_path):
    monkeypatch.setenv(at.CACHE_ENV, str(tmp_path / "x.json"))
    assert at.default_cache_path() == str(tmp_path / "x.json")
    monkeypatch.delenv(at.CACHE_ENV)
    assert at.default_cache_path().endswith(os.path.join("paper_2402_10488_amd",
                                                         "sweep_tuning.json"))
