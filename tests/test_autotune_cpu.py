"""The autotuner's choice between whole paths (autotune.choose_path), on the
CPU with stand-in steps: it keeps the fastest, caches the choice per key, and
ignores a cached choice that names a path it was not offered."""
import time

import pytest

from paper_1501_06663_amd import autotune


def test_choose_path_keeps_the_fastest_and_caches_it(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "t.json"))
    calls = {"slow": 0, "fast": 0}

    def slow():
        calls["slow"] += 1
        time.sleep(0.004)

    def fast():
        calls["fast"] += 1
        time.sleep(0.0005)

    paths = {"slow": slow, "fast": fast}
    r = autotune.choose_path(paths, key="k", reps=2, sync=lambda: None)
    assert r["path"] == "fast" and not r["cached"]
    assert set(r["trials"]) == {"slow", "fast"} and r["trials"]["fast"] < r["trials"]["slow"]
    before = dict(calls)
    again = autotune.choose_path(paths, key="k", sync=lambda: None)
    assert again["path"] == "fast" and again["cached"] and calls == before   # nothing timed
    # a cached path that is not among the offered ones is timed afresh
    other = autotune.choose_path({"slow": slow, "other": fast}, key="k", reps=1, sync=lambda: None)
    assert other["path"] == "other" and not other["cached"]
    with pytest.raises(ValueError):
        autotune.choose_path({}, sync=lambda: None)
