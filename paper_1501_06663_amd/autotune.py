"""Autotuner for the kernel shapes of liblrq.

The shapes (positions per lane in the LCP kernel, waves per LLR-filter block,
positions per covering-window block; lrq_set_tuning) change speed, never
results.  tune() times a caller-supplied step under each choice by coordinate
descent (one parameter at a time, the others held at the best so far) and
keeps the fastest; the choice is cached in a JSON file keyed by device and by
the workload's size class, so later runs reuse it without timing.

choose_path() does the same one level up, between whole paths that give the
same answers: the compact path (filter, then covering-window scans) and the
raw-LLR path (Section 4.1's first option: every position walks left over the
LLR array), which wins where LLRs are short and launches dominate.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Callable, Dict, Optional

from . import lrq

CACHE = os.environ.get("LRQ_TUNING_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "lrq", "tuning.json"))


def size_key(total: int, nseg: int, device: str = "gfx950") -> str:
    """Size class: total rounded to a power of two, segments to a power of four."""
    t = 1 << max(0, int(math.ceil(math.log2(max(total, 1)))))
    s = 4 ** max(0, int(math.ceil(math.log(max(nseg, 1), 4))))
    return "%s|n%d|s%d" % (device, t, s)


def _load() -> Dict[str, dict]:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(data: Dict[str, dict]) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def _time(step: Callable[[], None], sync: Callable[[], None], reps: int) -> float:
    step()
    sync()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        step()
        sync()
        best = min(best, time.perf_counter() - t0)
    return best


def tune(step: Callable[[], None], key: Optional[str] = None, reps: int = 3,
         use_cache: bool = True, sync: Optional[Callable[[], None]] = None) -> dict:
    """Pick and apply the fastest tuning for `step`; returns {"tuning", "seconds", "trials"}."""
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    cache = _load() if use_cache else {}
    if key is not None and key in cache:
        lrq.set_tuning(**cache[key]["tuning"])
        return dict(cache[key], cached=True)
    best = lrq.get_tuning()
    lrq.set_tuning(**best)
    best_s = _time(step, sync, reps)
    trials = [(dict(best), best_s)]
    for name, choices in lrq.TUNING_CHOICES.items():
        for v in choices:
            if v == best[name]:
                continue
            cand = dict(best, **{name: v})
            lrq.set_tuning(**cand)
            s = _time(step, sync, reps)
            trials.append((cand, s))
            if s < best_s:
                best, best_s = cand, s
    lrq.set_tuning(**best)
    res = {"tuning": best, "seconds": best_s,
           "trials": [{"tuning": c, "seconds": round(t, 6)} for c, t in trials]}
    if key is not None and use_cache:
        cache = _load()
        cache[key] = res
        _store(cache)
    return dict(res, cached=False)


def choose_path(paths: Dict[str, Callable[[], None]], key: Optional[str] = None, reps: int = 3,
                use_cache: bool = True, sync: Optional[Callable[[], None]] = None) -> dict:
    """The fastest of several steps that compute the same answers, each timed
    whole under the current kernel shapes; returns {"path", "seconds",
    "trials"} and caches the choice under key + "|path"."""
    if not paths:
        raise ValueError("no paths to choose from")
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    ckey = None if key is None else key + "|path"
    if ckey is not None and use_cache:
        cache = _load()
        if ckey in cache and cache[ckey].get("path") in paths:
            return dict(cache[ckey], cached=True)
    trials = {name: _time(step, sync, reps) for name, step in paths.items()}
    best = min(trials, key=trials.get)
    res = {"path": best, "seconds": trials[best],
           "trials": {k: round(v, 6) for k, v in trials.items()}}
    if ckey is not None and use_cache:
        cache = _load()
        cache[ckey] = res
        _store(cache)
    return dict(res, cached=False)
