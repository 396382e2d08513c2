"""Served path on the GPU: every request's answers are the same alone and in
the mix (integer outputs, so the tolerance is zero), and equal the oracle's
leftmost LR at the queried positions."""
import dataclasses

import numpy as np
import pytest

import oracle
from gpu_common import say
from paper_1501_06663_amd import serving, workloads

pytestmark = pytest.mark.gpu


def _all_at(o, pos):
    off, rec = o["all_offsets"], o["all_recs"]
    pos = np.asarray(pos, dtype=np.int64)
    outo = np.zeros(len(pos) + 1, dtype=np.int64)
    outo[1:] = np.cumsum(off[pos + 1] - off[pos])
    parts = [rec[off[k]:off[k + 1]] for k in pos]
    return outo, (np.concatenate(parts) if parts else np.zeros((0, 2), np.int32)).reshape(-1, 2)


def _same(a, b):
    if isinstance(a, tuple):
        return all(np.array_equal(x, y) for x, y in zip(a, b))
    return np.array_equal(a, b)


@pytest.mark.parametrize("device_sa", [True, False])
def test_alone_equals_mix(device_sa):
    """Leftmost and all-mode requests: each answer is the same when its
    string is served alone and in the mix, and equals the oracle's."""
    say("case: serving mix of 10 strings (leftmost and all mode), then each alone; device SA",
        device_sa)
    trace = list(workloads.serving_trace(2000.0, 10, seed=11, min_len=1e4, max_len=2e5,
                                         mean_gap=1e-3, max_batches=6, min_q=100, max_q=5000,
                                         all_fraction=0.4))
    assert {r.mode for r in trace} == {"leftmost", "all"}
    ex = serving.GpuExecutor(sa_threads=8, device_sa=device_sa)
    mix = serving.Server(ex, budget_bytes=1 << 30).run(trace)
    assert ex.errors() == 0
    assert len(mix.latencies) == sum(len(r.batches) for r in trace)
    for r in trace:
        alone = serving.Server(ex, budget_bytes=1 << 30).run([dataclasses.replace(
            r, arrival=0.0, batch_times=[0.0] * len(r.batches))])
        o = oracle.pipeline(r.text)
        for qi, pos in enumerate(r.batches):
            a, m = alone.results[(r.rid, qi)], mix.results[(r.rid, qi)]
            assert _same(a, m), (r.rid, qi)
            want = _all_at(o, pos) if r.mode == "all" else o["leftmost"][pos]
            assert _same(m, want), (r.rid, qi, r.mode)
    assert ex.errors() == 0


def test_short_record_buffers_and_many_launches(monkeypatch):
    """Every all-mode launch starts with a record buffer too short for its
    answers (one record per 64 positions), so each one overflows, reads and
    clears its error word and runs again at the exact size; a small query
    reserve splits the batches over many launches with several in flight and
    two build chains.  Answers equal the oracle's."""
    say("case: serving with short all-mode record buffers, 4 launches in flight, 2 build chains")
    monkeypatch.setattr(serving, "ALL_RECORDS_PER_POSITION", 1 / 64)
    trace = list(workloads.serving_trace(3000.0, 8, seed=17, min_len=1e4, max_len=1e5,
                                         mean_gap=5e-4, max_batches=5, min_q=200, max_q=3000,
                                         all_fraction=0.6))
    assert {r.mode for r in trace} == {"leftmost", "all"}
    ex = serving.GpuExecutor(sa_threads=4, build_chains=2)
    rep = serving.Server(ex, budget_bytes=1 << 30, query_reserve_bytes=128 << 10,
                         max_query_launches=4, max_build_chains=2).run(trace)
    assert ex.errors() == 0
    assert rep.query_launches > 4
    for r in trace:
        o = oracle.pipeline(r.text)
        for qi, pos in enumerate(r.batches):
            want = _all_at(o, pos) if r.mode == "all" else o["leftmost"][pos]
            assert _same(rep.results[(r.rid, qi)], want), (r.rid, qi, r.mode)


def test_budget_pressure_on_gpu():
    """Under a budget that fits the two largest strings, the device memory the
    server actually allocates (torch's peak of live allocations, measured
    around the run) stays within the budget, and every answer is right."""
    import torch
    say("case: serving under a budget that fits two strings")
    trace = list(workloads.serving_trace(5000.0, 8, seed=13, min_len=1e4, max_len=1e5,
                                         mean_gap=5e-4, max_batches=3, min_q=100, max_q=2000))
    ex = serving.GpuExecutor(sa_threads=4)
    need = sorted(ex.string_bytes(len(r.text)) for r in trace)
    reserve = 4 << 20
    budget = need[-1] + need[-2] + reserve
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    rep = serving.Server(ex, budget_bytes=budget, query_reserve_bytes=reserve).run(trace)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() - base
    say("  peak allocated %d, server's peak charge %d, budget %d" % (peak, rep.peak_budget, budget))
    assert rep.peak_budget <= budget and not rep.rejected
    assert peak <= budget, (peak, budget)
    for r in trace:
        want = oracle.pipeline(r.text, modes=("leftmost",))["leftmost"]
        for qi, pos in enumerate(r.batches):
            assert np.array_equal(rep.results[(r.rid, qi)], want[pos])
    assert ex.errors() == 0
