"""Scheduler logic of the continuous-batching server, on the CPU.

A mock executor stands in for the GPU: it answers builds and query batches
from the oracle after an injected delay.  It is test-only; the product path
is GpuExecutor.  Checked here: every answer matches the oracle, admission
respects the memory budget (strings wait, are never corrupted, and one that
can never fit is rejected), builds are released only after all of their
strings' queries are answered, and the report's figures are consistent."""
import time
from concurrent.futures import Future

import numpy as np
import pytest

import oracle
from paper_1501_06663_amd import serving, workloads


class MockExecutor:
    """Answers from the oracle after a delay; keeps its own count of the device
    bytes a GpuExecutor would hold (build buffers until the build completes,
    the resident index until release, query buffers until their results are
    taken) and the peak of that count."""

    def __init__(self, delay=0.002):
        self.delay = delay
        self.left = {}          # ref -> oracle leftmost records of that string
        self.released = set()
        self.builds = []
        self.held = 0
        self.peak = 0
        self.open_launches = 0
        self.max_open_launches = 0
        self.open_builds = 0
        self.max_open_builds = 0

    def _hold(self, b):
        self.held += b
        self.peak = max(self.peak, self.held)

    def string_bytes(self, n):
        return serving.device_bytes(n)

    def index_bytes(self, h):
        return serving.index_bytes(h["total"], h["nseg"])

    def query_bytes(self, items):
        return serving.query_bytes([len(p) for _, p, md in items if md != "all"],
                                   len({r for r, _, _ in items}),
                                   [len(p) for _, p, md in items if md == "all"])

    def query_bytes_sums(self, m, ma, nrefs):
        return serving.query_bytes_sums(m, ma, nrefs)

    def submit_sa(self, text):
        f = Future()
        f.set_result(None)      # the mock needs no SA
        return f

    def start_build(self, texts, sas):
        total = sum(len(x) for x in texts)
        h = {"id": len(self.builds), "done": time.perf_counter() + self.delay,
             "refs": [], "total": total, "nseg": len(texts),
             "transient": serving.build_bytes(total, len(texts))}
        self._hold(h["transient"] + serving.index_bytes(total, len(texts)))
        self.open_builds += 1
        self.max_open_builds = max(self.max_open_builds, self.open_builds)
        for b, t in enumerate(texts):
            ref = ("mock", h["id"], b)
            self.left[ref] = oracle.pipeline(t)
            h["refs"].append(ref)
        self.builds.append(h)
        return h

    def build_done(self, h):
        if time.perf_counter() < h["done"]:
            return False
        if "transient" in h:
            self.held -= h.pop("transient")
            self.open_builds -= 1
        return True

    def refs(self, h):
        return list(h["refs"])

    def release_build(self, h):
        self.released.add(h["id"])
        self.held -= serving.index_bytes(h["total"], h["nseg"])

    def start_queries(self, items):
        for ref, _, _ in items:
            assert ref[1] not in self.released, "query on a released build"
        qb = self.query_bytes(items)
        self._hold(qb)
        self.open_launches += 1
        self.max_open_launches = max(self.max_open_launches, self.open_launches)
        return {"done": time.perf_counter() + self.delay, "bytes": qb,
                "res": [all_at(self.left[ref], pos) if md == "all"
                        else self.left[ref]["leftmost"][np.asarray(pos)]
                        for ref, pos, md in items]}

    def queries_done(self, h):
        return time.perf_counter() >= h["done"]

    def query_results(self, h):
        self.held -= h["bytes"]
        self.open_launches -= 1
        return h["res"]


def all_at(o, pos):
    """The oracle's all-mode lists at the given positions, as CSR."""
    off, rec = o["all_offsets"], o["all_recs"]
    pos = np.asarray(pos, dtype=np.int64)
    cnt = off[pos + 1] - off[pos]
    outo = np.zeros(len(pos) + 1, dtype=np.int64)
    outo[1:] = np.cumsum(cnt)
    outr = (np.concatenate([rec[off[k]:off[k + 1]] for k in pos]) if len(pos)
            else np.zeros((0, 2), np.int32))
    return outo, outr.reshape(-1, 2)


def small_trace(count=10, seed=3, rate=400.0, all_fraction=0.0):
    return list(workloads.serving_trace(rate, count, seed=seed, min_len=200, max_len=4000,
                                        mean_gap=5e-4, max_batches=5, min_q=5, max_q=60,
                                        all_fraction=all_fraction))


def check_answers(trace, rep):
    for r in trace:
        o = oracle.pipeline(r.text)
        for qi, pos in enumerate(r.batches):
            got = rep.results[(r.rid, qi)]
            if r.mode == "all":
                want = all_at(o, pos)
                assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), (r.rid, qi)
            else:
                assert np.array_equal(got, o["leftmost"][pos]), (r.rid, qi)


def test_all_answers_match_the_oracle():
    trace = small_trace()
    ex = MockExecutor()
    rep = serving.Server(ex, budget_bytes=1 << 30).run(trace)
    check_answers(trace, rep)
    assert len(rep.latencies) == sum(len(r.batches) for r in trace)
    assert len(rep.ready) == len(trace) and not rep.rejected
    assert rep.positions == sum(len(p) for r in trace for p in r.batches)
    assert ex.released == {h["id"] for h in ex.builds}       # every build freed
    assert all(x >= 0 for x in rep.latencies)
    s = rep.summary()
    assert s["latency_p99_ms"] >= s["latency_p50_ms"] >= 0


RESERVE = 64 << 10   # query reserve of the tight-budget tests (batches of <= 60 positions)


def test_tiny_budget_serialises_admission():
    trace = small_trace(count=8, seed=5)
    largest = max(serving.device_bytes(len(r.text)) for r in trace)
    ex = MockExecutor()
    budget = largest + RESERVE
    rep = serving.Server(ex, budget_bytes=budget, query_reserve_bytes=RESERVE).run(trace)
    check_answers(trace, rep)
    assert rep.peak_budget <= budget           # never over budget; strings waited
    assert ex.peak <= budget                   # nor what the executor holds
    assert ex.held == 0
    assert rep.builds >= 2


@pytest.mark.parametrize("seed", [21, 22])
def test_held_bytes_stay_within_budget(seed):
    """Strings of one build stay resident until the build's last string
    leaves: the build's index is charged until then, so what the executor
    holds never exceeds the budget, whatever the eviction order."""
    trace = small_trace(count=14, seed=seed, rate=3000.0)
    sizes = sorted(serving.device_bytes(len(r.text)) for r in trace)
    budget = sizes[-1] + sizes[-2] + RESERVE
    ex = MockExecutor(delay=0.003)
    rep = serving.Server(ex, budget_bytes=budget, query_reserve_bytes=RESERVE).run(trace)
    check_answers(trace, rep)
    assert not rep.rejected
    assert ex.peak <= rep.peak_budget <= budget, (ex.peak, rep.peak_budget, budget)
    assert ex.held == 0


def test_string_larger_than_budget_is_rejected():
    trace = small_trace(count=6, seed=7)
    sizes = sorted(serving.device_bytes(len(r.text)) for r in trace)
    budget = sizes[-2] + RESERVE               # the largest string can never fit
    big = max(trace, key=lambda r: len(r.text))
    rep = serving.Server(MockExecutor(), budget_bytes=budget, query_reserve_bytes=RESERVE).run(trace)
    assert rep.rejected == [big.rid]
    for r in trace:
        if r.rid != big.rid:
            assert all((r.rid, qi) in rep.results for qi in range(len(r.batches)))


def test_builds_batch_strings_that_arrive_together():
    # all strings arrive at once: one build launch chain serves many strings
    trace = small_trace(count=12, seed=9, rate=1e9)
    ex = MockExecutor(delay=0.01)
    rep = serving.Server(ex, budget_bytes=1 << 30).run(trace)
    check_answers(trace, rep)
    assert rep.builds < len(trace)
    assert rep.query_launches < sum(len(r.batches) for r in trace)


@pytest.mark.parametrize("launches", [1, 3])
def test_query_launches_in_flight(launches):
    """Batches that have all arrived are split over several launches, each
    within its share of the reserve, and at most max_query_launches of them
    are in flight at once; the answers do not depend on the split."""
    trace = small_trace(count=10, seed=12, rate=1e9)
    ex = MockExecutor(delay=0.004)
    reserve = 12 << 10
    budget = sum(serving.device_bytes(len(r.text)) for r in trace) + reserve
    rep = serving.Server(ex, budget_bytes=budget, query_reserve_bytes=reserve,
                         max_query_launches=launches).run(trace)
    check_answers(trace, rep)
    assert ex.max_open_launches <= launches
    if launches > 1:
        assert ex.max_open_launches > 1
    assert ex.peak <= rep.peak_budget <= budget
    assert ex.held == 0
    with pytest.raises(ValueError):
        serving.Server(ex, budget_bytes=budget, max_query_launches=0)


@pytest.mark.parametrize("chains", [1, 2])
def test_build_chains_in_flight(chains):
    """Strings arriving while a build runs start another build chain, up to
    max_build_chains at once; answers and the budget are unaffected."""
    trace = small_trace(count=12, seed=14, rate=2000.0)
    ex = MockExecutor(delay=0.02)
    rep = serving.Server(ex, budget_bytes=1 << 30, max_build_chains=chains).run(trace)
    check_answers(trace, rep)
    assert ex.max_open_builds <= chains
    if chains > 1:
        assert ex.max_open_builds > 1
    assert ex.held == 0
    with pytest.raises(ValueError):
        serving.Server(ex, budget_bytes=1 << 30, max_build_chains=0)


def test_mixed_modes():
    """Leftmost and all-mode requests in one trace: every answer in its own
    mode, and the trace's other draws do not depend on the mode mix."""
    trace = small_trace(count=12, seed=31, rate=2000.0, all_fraction=0.5)
    plain = small_trace(count=12, seed=31, rate=2000.0)
    assert {r.mode for r in trace} == {"leftmost", "all"}
    for a, b in zip(trace, plain):
        assert a.arrival == b.arrival and np.array_equal(a.text, b.text)
    ex = MockExecutor()
    rep = serving.Server(ex, budget_bytes=1 << 30).run(trace)
    check_answers(trace, rep)
    assert rep.positions == sum(len(p) for r in trace for p in r.batches)
