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
    def __init__(self, delay=0.002):
        self.delay = delay
        self.left = {}          # ref -> oracle leftmost records of that string
        self.released = set()
        self.builds = []

    def submit_sa(self, text):
        f = Future()
        f.set_result(None)      # the mock needs no SA
        return f

    def start_build(self, texts, sas):
        h = {"id": len(self.builds), "done": time.perf_counter() + self.delay,
             "refs": []}
        for b, t in enumerate(texts):
            ref = ("mock", h["id"], b)
            self.left[ref] = oracle.pipeline(t, modes=("leftmost",))["leftmost"]
            h["refs"].append(ref)
        self.builds.append(h)
        return h

    def build_done(self, h):
        return time.perf_counter() >= h["done"]

    def refs(self, h):
        return list(h["refs"])

    def release_build(self, h):
        self.released.add(h["id"])

    def start_queries(self, items):
        for ref, _ in items:
            assert ref[1] not in self.released, "query on a released build"
        return {"done": time.perf_counter() + self.delay,
                "res": [self.left[ref][np.asarray(pos)] for ref, pos in items]}

    def queries_done(self, h):
        return time.perf_counter() >= h["done"]

    def query_results(self, h):
        return h["res"]


def small_trace(count=10, seed=3, rate=400.0):
    return list(workloads.serving_trace(rate, count, seed=seed, min_len=200, max_len=4000,
                                        mean_gap=5e-4, max_batches=5, min_q=5, max_q=60))


def check_answers(trace, rep):
    for r in trace:
        want = oracle.pipeline(r.text, modes=("leftmost",))["leftmost"]
        for qi, pos in enumerate(r.batches):
            assert np.array_equal(rep.results[(r.rid, qi)], want[pos]), (r.rid, qi)


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


def test_tiny_budget_serialises_admission():
    trace = small_trace(count=8, seed=5)
    largest = max(serving.device_bytes(len(r.text)) for r in trace)
    ex = MockExecutor()
    rep = serving.Server(ex, budget_bytes=largest).run(trace)
    check_answers(trace, rep)
    assert rep.peak_budget <= largest          # never over budget; strings waited
    assert rep.builds >= 2


def test_string_larger_than_budget_is_rejected():
    trace = small_trace(count=6, seed=7)
    sizes = sorted(serving.device_bytes(len(r.text)) for r in trace)
    budget = sizes[-2]                         # the largest string can never fit
    big = max(trace, key=lambda r: len(r.text))
    rep = serving.Server(MockExecutor(), budget_bytes=budget).run(trace)
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
