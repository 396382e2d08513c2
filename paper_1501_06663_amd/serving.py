"""Continuous-batching server for longest-repeat point queries.

Strings arrive over time, each followed by batches of positions to query
(Section 2's problem, asked position by position).  The server:

* admits arrived strings in arrival order while their device memory fits the
  HBM budget (a string that can never fit is rejected);
* builds suffix arrays on the device with the rest of the index (or on host
  threads, as the paper does, Section 5 opening), indexing every admitted
  string whose SA is ready in ONE batched launch chain (SA, rank scatter, LCP,
  LLR filter, all with segment offsets) on a build stream, with up to
  max_build_chains such chains in flight on streams of their own;
* keeps each string's compact index resident and answers every pending query
  batch, across all resident strings, with multi-string point-query launches
  (one per share of the query reserve, several in flight) on a query stream, so
  builds and queries of different strings overlap on the device;
* frees a build's memory when all of its strings have answered all of their
  query batches, which lets waiting strings in.

Latency of a query batch = completion time - its arrival time; time-to-ready
of a string = index ready - string arrival.  The device work goes through an
executor (GpuExecutor below; tests substitute a CPU mock), so the scheduling
logic is testable without a GPU.
"""
from __future__ import annotations

import time
from collections import deque
from concurrent.futures import Future, ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .workloads import Request

def _alloc(nbytes: int) -> int:
    """Device bytes torch's caching allocator takes for one tensor of nbytes
    (it rounds every allocation up to a multiple of 512 bytes)."""
    return (int(nbytes) + 511) // 512 * 512


def index_bytes(total: int, nseg: int = 1) -> int:
    """Device bytes a build keeps resident: the compact array (capacity one
    entry per position), its count and the block table."""
    from . import lrq
    return _alloc(8 * max(total, 1)) + _alloc(8) + _alloc(8 * lrq.block_entries(total))


def build_bytes(total: int, nseg: int = 1, device_sa: bool = True) -> int:
    """Device bytes a build holds only while it runs: text (+8 bytes of
    padding), segment offsets, SA, neighbour/LCP pairs, scratch and, with
    device suffix arrays, the SA construction's work buffer (all sized by the
    library's own sizing calls)."""
    from . import lrq
    t = max(total, 1)
    b = (_alloc(total + 8) + _alloc(8 * (nseg + 1)) + _alloc(4 * (total + 1)) + _alloc(8 * t)
         + _alloc(lrq.scratch_bytes(total, nseg)))
    if device_sa:
        b += _alloc(lrq.sa_work_bytes(total, nseg))
    return b


def device_bytes(n: int, device_sa: bool = True) -> int:
    """Budget charge of one string from admission until its build completes:
    the build's transient buffers and its resident index, as if it were built
    alone.  A batch of strings never needs more than the sum of their charges
    (every size above is linear in the length plus per-build constants)."""
    return index_bytes(n, 1) + build_bytes(n, 1, device_sa)


# First record buffer of an all-mode launch, per position.  A launch whose
# answers do not fit runs again with a buffer of the exact size; that larger
# buffer is not charged to the query reserve (the measured workloads have
# about two records per position, so it does not happen there).
ALL_RECORDS_PER_POSITION = 4


def query_bytes(npos: Sequence[int], nrefs: int, npos_all: Sequence[int] = ()) -> int:
    """Device bytes of one round of query launches: batches of npos positions
    in leftmost mode and of npos_all positions in all mode, on nrefs strings
    (string references, ids and positions of both launches, one record per
    leftmost position, and for all mode the CSR offsets, a first record buffer
    and the scratch that scans the counts)."""
    return query_bytes_sums(int(sum(npos)), int(sum(npos_all)), nrefs)


def query_bytes_sums(m: int, ma: int, nrefs: int) -> int:
    """query_bytes from the totals: m leftmost and ma all-mode positions on
    nrefs strings."""
    from . import lrq
    b = _alloc(8 * lrq.REF_WORDS * max(nrefs, 1))
    for q in (m, ma):
        if q:
            b += 2 * _alloc(4 * q)
    if m:
        b += _alloc(8 * m)
    if ma:
        b += (_alloc(8 * (ma + 1)) + _alloc(8 * ALL_RECORDS_PER_POSITION * ma)
              + _alloc(lrq.scratch_bytes(ma)) + _alloc(8))
    return b


# ------------------------------------------------------------------ executor --

class GpuExecutor:
    """Runs builds and query batches through liblrq: build_chains build
    streams and one query stream."""

    def __init__(self, device="cuda:0", sa_threads: int = 16, device_sa: bool = True,
                 build_chains: int = 2):
        import torch
        from . import lrq
        self.torch, self.lrq = torch, lrq
        self.dev = torch.device(device)
        self.build_streams = [torch.cuda.Stream(self.dev) for _ in range(max(1, build_chains))]
        self.stream_builds = [0] * len(self.build_streams)  # builds not yet done, per stream
        self.query_stream = torch.cuda.Stream(self.dev)
        # copies back of all-mode results and reads of a launch's error word,
        # issued once that launch has completed
        self.read_stream = torch.cuda.Stream(self.dev)
        self.device_sa = bool(device_sa)
        self.pool = ThreadPoolExecutor(max(1, sa_threads))
        # each build chain runs on a worker thread of its own: lrq_build_sa
        # waits for its stream between doubling rounds, and the scheduling
        # loop must keep dispatching queries (and other builds) meanwhile
        self.builder = ThreadPoolExecutor(len(self.build_streams))
        self.qscratch = torch.zeros(lrq.scratch_bytes(0), dtype=torch.uint8, device=self.dev)

    # device-memory sizes for the server's budget
    def string_bytes(self, n: int) -> int:
        return device_bytes(n, self.device_sa)

    def index_bytes(self, h) -> int:
        return index_bytes(h["total"], len(h["off"]) - 1)

    def query_bytes(self, items) -> int:
        return query_bytes([len(p) for _, p, md in items if md != "all"],
                           len({ref for ref, _, _ in items}),
                           [len(p) for _, p, md in items if md == "all"])

    def query_bytes_sums(self, m: int, ma: int, nrefs: int) -> int:
        return query_bytes_sums(m, ma, nrefs)

    # suffix arrays: on host threads (ctypes releases the GIL, so these run in
    # parallel), or nothing to do here when the build computes them
    def submit_sa(self, text: np.ndarray):
        if self.device_sa:
            f = Future()
            f.set_result(None)
            return f
        return self.pool.submit(self.lrq.build_sa_host, text)

    def start_build(self, texts: Sequence[np.ndarray], sas: Sequence[np.ndarray]):
        # the stream with the fewest unfinished builds (a free one if any)
        k = min(range(len(self.build_streams)), key=lambda i: self.stream_builds[i])
        self.stream_builds[k] += 1
        h = {"stream_index": k}
        h["future"] = self.builder.submit(self._build, h, list(texts),
                                          None if self.device_sa else list(sas),
                                          self.build_streams[k])
        return h

    def _build(self, h, texts, sas, stream):
        torch, lrq = self.torch, self.lrq
        lens = np.array([len(t) for t in texts], dtype=np.int64)
        off = np.zeros(len(texts) + 1, dtype=np.int64)
        off[1:] = np.cumsum(lens)
        total = int(off[-1])
        text = np.concatenate(texts) if texts else np.zeros(0, np.uint8)
        h.update({"off": off, "total": total})
        with torch.cuda.stream(stream):
            t = max(total, 1)
            # 8 bytes of padding keep the text's tail readable as whole words
            h["text"] = torch.from_numpy(np.concatenate([text, np.zeros(8, np.uint8)])).to(self.dev, non_blocking=False)
            h["seg"] = torch.from_numpy(off).to(self.dev)
            if sas is None:
                h["sa"] = torch.empty(t, dtype=torch.int32, device=self.dev)
                work = torch.empty(lrq.sa_work_bytes(total, len(texts)), dtype=torch.uint8,
                                   device=self.dev)
                lrq.build_sa(h["text"], total, h["seg"], len(texts), h["sa"], work,
                             stream)
                del work
            else:
                sa = np.concatenate(sas) if sas else np.zeros(0, np.int32)
                h["sa"] = torch.from_numpy(np.concatenate([sa, np.zeros(1, np.int32)])).to(self.dev, non_blocking=False)
            h["work"] = torch.empty(2 * t, dtype=torch.int32, device=self.dev)
            h["llrc"] = torch.empty((t, 2), dtype=torch.int32, device=self.dev)
            h["count"] = torch.zeros(1, dtype=torch.int64, device=self.dev)
            h["blocks"] = torch.zeros(lrq.block_entries(total), dtype=torch.int64, device=self.dev)
            h["scratch"] = torch.zeros(lrq.scratch_bytes(total, len(texts)), dtype=torch.uint8,
                                       device=self.dev)
            lrq.index_build(h["text"], h["sa"], total, h["seg"], len(texts), h["work"], h["llrc"],
                            h["count"], h["blocks"], None, h["scratch"], stream)
            h["event"] = torch.cuda.Event()
            h["event"].record(stream)
        return h

    def build_done(self, h) -> bool:
        if not h["future"].done():
            return False
        h["future"].result()  # re-raises a failed build
        if not h["event"].query():
            return False
        if not h.get("counted_done"):
            self.stream_builds[h["stream_index"]] -= 1
            h["counted_done"] = True
        # transient buffers are no longer needed once the build has completed
        for k in ("text", "sa", "work", "scratch"):
            h.pop(k, None)
        return True

    def refs(self, h) -> List[Tuple[int, int, int, int, int]]:
        llrc, blocks = h["llrc"].data_ptr(), h["blocks"].data_ptr()
        off = h["off"]
        return [(llrc, blocks, h["total"], int(off[b]), int(off[b + 1] - off[b]))
                for b in range(len(off) - 1)]

    def release_build(self, h):
        h.clear()

    def start_queries(self, items: Sequence[Tuple[tuple, np.ndarray, str]]):
        """items: (ref, positions, mode) per query batch.  One launch answers
        every leftmost batch and one launch chain every all-mode batch."""
        torch, lrq = self.torch, self.lrq
        uniq: Dict[tuple, int] = {}
        groups = {"leftmost": ([], [], []), "all": ([], [], [])}
        order = []
        for ref, pos, mode in items:
            s = uniq.setdefault(ref, len(uniq))
            sids, poss, sizes = groups["all" if mode == "all" else "leftmost"]
            order.append(("all" if mode == "all" else "leftmost", len(sizes)))
            sids.append(s)
            poss.append(pos)
            sizes.append(len(pos))
        refs = np.array(list(uniq.keys()), dtype=np.int64).reshape(-1, lrq.REF_WORDS)
        h = {"order": order, "sizes": {g: v[2] for g, v in groups.items()}}
        # inputs and results go through pinned host buffers with asynchronous
        # copies on the query stream, so the scheduling loop never waits for a
        # transfer; the launch's event covers the copies back
        h["refs_host"] = self._pinned(refs)
        with torch.cuda.stream(self.query_stream):
            h["refs"] = h["refs_host"].to(self.dev, non_blocking=True)
            for g, (sids, poss, sizes) in groups.items():
                m = int(sum(sizes))
                if not m:
                    continue
                # positions copied straight into the pinned buffer; the
                # per-position string ids are expanded on the device from one
                # (string, count) pair per batch
                hp = torch.empty(m, dtype=torch.int32, pin_memory=True)
                hv = hp.numpy()
                at = 0
                for pos_b, n_b in zip(poss, sizes):
                    hv[at:at + n_b] = pos_b
                    at += n_b
                hb = torch.from_numpy(np.array([sids, sizes], dtype=np.int64)).pin_memory()
                h[g + "_host"] = (hp, hb)
                pos = hp.to(self.dev, non_blocking=True)
                per = hb.to(self.dev, non_blocking=True)
                sid = torch.repeat_interleave(per[0].to(torch.int32), per[1], output_size=m)
                h[g + "_in"] = (sid, pos, m)
                if g == "leftmost":
                    h["out"] = torch.empty((m, 2), dtype=torch.int32, device=self.dev)
                    lrq.query_multi(h["refs"], len(uniq), sid, pos, m, h["out"], self.qscratch,
                                    self.query_stream)
                    h["out_host"] = torch.empty((m, 2), dtype=torch.int32, pin_memory=True)
                    h["out_host"].copy_(h["out"], non_blocking=True)
                else:
                    h["ascratch"] = torch.zeros(lrq.scratch_bytes(m), dtype=torch.uint8,
                                                device=self.dev)
                    h["offsets"] = torch.empty(m + 1, dtype=torch.int64, device=self.dev)
                    self._launch_all(h, len(uniq), int(ALL_RECORDS_PER_POSITION * m))
            h["event"] = torch.cuda.Event()
            h["event"].record(self.query_stream)
        return h

    @staticmethod
    def _pinned(a: np.ndarray):
        import torch
        t = torch.empty(a.shape, dtype=torch.int64, pin_memory=True)
        t.numpy()[...] = a
        return t

    def _launch_all(self, h, nrefs, cap):
        """All-mode launch chain into a record buffer of `cap` records; the
        record total comes back through a pinned host word, so nothing here
        waits for the device."""
        torch, lrq = self.torch, self.lrq
        sid, pos, m = h["all_in"]
        h["cap"] = cap
        h["recs"] = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=self.dev)
        lrq.query_multi(h["refs"], nrefs, sid, pos, m, None, h["ascratch"], self.query_stream,
                        mode=lrq.ALL, offsets=h["offsets"], recs=h["recs"], capacity=cap,
                        want_total=False)
        h["total"] = torch.empty(1, dtype=torch.int64, pin_memory=True)
        h["total"].copy_(h["offsets"][m:], non_blocking=True)

    def queries_done(self, h) -> bool:
        if not h["event"].query():
            return False
        if "all_in" not in h or "offsets_host" in h:
            return True
        torch = self.torch
        total = int(h["total"][0])
        # the launch's buffers are used on the read-back stream too: the
        # allocator must not hand them out again before that stream is done
        for k in ("ascratch", "offsets", "recs"):
            h[k].record_stream(self.read_stream)
        if total > h["cap"]:
            # the first record buffer was short (rare): read (which clears)
            # the overflow bit it flagged and run the all-mode chain again at
            # the exact size, after the clearing
            errs = self.lrq.read_errors(h["ascratch"], self.read_stream)
            if errs & ~self.lrq.ERR_CAPACITY:
                raise RuntimeError("all-mode point queries: device error bits %d" % errs)
            self.query_stream.wait_stream(self.read_stream)
            with torch.cuda.stream(self.query_stream):
                self._launch_all(h, int(h["refs"].shape[0]), total)
                h["event"] = torch.cuda.Event()
                h["event"].record(self.query_stream)
            return False
        # the chain is complete: bring back exactly the offsets and records it
        # wrote, on the read-back stream (the query stream may already hold
        # later launches), and finish when those copies have
        m = h["all_in"][2]
        h["offsets_host"] = torch.empty(m + 1, dtype=torch.int64, pin_memory=True)
        h["recs_host"] = torch.empty((max(total, 1), 2), dtype=torch.int32, pin_memory=True)
        with torch.cuda.stream(self.read_stream):
            h["offsets_host"].copy_(h["offsets"], non_blocking=True)
            if total:
                h["recs_host"][:total].copy_(h["recs"][:total], non_blocking=True)
            h["event"] = torch.cuda.Event()
            h["event"].record(self.read_stream)
        return False

    def query_results(self, h) -> List:
        """Per batch, in the order given: leftmost records (m, 2), or for an
        all-mode batch (offsets[m+1] from 0, records)."""
        res = {}
        if "out" in h:
            out, at, parts = h["out_host"].numpy(), 0, []
            for s in h["sizes"]["leftmost"]:
                parts.append(out[at:at + s])
                at += s
            res["leftmost"] = parts
        if "all_in" in h:
            errs = self.lrq.read_errors(h["ascratch"], self.read_stream)
            if errs:
                raise RuntimeError("all-mode point queries: device error bits %d" % errs)
            off = h["offsets_host"].numpy()
            recs = h["recs_host"].numpy()
            at, parts = 0, []
            for s in h["sizes"]["all"]:
                o = off[at:at + s + 1]
                parts.append((o - o[0], recs[o[0]:o[-1]]))
                at += s
            res["all"] = parts
        return [res[g][i] for g, i in h["order"]]

    def errors(self) -> int:
        return self.lrq.read_errors(self.qscratch, self.query_stream)


# -------------------------------------------------------------------- server --

@dataclass(eq=False)
class _String:
    req: Request
    need: int
    sa_future: object = None
    sa: Optional[np.ndarray] = None
    build: Optional[dict] = None
    ref: Optional[tuple] = None
    ready_at: Optional[float] = None
    next_batch: int = 0          # first query batch not yet dispatched
    open_batches: int = 0        # dispatched, not completed
    done_batches: int = 0


@dataclass
class ServeReport:
    latencies: List[float] = field(default_factory=list)        # per query batch, s
    ready: List[float] = field(default_factory=list)            # per string, s
    results: Dict[Tuple[int, int], np.ndarray] = field(default_factory=dict)
    rejected: List[int] = field(default_factory=list)
    positions: int = 0
    chars: int = 0
    makespan: float = 0.0
    builds: int = 0
    query_launches: int = 0
    peak_budget: int = 0

    def summary(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        rdy = np.array(self.ready) if self.ready else np.zeros(1)
        return {
            "query_batches": len(self.latencies), "strings": len(self.ready),
            "positions": self.positions, "chars_indexed": self.chars,
            "makespan_s": round(self.makespan, 4),
            "positions_per_s": round(self.positions / self.makespan, 1) if self.makespan else 0.0,
            "chars_indexed_per_s": round(self.chars / self.makespan, 1) if self.makespan else 0.0,
            "latency_p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "latency_p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "ready_p50_ms": round(float(np.percentile(rdy, 50)) * 1e3, 3),
            "ready_p99_ms": round(float(np.percentile(rdy, 99)) * 1e3, 3),
            "build_launch_chains": self.builds, "query_launches": self.query_launches,
            "peak_budget_bytes": self.peak_budget, "rejected": len(self.rejected),
        }


class Server:
    """Replays a request trace against the executor in real time.

    Budget accounting, in device bytes (the executor's own sizes): a string is
    charged its build-alone need from admission until its build completes;
    then its build is charged the resident index it keeps, once, until the
    build is released.  In-flight query launches are charged against a
    separate reserve (query_reserve_bytes, part of the budget),
    which strings are never admitted into, so builds, resident indexes and
    query buffers together stay within budget_bytes.  Up to
    max_query_launches launches are in flight (they run in order on one
    stream; the host prepares the next while the device runs the last).  A
    launch gathers arrived batches while they fit its share of the reserve
    (the reserve over max_query_launches) and what the reserve has left; with
    nothing in flight it takes at least one batch."""

    def __init__(self, executor, budget_bytes: int = 16 << 30, max_build_chars: int = 64 << 20,
                 query_reserve_bytes: int = 256 << 20, max_query_launches: int = 4,
                 max_build_chains: int = 2, clock=time.perf_counter):
        if not 0 < query_reserve_bytes < budget_bytes:
            raise ValueError("the query reserve must be positive and below the budget")
        if max_query_launches < 1 or max_build_chains < 1:
            raise ValueError("at least one query launch and one build must be allowed in flight")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.reserve = int(query_reserve_bytes)
        self.max_query_launches = int(max_query_launches)
        self.max_build_chains = int(max_build_chains)
        self.max_build_chars = int(max_build_chars)
        self.clock = clock

    def run(self, requests: Sequence[Request], keep_results: bool = True) -> ServeReport:
        rep = ServeReport()
        ex = self.ex
        arrivals = deque(sorted(requests, key=lambda r: r.arrival))
        waiting: deque = deque()            # arrived, not admitted
        admitted: List[_String] = []        # SA in progress or ready, not yet built
        building: List[Tuple[dict, List[_String]]] = []
        resident: List[_String] = []
        builds_live: Dict[int, List] = {}   # id(build) -> [build, strings alive, bytes held]
        inflight: List[Tuple[dict, List[Tuple[_String, int, float]], int]] = []
        used = 0                            # strings and builds
        qused = 0                           # query launches in flight
        room = self.budget - self.reserve   # for strings and builds
        t0 = self.clock()
        pending = len(arrivals)

        def now():
            return self.clock() - t0

        while pending:
            t = now()
            # 1. arrivals
            while arrivals and arrivals[0].arrival <= t:
                r = arrivals.popleft()
                waiting.append(_String(r, ex.string_bytes(len(r.text))))
            # 2. admission by budget, in arrival order
            while waiting and used + waiting[0].need <= room:
                s = waiting.popleft()
                used += s.need
                rep.peak_budget = max(rep.peak_budget, used + qused)
                s.sa_future = ex.submit_sa(s.req.text)
                admitted.append(s)
            if waiting and waiting[0].need > room:
                s = waiting.popleft()          # can never fit
                rep.rejected.append(s.req.rid)
                pending -= 1
            # 3. build every string whose SA is ready, as one batch, while
            #    fewer than max_build_chains builds are in flight
            if len(building) < self.max_build_chains:
                ready = []
                chars = 0
                for s in admitted:
                    if s.sa_future.done() and chars + len(s.req.text) <= max(self.max_build_chars, len(s.req.text)):
                        s.sa = s.sa_future.result()
                        ready.append(s)
                        chars += len(s.req.text)
                if ready:
                    admitted = [s for s in admitted if all(s is not x for x in ready)]
                    h = ex.start_build([s.req.text for s in ready], [s.sa for s in ready])
                    building.append((h, ready))
                    rep.builds += 1
            # 4. builds that finished: strings become resident; the strings'
            #    charges give way to the one resident index the build keeps
            for item in list(building):
                h, strs = item
                if ex.build_done(h):
                    building = [x for x in building if x is not item]
                    refs = ex.refs(h)
                    held = ex.index_bytes(h)
                    used += held - sum(s.need for s in strs)
                    builds_live[id(h)] = [h, len(strs), held]
                    tr = now()
                    for s, ref in zip(strs, refs):
                        s.build, s.ref, s.ready_at = h, ref, tr
                        s.sa = None
                        rep.ready.append(tr - s.req.arrival)
                        rep.chars += len(s.req.text)
                        resident.append(s)
            # 5. multi-string query launches for the arrived batches, up to
            #    max_query_launches in flight, each within its share of the
            #    query reserve (a launch takes at least one batch when none is
            #    in flight)
            share = self.reserve // self.max_query_launches
            while len(inflight) < self.max_query_launches:
                t = now()
                items, meta = [], []
                m = ma = 0
                refs = set()
                full = False
                for s in resident:
                    while s.next_batch < len(s.req.batches) and s.req.batch_times[s.next_batch] <= t:
                        qi = s.next_batch
                        n = len(s.req.batches[qi])
                        is_all = s.req.mode == "all"
                        m2, ma2 = (m, ma + n) if is_all else (m + n, ma)
                        nb = ex.query_bytes_sums(m2, ma2, len(refs) + (s.ref not in refs))
                        if (items or inflight) and (nb > share or qused + nb > self.reserve):
                            full = True
                            break
                        m, ma = m2, ma2
                        refs.add(s.ref)
                        items.append((s.ref, s.req.batches[qi], s.req.mode))
                        meta.append((s, qi, s.req.batch_times[qi]))
                        s.next_batch += 1
                        s.open_batches += 1
                    if full:
                        break
                if not items:
                    break
                qb = ex.query_bytes(items)
                qused += qb
                rep.peak_budget = max(rep.peak_budget, used + qused)
                inflight.append((ex.start_queries(items), meta, qb))
                rep.query_launches += 1
                if not full:
                    break
            # 6. finished query launches
            for item in list(inflight):
                h, meta, qb = item
                if ex.queries_done(h):
                    inflight = [x for x in inflight if x is not item]
                    qused -= qb
                    tq = now()
                    res = ex.query_results(h)
                    for (s, qi, arr), r in zip(meta, res):
                        rep.latencies.append(tq - arr)
                        rep.positions += len(s.req.batches[qi])
                        if keep_results:
                            rep.results[(s.req.rid, qi)] = r
                        s.open_batches -= 1
                        s.done_batches += 1
            # 7. evict strings whose batches are all answered; a build's memory
            #    is returned when its last string leaves
            for s in list(resident):
                if s.done_batches == len(s.req.batches):
                    resident = [x for x in resident if x is not s]
                    pending -= 1
                    live = builds_live[id(s.build)]
                    live[1] -= 1
                    if live[1] == 0:
                        ex.release_build(live[0])
                        used -= live[2]
                        del builds_live[id(s.build)]
                    s.build = s.ref = None
            # yield the interpreter lock every round: the SA and build threads
            # need it between their (lock-free) library calls, and a polling
            # loop that kept it would make each of their steps wait for the
            # interpreter's switch interval
            time.sleep(0)
        rep.makespan = now()
        return rep
