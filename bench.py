#!/usr/bin/env python3
"""Throughput of the all-positions longest-repeat query on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Headline workload: the batch of 512 independent DNA-like strings (lengths
log-uniform in [2^10, 2^20], 89,591,335 characters in all, seed 0) whose text,
segment offsets and segment-local suffix arrays are resident in HBM.  One step
is the whole hot path over the batch, one launch per stage: rank scatter ->
text-order LCP -> LLR filter (compaction) -> one scan that writes the leftmost
LR and all LRs of every position.  The step reads the all-mode record total
back and checks it against the record buffer (sized once, before timing, by
the count call; a short buffer would be enlarged and the scan repeated).

Beside the headline: the same 512 strings one string per launch chain (the
plain path), the batched step replayed from a HIP graph, the step with the
count pass included (an all-mode query that does not know its output size),
end to end from the host text, per-kernel figures and the roofline row of the
dominant kernel (HIP events on the kernels' own stream).  Further legs: the
single-string workloads (65,536 uniform, 2^24 DNA-like, 2^22 Fibonacci word,
2^26 Markov text), random-access probes sized to each leg's own tables,
serving at its measured capacity, and the CPU oracle on the batch's strings.

Inputs are synthetic (paper_1501_06663_amd.workloads), seeded.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
METRIC = "string positions/sec for all-positions LR query; batched vs plain on 1 GPU"
ENOSPC = -3
BOX_CPU_SHARE = 16   # host CPUs a one-GPU job may keep busy


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Plain:
    """Device buffers and one step of the hot path for one string or batch."""

    def __init__(self, text_np, sa_np, seg_off_np=None, dev=None):
        import torch
        from paper_1501_06663_amd import lrq
        self.lrq = lrq
        self.n = len(text_np)
        n = max(self.n, 1)
        self.dev = dev
        self.text = torch.from_numpy(text_np).to(dev)
        self.sa = torch.from_numpy(sa_np).to(dev)
        self.seg = None if seg_off_np is None else torch.from_numpy(seg_off_np).to(dev)
        self.nseg = 1 if seg_off_np is None else len(seg_off_np) - 1
        self.work = torch.empty(2 * n, dtype=torch.int32, device=dev)
        self.llrc = torch.empty((n, 2), dtype=torch.int32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int64, device=dev)
        self.blocks = torch.zeros(lrq.block_entries(self.n), dtype=torch.int64, device=dev)
        self.out = torch.empty((n, 2), dtype=torch.int32, device=dev)
        self.offs = torch.empty(self.n + 1, dtype=torch.int64, device=dev)
        self.scratch = torch.zeros(lrq.scratch_bytes(self.n, self.nseg), dtype=torch.uint8, device=dev)
        self.L = None  # the raw path's LLR array, allocated on first use
        # the all-mode record buffer, sized once here by the count call
        self.build()
        self.cap = lrq.lr_all_count(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.scratch)
        self.recs = torch.empty((max(self.cap, 1), 2), dtype=torch.int32, device=dev)
        self.total = self.cap

    def _grow(self, need):
        import torch
        if need > self.recs.shape[0]:
            self.recs = torch.empty((need, 2), dtype=torch.int32, device=self.dev)

    def build(self):
        self.lrq.index_build(self.text, self.sa, self.n, self.seg, self.nseg, self.work, self.llrc,
                             self.count, self.blocks, None, self.scratch)

    def scan(self, check=True):
        """Both modes in one pass into the record buffer.  With check, the call
        reads the record total back; a buffer it finds short is enlarged and
        the scan repeated (the records past its end were not written)."""
        l = self.lrq
        cap = int(self.recs.shape[0])
        try:
            tot = l.lr_both(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.out, self.offs,
                            self.recs, cap, self.scratch, want_total=check)
        except l.LrqError as e:
            if not check or e.status != ENOSPC:
                raise
            need = int(self.offs[self.n].item())
            l.read_errors(self.scratch)          # clears the overflow bit
            self._grow(need)
            tot = l.lr_both(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.out, self.offs,
                            self.recs, int(self.recs.shape[0]), self.scratch)
        if check:
            self.total = tot

    def step(self, check=True):
        """The hot path: build the index, then leftmost and all modes in one
        pass over the compact array."""
        self.build()
        self.scan(check)

    def cold_step(self):
        """The step of an all-mode query that does not know its record total:
        the count pass sizes the buffer (reallocated only when short), then
        the one-pass scan fills it."""
        l = self.lrq
        self.build()
        need = l.lr_all_count(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.scratch)
        self._grow(need)
        l.lr_both(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.out, self.offs, self.recs,
                  int(self.recs.shape[0]), self.scratch, want_total=False)

    def step_raw(self):
        """The raw-LLR path (Section 4.1; Algorithms 1 and 3 over L, no
        compaction): rank scatter, LCP pairs, Lemma-1 lengths, then the
        leftmost and all-mode walks."""
        import torch
        l = self.lrq
        if self.L is None:
            self.L = torch.empty(max(self.n, 1) + 2, dtype=torch.int32, device=self.out.device)
        l.rank_scatter(self.sa, self.n, self.seg, self.nseg, self.work, None, self.scratch)
        l.plcp(self.text, self.n, self.seg, self.nseg, self.work, self.scratch)
        l.llr_lengths(self.work, self.n, self.L)
        l.lr_all_raw(self.L, self.n, self.seg, self.nseg, self.offs, self.recs, int(self.recs.shape[0]),
                     self.scratch, want_total=False, out=self.out)

    def step_separate(self):
        """The same results from the two single-mode scans (the paper's two
        queries), for per-mode figures."""
        l = self.lrq
        self.build()
        l.lr_leftmost(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.out, self.scratch)
        l.lr_all(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.offs, self.recs,
                 int(self.recs.shape[0]), self.scratch, want_total=False)


def timed(fn, steps, warmup, record_kernels=False, only=None):
    """Seconds per step over `steps` steps after `warmup` untimed ones.  With
    record_kernels, HIP events bracket every kernel launch (or only launches of
    the kernel `only`, which leaves the other kernels' launches undisturbed);
    returns [(kernel, ms)] for them."""
    import torch
    from paper_1501_06663_amd import lrq
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if record_kernels:
        lrq.timing_only(only)
        lrq.timing_start(1 << 20)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = lrq.timing_collect() if record_kernels else []
    if record_kernels:
        lrq.timing_only(None)
    return (t1 - t0) / steps, kern


def algorithmic_bytes(name, n, m, recs):
    """Bytes per launch each kernel must move, from the data it reads and writes
    (int32 positions): the arrays named beside each entry, once each."""
    table = {
        "rank_scatter_kernel": 12.0 * n,                     # SA 4 in, neighbour pair 8 out
        "plcp_chunks_kernel": 19.0 * n,                      # pairs 8 in + 8 out, text 1, two compared chars
        "plcp_chunks_l_kernel": 15.0 * n,                    # pairs 8 in, L 4 out, text 1, two compared chars
        "plcp_llr_kernel": 11.0 * n + 8.0 * m,               # pairs 8 in, text 1, two chars, compact out
        "llr_filter_kernel": 8.0 * n + 8.0 * m,              # LCP pairs in, compact array out
        "llr_filter_l_kernel": 4.0 * n + 8.0 * m,            # L in, compact array out
        "lr_leftmost_kernel": 8.0 * m + 8.0 * n,             # compact array in, one record per position
        "lr_all_count_kernel": 8.0 * m,                      # compact array in, one total out
        "lr_all_kernel": 8.0 * m + 8.0 * n + 8.0 * recs,     # compact array in, CSR out
        "lr_both_kernel": 8.0 * m + 16.0 * n + 8.0 * recs,   # compact array in, leftmost + CSR out
    }
    return table.get(name)


def kernel_table(kern, steps, n, m, recs):
    agg = {}
    for name, ms in kern:
        name = name.split("<")[0]
        a = agg.setdefault(name, [0.0, 0])
        a[0] += ms
        a[1] += 1
    rows = {}
    for name, (tot, cnt) in agg.items():
        avg_ms = tot / cnt
        b = algorithmic_bytes(name, n, m, recs)
        row = {"launches_per_step": cnt / steps, "avg_us": round(avg_ms * 1e3, 2),
               "ms_per_step": round(tot / steps, 4)}
        if b is not None:
            gbps = b / (avg_ms * 1e-3) / 1e9
            row.update({"alg_bytes": int(b), "achieved_GBps": round(gbps, 1),
                        "frac_of_hbm_peak": round(gbps / PEAK_HBM_GBPS, 4)})
        rows[name] = row
    return rows


# ------------------------------------------------------- memory-system probes --

_PROBE = None


def probe_lib():
    """paper_1501_06663_amd/csrc/probe.hip: a streaming copy and random 8-byte
    gathers / scatters through an index array."""
    global _PROBE
    if _PROBE is None:
        import ctypes as C
        from paper_1501_06663_amd import build as B
        lib = C.CDLL(B.PROBE_LIB)
        for f in (lib.probe_copy, lib.probe_gather, lib.probe_scatter):
            f.restype = C.c_int
        lib.probe_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        lib.probe_gather.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                     C.c_void_p]
        lib.probe_scatter.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                      C.c_void_p]
        _PROBE = lib
    return _PROBE


def _event_clock(fn, reps, flush=None):
    """Mean seconds of fn() over reps runs, each timed alone with HIP events on
    torch's current stream (the probes launch there), after flush() if given."""
    import torch
    fn()
    tot = 0.0
    for _ in range(reps):
        if flush is not None:
            flush()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        tot += a.elapsed_time(b) * 1e-3
    return tot / reps


def copy_ceiling(dev, nbytes=1 << 30, reps=5):
    """Streaming-copy bandwidth (read + write) over nbytes, GB/s."""
    import torch
    lib = probe_lib()
    st = torch.cuda.current_stream().cuda_stream
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    sec = _event_clock(lambda: lib.probe_copy(a.data_ptr(), b.data_ptr(), nbytes // 16, st), reps)
    del a, b
    return round(2 * nbytes / sec / 1e9, 1)


def random_probes(dev, n, text_table_bytes, off=None, reps=4):
    """Ceilings for the two random-access kernels at one workload's own sizes.

    scatter: n random 8-byte writes through a permutation into a table of 8n
    bytes (the rank scatter's neighbour-pair array);
    gather: 2n random 8-byte reads from a table of text_table_bytes (the text
    as the LCP walk reads it, packed or not: two neighbour-side reads per
    position).  For a batch (segment offsets `off`), both are measured twice:
    uniform over the whole table, and confined to the strings the way the
    kernels' accesses are (slot g writes to a random position of its own
    string, and the reads for position p fall in p's string's part of the
    text), in the batch's own slot order.  Before each timed run a 512 MiB
    copy evicts the last-level cache, as the other stages of a step do."""
    import torch
    lib = probe_lib()
    st = torch.cuda.current_stream().cuda_stream
    fa = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
    fb = torch.empty_like(fa)

    def flush():
        lib.probe_copy(fa.data_ptr(), fb.data_ptr(), fa.numel() // 16, st)

    n = max(int(n), 1)
    tn = max(int(text_table_bytes) // 8, 1)

    def scatter_rate(perm):
        table = torch.zeros(n, dtype=torch.int64, device=dev)
        vals = torch.ones(n, dtype=torch.int64, device=dev)
        sec = _event_clock(lambda: lib.probe_scatter(perm.data_ptr(), vals.data_ptr(),
                                                     table.data_ptr(), n, n, st), reps, flush)
        return n / sec / 1e9

    def gather_rate(gidx):
        gtab = torch.zeros(tn, dtype=torch.int64, device=dev)
        gout = torch.empty(2 * n, dtype=torch.int64, device=dev)
        sec = _event_clock(lambda: lib.probe_gather(gidx.data_ptr(), gtab.data_ptr(), tn,
                                                    gout.data_ptr(), 2 * n, st), reps, flush)
        return 2 * n / sec / 1e9

    out = {"scatter_table_bytes": 8 * n,
           "scatter8_G_per_s": round(scatter_rate(torch.randperm(n, device=dev, dtype=torch.int32)), 2),
           "gather_table_bytes": 8 * tn,
           "gather8_G_per_s": round(gather_rate(torch.randint(0, tn, (2 * n,), device=dev,
                                                              dtype=torch.int32)), 2)}
    if off is not None and len(off) > 2 and int(off[-1]) == n:
        offs = torch.from_numpy(np.asarray(off, dtype=np.int64)).to(dev)
        lens = offs[1:] - offs[:-1]
        sid = torch.repeat_interleave(torch.arange(len(lens), device=dev), lens)
        # sorting by (string, random key) keeps every string's slots in place
        # and sends each slot to a random position of its own string
        key = sid * (1 << 32) + torch.randint(0, 1 << 31, (n,), device=dev, dtype=torch.int64)
        perm = torch.argsort(key).to(torch.int32)
        del key
        out["scatter8_in_strings_G_per_s"] = round(scatter_rate(perm), 2)
        del perm
        rs = sid.repeat_interleave(2)
        pos = offs[rs] + (torch.rand(2 * n, device=dev) * lens[rs].to(torch.float32)).to(torch.int64)
        pos = torch.minimum(pos, offs[rs + 1] - 1)
        gidx = (pos * (8 * tn) // n // 8).clamp_(0, tn - 1).to(torch.int32)
        del rs, pos, sid
        out["gather8_in_strings_G_per_s"] = round(gather_rate(gidx), 2)
        out["longest_string"] = int(lens.max())
        del gidx
    del fa, fb
    torch.cuda.empty_cache()
    return out


def text_table_bytes(text):
    """Bytes of the text as the LCP kernels read it: 1, 2 or 4 bits per
    character for at most 2, 4 or 16 distinct byte values, else bytes."""
    sigma = max(int(np.count_nonzero(np.bincount(text, minlength=256))), 1)
    bits = 1 if sigma <= 2 else 2 if sigma <= 4 else 4 if sigma <= 16 else 8
    return max(len(text) * bits // 8, 8)


def random_access(kt, n, probes):
    """The random-access kernels against the probes of their own access
    pattern and size."""
    out = {}
    # a batch's kernels are compared with the probes confined to its strings
    scat = probes.get("scatter8_in_strings_G_per_s", probes["scatter8_G_per_s"])
    gath = probes.get("gather8_in_strings_G_per_s", probes["gather8_G_per_s"])
    within = "within each string" if "scatter8_in_strings_G_per_s" in probes else "uniform"
    rs = kt.get("rank_scatter_kernel")
    if rs:
        rate = n / (rs["avg_us"] * 1e-6) / 1e9
        out["rank_scatter_kernel"] = {
            "random_8B_writes_per_position": 1, "G_writes_per_s": round(rate, 2),
            "probe_scatter8_G_per_s": scat, "probe_pattern": within,
            "probe_table_bytes": probes["scatter_table_bytes"],
            "frac_of_probe": round(rate / scat, 3)}
    for name in ("plcp_chunks_kernel", "plcp_chunks_l_kernel", "plcp_llr_kernel"):
        r = kt.get(name)
        if r:
            rate = 2 * n / (r["avg_us"] * 1e-6) / 1e9
            out[name] = {
                "random_text_reads_per_position": 2, "G_reads_per_s": round(rate, 2),
                "probe_gather8_G_per_s": gath, "probe_pattern": within,
                "probe_table_bytes": probes["gather_table_bytes"],
                "frac_of_probe": round(rate / gath, 3),
                "note": "two neighbour-side text reads per position at most (Kasai's bound "
                        "skips some; long compares read more words)"}
    return out


# ------------------------------------------------------------------ traffic --

TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_traffic_%s.md")  # per workload
# the kernels' source: the device code and the layout/tile constants it includes
DEVICE_SOURCES = [os.path.join(ROOT, "paper_1501_06663_amd", "csrc", f)
                  for f in ("lrq_device.hip", "lrq_internal.h")]


def pmc_traffic(kernel, workload):
    """Bytes per launch of `kernel` as rocprofv3's FETCH_SIZE + WRITE_SIZE
    counters read them (scaled by what they read for a copy kernel of known
    size), from the committed counter summary of this workload.  These
    counters count traffic between the L2 and the memory fabric, so lines
    served by the last-level cache count too.  None when that summary does not
    cover the kernel, or when the kernel source has changed since the counters
    were taken (the summary records the source's SHA-256)."""
    import hashlib
    try:
        with open(TRAFFIC_SUMMARY % workload) as f:
            lines = [l for l in f if l.startswith("traffic-json: ")]
        rec = json.loads(lines[-1][len("traffic-json: "):])
        h = hashlib.sha256()
        for path in DEVICE_SOURCES:
            with open(path, "rb") as f:
                h.update(f.read())
        digest = h.hexdigest()
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_sha256") != digest:
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


# --------------------------------------------------------------- CPU oracle --

def host_info():
    """The host CPU: model, logical CPUs, the CPUs this process may run on and
    the cgroup's CPU quota."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, p = f.read().split()[:2]
            quota = None if q == "max" else round(int(q) / int(p), 2)
    except (OSError, ValueError):
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "cpus_allowed": aff,
            "cgroup_cpu_quota": quota}


def cpu_baseline(text, off, min_seconds, sample_frac=0.25):
    """The oracle on the headline batch's strings.  Strings are taken in a
    seeded random order until they hold sample_frac of the batch's
    characters; each gets the oracle's own suffix sort (untimed: the GPU step
    starts from resident suffix arrays too), then the step's span -- Rank,
    Kasai LCP, Lemma-1 lengths, compaction, Algorithm 1 and Algorithm 3
    walks -- is run over the whole sample, repeatedly until min_seconds have
    passed, with the oracle's per-position loops on the machine's CPU share, and
    once more on one thread."""
    import oracle
    info = host_info()
    threads = oracle.set_threads(max(1, min(info["cpus_allowed"] or 1, BOX_CPU_SHARE)))
    nseg = len(off) - 1
    order = np.random.default_rng(0).permutation(nseg)
    want = sample_frac * len(text)
    sample, chars = [], 0
    t0 = time.perf_counter()
    for b in order:
        if chars >= want:
            break
        s = np.ascontiguousarray(text[off[b]:off[b + 1]])
        sample.append((s, oracle.suffix_array(s)))
        chars += len(s)
    sa_s = time.perf_counter() - t0
    stages = {"rank": 0.0, "lcp_kasai": 0.0, "lemma1_lengths": 0.0, "compaction": 0.0,
              "alg1_leftmost_raw": 0.0, "alg3_all_raw": 0.0}

    def span():
        for s, sa in sample:
            t = [time.perf_counter()]
            rk = oracle.rank(sa)
            t.append(time.perf_counter())
            lc = oracle.lcp(s, sa, rk)
            t.append(time.perf_counter())
            L = oracle.llr_lengths(rk, lc)
            t.append(time.perf_counter())
            oracle.compact(L)
            t.append(time.perf_counter())
            oracle.lr_leftmost_raw(L)
            t.append(time.perf_counter())
            oracle.lr_all_raw(L)
            t.append(time.perf_counter())
            for i, key in enumerate(stages):
                stages[key] += t[i + 1] - t[i]

    reps, spent = 0, 0.0
    while reps == 0 or spent < min_seconds:
        t1 = time.perf_counter()
        span()
        spent += time.perf_counter() - t1
        reps += 1
    oracle.set_threads(1)
    t1 = time.perf_counter()
    for key in stages:
        stages[key] = stages[key] / reps
    saved = dict(stages)
    span()
    one_s = time.perf_counter() - t1
    oracle.set_threads(threads)
    return {"value": round(chars * reps / spent, 1), "unit": "positions/s", "cores": threads,
            "kind": "oracle",
            "single_thread_positions_per_s": round(chars / one_s, 1),
            "host": info,
            "sample": ("%d of the headline batch's 512 DNA-like strings (%d characters, a seeded "
                       "random choice covering %.0f%% of the batch); timed span = Rank, Kasai LCP, "
                       "Lemma-1 lengths, compaction, Algorithm 1 and Algorithm 3 walks over every "
                       "string of the sample (the GPU step's span, from resident suffix arrays), "
                       "run %d times in %.2f s on %d threads (the CPU share of a one-GPU job on this "
                       "host); the oracle's suffix sorts of the sample took a further %.2f s, untimed"
                       % (len(sample), chars, 100.0 * chars / max(len(text), 1), reps, spent, threads,
                          sa_s)),
            "stage_s_per_rep": {k: round(v, 4) for k, v in saved.items()}}


# ------------------------------------------------------------------- legs --

def parse_tuning(s):
    if not s:
        return None
    out = {}
    for kv in s.split(","):
        k, v = kv.split("=")
        out[k.strip()] = int(v)
    return out


def measure(plain, steps, warmup, tune, tuning=None):
    """Choose the kernel shapes (fixed, autotuned or the defaults), then time
    `steps` steps of the hot path on one prepared string or batch:
    positions/s, per-kernel table, spans, the cold all-mode step, and the
    roofline row of the kernel that takes the most time per step."""
    from paper_1501_06663_amd import lrq
    n = plain.n
    m = plain.count.item()
    log("n %d: compact entries %d, all-mode records %d" % (n, m, plain.cap))
    if tuning is not None:
        lrq.set_tuning(**tuning)
        tuned = {"chosen": lrq.get_tuning(), "fixed": True}
    elif tune:
        from paper_1501_06663_amd import autotune
        t = autotune.tune(plain.step, key=autotune.size_key(n, plain.nseg), reps=3, use_cache=False)
        tuned = {"chosen": t["tuning"], "trials": t["trials"]}
        log("tuning %s (%.3f ms)" % (t["tuning"], t["seconds"] * 1e3))
    else:
        lrq.set_tuning()
        tuned = {"chosen": lrq.get_tuning(), "defaults": True}
    # Per-kernel breakdown: untimed steps with events around every launch (the
    # events add a few microseconds per launch, so these steps are not the
    # headline figure).
    bsteps = max(3, min(steps, 10))
    _, kern = timed(plain.step, bsteps, warmup, record_kernels=True)
    kt = kernel_table(kern, bsteps, n, m, plain.cap)
    dname, _ = max((r for r in kt.items() if "alg_bytes" in r[1]),
                   key=lambda kv: kv[1]["ms_per_step"])
    # The timed steps: events around the dominant kernel's launches only.
    sec, dkern = timed(plain.step, steps, 1, record_kernels=True, only=dname)
    errs = lrq.read_errors(plain.scratch)
    if errs:
        raise SystemExit("device error bits %d" % errs)
    if plain.total != plain.cap:
        raise SystemExit("record total changed between steps: %d vs %d" % (plain.total, plain.cap))
    log("step %.3f ms -> %.3e positions/s" % (sec * 1e3, n / sec))
    drow = kernel_table(dkern, steps, n, m, plain.cap)[dname]
    roofline = {"bound": "hbm", "kernel": dname, "achieved": drow["achieved_GBps"],
                "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": drow["frac_of_hbm_peak"],
                "avg_us": drow["avg_us"]}
    # the single-mode scans, timed on their own (same index, same buffers)
    ssteps = max(3, steps // 2)
    _, skern = timed(plain.step_separate, ssteps, 1, record_kernels=True)
    if lrq.read_errors(plain.scratch):
        raise SystemExit("device error bits after the single-mode scans")
    st = kernel_table(skern, ssteps, n, m, plain.cap)
    modes = {k: st[k] for k in ("lr_leftmost_kernel", "lr_all_kernel") if k in st}
    # an all-mode query that sizes its output first
    csec, ckern = timed(plain.cold_step, ssteps, 1, record_kernels=True, only="lr_all_count_kernel")
    if lrq.read_errors(plain.scratch):
        raise SystemExit("device error bits after the cold steps")
    count_row = kernel_table(ckern, ssteps, n, m, plain.cap).get("lr_all_count_kernel")
    both = dict(kt)
    both.update(modes)
    # build = rank scatter .. filter; the scans; and filter + scan (the paper's
    # timed span: LLR array and walks from a resident LCP)
    spans = {}
    filt = "llr_filter_l_kernel" if "llr_filter_l_kernel" in both else "llr_filter_kernel"
    for name, calls in (("build", [c for c in kt if not c.startswith("lr_")]),
                        ("both_scan", ("lr_both_kernel",)),
                        ("leftmost_scan", ("lr_leftmost_kernel",)),
                        ("all_scan", ("lr_all_kernel",)),
                        ("filter_plus_leftmost", (filt, "lr_leftmost_kernel")),
                        ("filter_plus_all", (filt, "lr_all_kernel"))):
        if not all(c in both for c in calls):
            continue
        ms = sum(both[c]["ms_per_step"] for c in calls)
        spans[name] = {"ms": round(ms, 4), "positions_per_s": round(n / (ms * 1e-3), 1)}
    return {"sec": sec, "positions_per_s": round(n / sec, 1), "ms_per_step": round(sec * 1e3, 4),
            "kernels": kt, "single_mode_kernels": modes, "spans": spans, "roofline": roofline,
            "cold_step": {"ms_per_step": round(csec * 1e3, 4), "positions_per_s": round(n / csec, 1),
                          "count_kernel_us": None if count_row is None else count_row["avg_us"]},
            "tuning": tuned, "compact_entries": int(m), "all_mode_records": int(plain.cap)}


def raw_leg(plain, steps, warmup):
    """The raw-LLR path (Plain.step_raw) on the same string or batch: step
    time, per-kernel breakdown, and whether its answers equal the compact
    path's, element by element."""
    import torch
    from paper_1501_06663_amd import lrq
    n = plain.n
    plain.step()
    torch.cuda.synchronize()
    ref = (plain.out[:n].clone(), plain.offs.clone(), plain.recs[:plain.total].clone())
    lrq.read_errors(plain.scratch)  # clears the error word
    sec, _ = timed(plain.step_raw, steps, warmup)
    bsteps = max(3, min(steps, 10))
    _, kern = timed(plain.step_raw, bsteps, 1, record_kernels=True)
    errs = lrq.read_errors(plain.scratch)
    same = (errs == 0 and torch.equal(plain.out[:n], ref[0]) and torch.equal(plain.offs, ref[1])
            and torch.equal(plain.recs[:plain.total], ref[2]))
    kt = kernel_table(kern, bsteps, n, plain.count.item(), plain.cap)
    # Lemma 4's alpha: the mean LLR length, the mean number of LLRs covering a
    # position, hence the mean walk
    alpha = float(plain.L[:n].double().mean().item()) if n else 0.0
    log("raw path: step %.3f ms (%s), alpha %.2f, same answers as the compact path: %s"
        % (sec * 1e3, "errors %d" % errs if errs else "no errors", alpha, same))
    # the autotuner's choice between the two paths for this workload
    from paper_1501_06663_amd import autotune
    pick = autotune.choose_path({"compact": plain.step, "raw": plain.step_raw}, use_cache=False)
    log("path choice: %s %s" % (pick["path"], pick["trials"]))
    return {"ms_per_step": round(sec * 1e3, 4), "positions_per_s": round(n / sec, 1),
            "path_choice": {"chosen": pick["path"], "seconds": pick["trials"]},
            "alpha_mean_llr_length": round(alpha, 3),
            "compact_entries_per_position": round(plain.count.item() / max(n, 1), 4),
            "kernels_us": {k: v["avg_us"] for k, v in kt.items()},
            "same_answers_as_compact": bool(same), "error_bits": int(errs)}


def end_to_end(plain, text, sa, off, host_sa_s):
    """From the host: (a) host SA + pageable copies of text and SA + one step;
    (b) text copy + SA on the device + one step (best of three)."""
    import torch
    from paper_1501_06663_amd import lrq
    n = plain.n
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain.text.copy_(torch.from_numpy(text))
    plain.sa.copy_(torch.from_numpy(sa))
    torch.cuda.synchronize()
    h2d_s = time.perf_counter() - t0
    step_s, _ = timed(plain.step, 3, 1)
    sa_work = torch.empty(lrq.sa_work_bytes(n, plain.nseg), dtype=torch.uint8, device=plain.dev)
    runs = []
    for rep in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain.text.copy_(torch.from_numpy(text))
        t1 = time.perf_counter()
        lrq.build_sa(plain.text, n, plain.seg, plain.nseg, plain.sa, sa_work)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        plain.step()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if rep:  # the first repetition warms up
            runs.append((t1 - t0, t2 - t1, t3 - t2, t3 - t0))
    if lrq.read_errors(plain.scratch):
        raise SystemExit("device error bits after the device-SA runs")
    if not np.array_equal(plain.sa.cpu().numpy(), sa):
        raise SystemExit("device SA differs from the host SA")
    del sa_work
    best = min(runs, key=lambda x: x[3])
    log("device SA %.2f ms; end to end %.2f ms" % (best[1] * 1e3, best[3] * 1e3))
    e2e_s = host_sa_s + h2d_s + step_s
    return {"host_sa": {"host_sa_s": round(host_sa_s, 3), "h2d_ms": round(h2d_s * 1e3, 3),
                        "step_ms": round(step_s * 1e3, 4), "positions_per_s": round(n / e2e_s, 1)},
            "device_sa": {"text_h2d_ms": round(best[0] * 1e3, 3), "device_sa_ms": round(best[1] * 1e3, 3),
                          "step_ms": round(best[2] * 1e3, 3), "total_ms": round(best[3] * 1e3, 3),
                          "positions_per_s": round(n / best[3], 1)}}


def int64_leg(plain, steps, warmup):
    """The same step through the 64-bit calls (lrq64_index_build +
    lrq64_lr_both: int64 SA, positions, lengths and records), on the same
    resident strings, checked against the 32-bit step's outputs."""
    import torch
    l = plain.lrq
    dev, n = plain.dev, plain.n
    t = max(n, 1)
    sa = plain.sa.to(torch.int64)
    work = torch.empty((t, 2), dtype=torch.int64, device=dev)
    llrc = torch.empty((t, 2), dtype=torch.int64, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    blocks = torch.zeros(l.block_entries(n), dtype=torch.int64, device=dev)
    out = torch.empty((t, 2), dtype=torch.int64, device=dev)
    offs = torch.empty(n + 1, dtype=torch.int64, device=dev)
    cap = int(plain.total)
    recs = torch.empty((max(cap, 1), 2), dtype=torch.int64, device=dev)
    scratch = torch.zeros(l.scratch_bytes64(n, plain.nseg), dtype=torch.uint8, device=dev)
    tot = [0]

    def step():
        l.index_build64(plain.text, sa, n, plain.seg, plain.nseg, work, llrc, count, blocks, None,
                        scratch)
        tot[0] = l.lr_both64(llrc, blocks, n, plain.seg, plain.nseg, out, offs, recs, cap, scratch)
    sec, _ = timed(step, steps, warmup)
    plain.step()
    torch.cuda.synchronize()
    same = (tot[0] == plain.total and torch.equal(out, plain.out.to(torch.int64))
            and torch.equal(offs, plain.offs)
            and torch.equal(recs[:tot[0]], plain.recs[:plain.total].to(torch.int64))
            and l.read_errors(scratch) == 0)
    if not same:
        raise SystemExit("the 64-bit calls disagree with the 32-bit ones on the batch")
    log("64-bit calls: %.3f ms per step" % (sec * 1e3))
    return {"ms_per_step": round(sec * 1e3, 4), "positions_per_s": round(n / sec, 1),
            "same_answers_as_int32": True,
            "note": "lrq64_index_build + lrq64_lr_both on the same strings: int64 SA, positions, "
                    "lengths and records (16-byte pairs); the build runs the filter with its own "
                    "look-back"}


def headline_leg(args, dev, tuning):
    """The batch of 512 strings: the timed step, the graph replay, the cold
    step, the plain one-string-per-launch path on the same strings, end to
    end, raw path, probes."""
    import torch
    from paper_1501_06663_amd import lrq, workloads
    text, off = workloads.config4()
    t0 = time.perf_counter()
    sa = lrq.build_sa_host_batch(text, off)
    host_sa_s = time.perf_counter() - t0
    nseg = len(off) - 1
    log("batch: %d strings, %d chars, host SA %.2f s" % (nseg, len(text), host_sa_s))
    bat = Plain(text, sa, off, dev)
    meas = measure(bat, args.steps, args.warmup, not args.no_tune, tuning)
    leg = {"meas": meas, "text": text, "off": off, "n": bat.n}
    if args.plain_only:
        return leg
    # the same step captured once in a HIP graph and replayed (no host read of
    # the total inside a graph; the buffer is already the right size)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bat.step(check=False)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bat.step(check=False)
    gsec, _ = timed(graph.replay, max(3, args.steps // 2), 1)
    del graph
    if lrq.read_errors(bat.scratch):
        raise SystemExit("device error bits after the graph replays")
    leg["graph"] = {"ms_per_step": round(gsec * 1e3, 4), "positions_per_s": round(bat.n / gsec, 1)}
    leg["e2e"] = end_to_end(bat, text, sa, None, host_sa_s)
    leg["raw_path"] = raw_leg(bat, max(3, args.steps // 2), args.warmup)
    leg["int64_path"] = int64_leg(bat, max(3, args.steps // 2), args.warmup)
    del bat
    torch.cuda.empty_cache()
    # the plain path: the same strings, one launch chain per string (each
    # string's record buffer sized beforehand, no host read per string, one
    # synchronisation at the end), under the same kernel shapes
    singles = [Plain(text[off[b]:off[b + 1]].copy(), sa[off[b]:off[b + 1]].copy(), None, dev)
               for b in range(nseg)]

    def one_per_launch():
        for p in singles:
            p.step(check=False)
    ssec, _ = timed(one_per_launch, 3, 1)
    bad = [b for b, p in enumerate(singles) if lrq.read_errors(p.scratch)]
    if bad:
        raise SystemExit("device error bits in the one-per-launch strings %s" % bad[:5])
    del singles
    torch.cuda.empty_cache()
    leg["one_per_launch"] = {"ms_per_step": round(ssec * 1e3, 4),
                             "positions_per_s": round(len(text) / ssec, 1)}
    log("batched %.3f ms vs one string per launch %.3f ms" % (meas["sec"] * 1e3, ssec * 1e3))
    leg["probes"] = random_probes(dev, len(text), text_table_bytes(text), off)
    leg["random_access"] = random_access(meas["kernels"], len(text), leg["probes"])
    return leg


SINGLE_CONFIGS = (
    ("uniform_64k", "plain i.i.d. uniform ACGT, n=65,536, seed 0", "config1"),
    ("dna16m", "plain DNA-like string, n=16,777,216, P(ACGT)=.3/.2/.2/.3, 2000 planted mutated "
               "copies (log-uniform 50-5000), seed 0", "config2"),
    ("fibonacci_4m", "plain Fibonacci word, n=2^22", "config3a"),
    ("markov64m", "plain order-2 Markov text over 96 printable symbols, Zipf(1.1), n=2^26, seed 0",
     "config3b"),
)


def single_leg(name, desc, make, args, dev, tuning=None, extras=True):
    """The step on one single-string workload."""
    import torch
    from paper_1501_06663_amd import lrq, workloads
    t0 = time.perf_counter()
    text = getattr(workloads, make)()
    t1 = time.perf_counter()
    sa = lrq.build_sa_host(text)
    host_sa_s = time.perf_counter() - t1
    log("%s: n %d, generate %.2f s, host SA %.2f s" % (name, len(text), t1 - t0, host_sa_s))
    plain = Plain(text, sa, None, dev)
    steps = max(3, args.steps // 2) if extras else args.steps
    meas = measure(plain, steps, args.warmup, not args.no_tune, tuning)
    del meas["sec"]
    meas["workload"] = desc
    if extras:
        if name != "fibonacci_4m":  # its LLRs are ~10^6 long: the raw walks do not apply
            meas["raw_path"] = raw_leg(plain, steps, args.warmup)
        if name == "dna16m":
            meas["e2e"] = end_to_end(plain, text, sa, None, host_sa_s)
        meas["probes"] = random_probes(dev, len(text), text_table_bytes(text))
        meas["random_access"] = random_access(meas["kernels"], len(text), meas["probes"])
        for k, row in list(meas["kernels"].items()) + list(meas["single_mode_kernels"].items()):
            row["traffic"] = pmc_traffic(k, name)
    del plain, text, sa
    torch.cuda.empty_cache()
    return meas


def serving_leg(args):
    """Serving at its measured capacity.  The capacity run replays the trace
    with every string and every query batch arriving at once, so that nothing
    waits on the trace's clock: strings processed per second of that run is
    what the server sustains.  The same strings and query batches then arrive
    with the trace's own timing (Poisson arrivals, 2 ms mean gaps between a
    string's batches) at 0.5, 0.8 and 1.0 times that rate."""
    from paper_1501_06663_amd import serving, workloads
    ex = serving.GpuExecutor(sa_threads=BOX_CPU_SHARE)
    base_rate = 100.0
    t0 = time.perf_counter()
    trace = list(workloads.serving_trace(base_rate, args.serving_strings, seed=0,
                                         all_fraction=args.serving_all_fraction))
    n_all = sum(r.mode == "all" for r in trace)
    log("serving trace: %d strings (%d in all mode), %d chars, %d query batches, %d positions "
        "(%.1f s to generate)" % (
            len(trace), n_all, sum(len(r.text) for r in trace), sum(len(r.batches) for r in trace),
            sum(sum(len(b) for b in r.batches) for r in trace), time.perf_counter() - t0))
    budget = 32 << 30
    shape = {"budget_bytes": budget, "query_reserve_bytes": 256 << 20, "max_query_launches": 4,
             "max_build_chains": 2}

    def server():
        return serving.Server(ex, **shape)

    # warm-up: one whole backlog run, so that the allocators (device and
    # pinned host memory) have grown to the trace's needs before anything is
    # timed; then three backlog runs, whose makespan moves with the host's
    # scheduling: the capacity is their median
    server().run(workloads.retime(trace, 0.0, 0.0), keep_results=False)
    runs = sorted((server().run(workloads.retime(trace, 0.0, 0.0), keep_results=False)
                   for _ in range(3)), key=lambda r: r.makespan)
    sat = runs[1]
    ssum = sat.summary()
    cap = len(trace) / sat.makespan
    log("serving capacity %.1f strings/s (%.3e positions/s; backlog runs %s strings/s)" % (
        cap, ssum["positions_per_s"], ", ".join("%.1f" % (len(trace) / r.makespan) for r in runs)))
    legs = []
    for frac in (0.5, 0.8, 1.0):
        rate = frac * cap
        rep = server().run(workloads.retime(trace, base_rate / rate), keep_results=False)
        summ = rep.summary()
        summ["fraction_of_capacity"] = frac
        summ["arrival_rate_strings_per_s"] = round(rate, 2)
        legs.append(summ)
        log("  %.1f x capacity: p50 %.2f ms p99 %.2f ms, ready p99 %.2f ms, %.3e positions/s" % (
            frac, summ["latency_p50_ms"], summ["latency_p99_ms"], summ["ready_p99_ms"],
            summ["positions_per_s"]))
    if ex.errors():
        raise SystemExit("serving: device error bits")
    return {
        "workload": "Poisson arrivals of %d DNA-like or protein-like strings, lengths log-uniform "
                    "in [1e4, 4e6]; 1-64 query batches each of 1e3-1e5 uniform positions, "
                    "exponential gaps of mean 2 ms after the string's arrival; %d strings ask "
                    "for all LRs of their positions, the rest for the leftmost; device suffix "
                    "arrays; seed 0" % (len(trace), n_all),
        "server": shape,
        "capacity_run": "every string and query batch arriving at t = 0; the median of three "
                        "such runs",
        "capacity_runs_strings_per_s": [round(len(trace) / r.makespan, 2) for r in runs],
        "capacity_strings_per_s": round(cap, 2),
        "capacity_positions_per_s": ssum["positions_per_s"],
        "capacity_chars_indexed_per_s": ssum["chars_indexed_per_s"],
        "saturated": ssum, "legs": legs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=("batch512", "dna16m", "markov64m", "fibonacci_4m",
                                           "uniform_64k"), default="batch512",
                    help="the workload of the headline step (default: the 512-string batch)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serving-all-fraction", type=float, default=0.25,
                    help="share of served strings whose batches ask for all LRs")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall time the oracle baseline repeats its span for")
    ap.add_argument("--plain-only", action="store_true",
                    help="only the headline workload's timed step (profiling runs)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the single-string legs")
    ap.add_argument("--no-tune", action="store_true", help="keep the default kernel shapes")
    ap.add_argument("--tuning", type=str, default="",
                    help="fixed kernel shapes, e.g. plcp_chunk=8,llr_waves=8,lr_tile=2048,fuse_filter=0")
    ap.add_argument("--serving-strings", type=int, default=192)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of known "
                         "traffic, to calibrate profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (--gpus %d "
              "is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1501_06663_amd import lrq  # noqa: F401  (fails loudly without liblrq.so)
    dev = torch.device("cuda:0")
    tuning = parse_tuning(args.tuning)

    if args.copy_mib:
        # one launch of the probe library's streaming copy_kernel: a kernel whose
        # traffic is known exactly (copy_mib MiB read, copy_mib MiB written)
        src = torch.ones(args.copy_mib << 18, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        rc = probe_lib().probe_copy(src.data_ptr(), dst.data_ptr(), (args.copy_mib << 20) // 16,
                                    torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        if rc != 0:
            raise SystemExit("probe_copy failed: %d" % rc)
        log("calibration copy_kernel: %d MiB read + %d MiB written" % (args.copy_mib, args.copy_mib))
        del src, dst

    if args.workload != "batch512":
        # a single-string workload as the headline (profiling runs)
        name, desc, make = [c for c in SINGLE_CONFIGS if c[0] == args.workload][0]
        meas = single_leg(name, desc, make, args, dev, tuning, extras=not args.plain_only)
        n = {"uniform_64k": 65536, "dna16m": 1 << 24, "fibonacci_4m": 1 << 22,
             "markov64m": 1 << 26}[name]
        print(json.dumps({"metric": METRIC, "value": meas["positions_per_s"], "unit": "positions/s",
                          "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": meas["ms_per_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "int32",
                          "data": "synthetic", "config": {"workload": desc, "n": n},
                          "roofline": meas["roofline"], "leg": meas}), flush=True)
        return

    head = headline_leg(args, dev, tuning)
    meas = head["meas"]
    n = head["n"]
    sec, kt = meas["sec"], meas["kernels"]
    roofline = dict(meas["roofline"])
    roofline["traffic"] = pmc_traffic(roofline["kernel"], "batch512")
    roofline["traffic_source"] = ("rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, scaled by a copy "
                                  "kernel of known size (profiles/pmc_traffic_batch512.md); counted "
                                  "between L2 and the memory fabric, so last-level-cache hits are "
                                  "included: an upper bound on HBM bytes")
    for k, row in list(kt.items()) + list(meas["single_mode_kernels"].items()):
        row["traffic"] = pmc_traffic(k, "batch512")
    wdesc = ("batched: 512 independent DNA-like strings, lengths log-uniform in [2^10, 2^20], "
             "%d characters in all, seed 0; one launch per stage with segment offsets" % n)
    result = {
        "metric": METRIC, "value": round(n / sec, 1), "unit": "positions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wdesc, "strings": 512, "positions": n,
                   "span": "rank scatter + text-order LCP + LLR filter + one scan giving the leftmost "
                           "LR and all LRs of every position, with a host read of the record total; "
                           "text, segment offsets and suffix arrays resident in HBM; record buffer "
                           "sized before timing (cold_step includes the count pass)",
                   "compact_entries": int(meas["compact_entries"]),
                   "all_mode_records": int(meas["all_mode_records"])},
        "roofline": roofline,
    }
    if not args.plain_only:
        op = head["one_per_launch"]
        result["batched_vs_plain"] = {
            "batched_positions_per_s": round(n / sec, 1), "batched_ms": round(sec * 1e3, 4),
            "plain_one_string_per_launch_positions_per_s": op["positions_per_s"],
            "plain_one_string_per_launch_ms": op["ms_per_step"],
            "speedup": round(op["ms_per_step"] / (sec * 1e3), 3),
            "batched_graph_positions_per_s": head["graph"]["positions_per_s"],
            "batched_graph_ms": head["graph"]["ms_per_step"]}
    result.update({"kernels": kt, "single_mode_kernels": meas["single_mode_kernels"],
                   "spans": meas["spans"], "cold_step": meas["cold_step"], "tuning": meas["tuning"]})
    for k in ("e2e", "raw_path", "int64_path", "probes", "random_access"):
        if k in head:
            result[k] = head[k]
    if not args.plain_only:
        result["ceilings"] = {"copy_GBps": copy_ceiling(dev)}
        log("copy ceiling %s GB/s" % result["ceilings"]["copy_GBps"])
    if not args.plain_only and not args.no_configs:
        legs = {}
        for name, desc, make in SINGLE_CONFIGS:
            legs[name] = single_leg(name, desc, make, args, dev, tuning)
        result["other_configs"] = legs
    if not args.plain_only and not args.no_serving:
        result["served"] = serving_leg(args)
    if not args.no_cpu and not args.plain_only:
        log("cpu baseline (oracle) on the batch's strings, >= %.0f s" % args.cpu_seconds)
        result["cpu_baseline"] = cpu_baseline(head["text"], head["off"], args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
