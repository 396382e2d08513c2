#!/usr/bin/env python3
"""Throughput of the all-positions longest-repeat query on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

One step is the whole hot path over one DNA-like string of 16,777,216
characters whose text and suffix array are already resident in HBM: rank
scatter -> text-order LCP -> LLR filter (compaction) -> leftmost LR of every
position -> all LRs of every position (one pass into a buffer sized once,
before timing, by the count call).  The JSON line reports
positions per second of that step, the roofline of its dominant kernel (HIP
events on the kernels' own stream), per-kernel figures, the batched path
(512 strings in one launch per stage) against the same strings one per
launch, and the CPU oracle timed on a bounded sample.

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
        # size the all-mode output once; every step then runs the one-pass kernel
        self.build()
        self.cap = lrq.lr_all_count(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.scratch)
        self.recs = torch.empty((max(self.cap, 1), 2), dtype=torch.int32, device=dev)

    def build(self):
        self.lrq.index_build(self.text, self.sa, self.n, self.seg, self.nseg, self.work, self.llrc,
                             self.count, self.blocks, None, self.scratch)

    def step(self):
        """The hot path: build the index, then leftmost and all modes in one
        pass over the compact array."""
        self.build()
        self.lrq.lr_both(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.out, self.offs,
                         self.recs, self.cap, self.scratch, want_total=False)

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
        l.lr_all_raw(self.L, self.n, self.seg, self.nseg, self.offs, self.recs, self.cap,
                     self.scratch, want_total=False, out=self.out)

    def step_separate(self):
        """The same results from the two single-mode scans (the paper's two
        queries), for per-mode figures."""
        l = self.lrq
        self.build()
        l.lr_leftmost(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.out, self.scratch)
        l.lr_all(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.offs, self.recs, self.cap,
                 self.scratch, want_total=False)


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
    rho = m / n
    table = {
        "rank_scatter_kernel": 12.0 * n,                     # SA 4 in, neighbour pair 8 out
        "plcp_chunks_kernel": 19.0 * n,                      # pairs 8 in + 8 out, text 1, two compared chars
        "plcp_llr_kernel": 11.0 * n + 8.0 * m,               # pairs 8 in, text 1, two chars, compact out
        "llr_filter_kernel": 8.0 * n + 8.0 * m,              # LCP pairs in, compact array out
        "lr_leftmost_kernel": 8.0 * m + 8.0 * n,             # compact array in, one record per position
        "lr_all_kernel": 8.0 * m + 8.0 * n + 8.0 * recs,     # compact array in, CSR out
        "lr_both_kernel": 8.0 * m + 16.0 * n + 8.0 * recs,   # compact array in, leftmost + CSR out
    }
    del rho
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


def ceilings(dev, reps=5):
    """What the memory system sustains for the hot path's access patterns
    (paper_1501_06663_amd/csrc/probe.hip): a streaming copy, and random 8-byte
    gathers / scatters over tables the size of the 16M workload's text (16 MiB)
    and neighbour-pair array (128 MiB)."""
    import ctypes as C
    import torch
    from paper_1501_06663_amd import build as B
    lib = C.CDLL(B.PROBE_LIB)
    for f in (lib.probe_copy, lib.probe_gather, lib.probe_scatter):
        f.restype = C.c_int
    lib.probe_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    lib.probe_gather.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]
    lib.probe_scatter.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p]
    st = torch.cuda.current_stream().cuda_stream

    def clock(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    out = {}
    nbytes = 1 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    sec = clock(lambda: lib.probe_copy(a.data_ptr(), b.data_ptr(), nbytes // 16, st))
    out["copy_GBps"] = round(2 * nbytes / sec / 1e9, 1)
    del a, b
    rng = np.random.default_rng(0)
    n = 1 << 24
    vals = torch.empty(n, dtype=torch.int64, device=dev)
    for name, tbytes in (("16MiB", 16 << 20), ("128MiB", 128 << 20)):
        tn = tbytes // 8
        table = torch.zeros(tn, dtype=torch.int64, device=dev)
        idx = torch.from_numpy(rng.integers(0, tn, n).astype(np.uint32)).to(dev)
        sec = clock(lambda: lib.probe_gather(idx.data_ptr(), table.data_ptr(), tn, vals.data_ptr(), n, st))
        out["gather8_%s_Gaccess_per_s" % name] = round(n / sec / 1e9, 2)
        perm = torch.from_numpy(rng.permutation(tn)[:n].astype(np.uint32)).to(dev)
        m = min(n, tn)
        sec = clock(lambda: lib.probe_scatter(perm.data_ptr(), vals.data_ptr(), table.data_ptr(), tn, m, st))
        out["scatter8_%s_Gaccess_per_s" % name] = round(m / sec / 1e9, 2)
        del table, idx, perm
    return out


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_traffic_%s.md")  # per workload
DEVICE_SOURCE = os.path.join(ROOT, "paper_1501_06663_amd", "csrc", "lrq_device.hip")


def pmc_traffic(kernel, workload="dna16m"):
    """HBM bytes per launch of `kernel` as rocprofv3's FETCH_SIZE + WRITE_SIZE
    counters read them (scaled by what they read for a copy kernel of known
    size), from the committed counter summary of this workload.  None when that
    summary does not cover the kernel, or when the kernel source has changed
    since the counters were taken (the summary records the source's SHA-256)."""
    import hashlib
    try:
        with open(TRAFFIC_SUMMARY % workload) as f:
            lines = [l for l in f if l.startswith("traffic-json: ")]
        rec = json.loads(lines[-1][len("traffic-json: "):])
        with open(DEVICE_SOURCE, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_sha256") != digest:
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def cpu_baseline(text, min_seconds):
    """The oracle on the benchmark's own string: its suffix sort (untimed, the
    GPU step starts from a resident SA too), then the step's span -- Rank, Kasai
    LCP, Lemma-1 lengths, compaction, Algorithm 1 and Algorithm 3 walks --
    repeated until min_seconds of CPU time have passed."""
    import oracle
    threads = oracle.set_threads(min(os.cpu_count() or 1, 16))
    n = len(text)
    t0 = time.perf_counter()
    sa = oracle.suffix_array(text)
    sa_s = time.perf_counter() - t0
    stages = {"rank": 0.0, "lcp_kasai": 0.0, "lemma1_lengths": 0.0, "compaction": 0.0,
              "alg1_leftmost_raw": 0.0, "alg3_all_raw": 0.0}
    reps, spent = 0, 0.0
    while reps == 0 or spent < min_seconds:
        t = [time.perf_counter()]
        rk = oracle.rank(sa)
        t.append(time.perf_counter())
        lc = oracle.lcp(text, sa, rk)
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
        spent += t[-1] - t[0]
        reps += 1
    # the same span once more on one thread (the per-position loops are the
    # oracle's only parallel parts), for the single-core figure
    oracle.set_threads(1)
    t1 = time.perf_counter()
    rk = oracle.rank(sa)
    lc = oracle.lcp(text, sa, rk)
    L = oracle.llr_lengths(rk, lc)
    oracle.compact(L)
    oracle.lr_leftmost_raw(L)
    oracle.lr_all_raw(L)
    one_s = time.perf_counter() - t1
    oracle.set_threads(threads)
    return {"value": round(n * reps / spent, 1), "unit": "positions/s", "cores": threads,
            "single_thread_positions_per_s": round(n / one_s, 1),
            "kind": "oracle",
            "sample": ("the benchmark's own DNA-like string (%d characters); timed span = Rank, Kasai "
                       "LCP, Lemma-1 lengths, compaction, Algorithm 1 and Algorithm 3 walks (the GPU "
                       "step's span, from a resident SA), run %d times in %.2f s; the oracle's own "
                       "suffix sort took a further %.2f s, untimed" % (n, reps, spent, sa_s)),
            "stage_s_per_rep": {k: round(v / reps, 4) for k, v in stages.items()}}


def measure(plain, steps, warmup, tune):
    """Autotune (optionally), then time `steps` steps of the hot path on one
    prepared string or batch: positions/s, per-kernel table, spans, and the
    roofline row of the kernel that takes the most time per step."""
    from paper_1501_06663_amd import lrq
    n = plain.n
    m = plain.count.item()
    log("n %d: compact entries %d, all-mode records %d" % (n, m, plain.cap))
    tuned = None
    if tune:
        from paper_1501_06663_amd import autotune
        t = autotune.tune(plain.step, key=autotune.size_key(n, plain.nseg), reps=3, use_cache=False)
        tuned = {"chosen": t["tuning"], "trials": t["trials"]}
        log("tuning %s (%.3f ms)" % (t["tuning"], t["seconds"] * 1e3))
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
    both = dict(kt)
    both.update(modes)
    # build = rank scatter .. filter; the scans; and filter + scan (the paper's
    # timed span: LLR array and walks from a resident LCP)
    spans = {}
    for name, calls in (("build", [c for c in kt if not c.startswith("lr_")]),
                        ("both_scan", ("lr_both_kernel",)),
                        ("leftmost_scan", ("lr_leftmost_kernel",)),
                        ("all_scan", ("lr_all_kernel",)),
                        ("filter_plus_leftmost", ("llr_filter_kernel", "lr_leftmost_kernel")),
                        ("filter_plus_all", ("llr_filter_kernel", "lr_all_kernel"))):
        if not all(c in both for c in calls):
            continue
        ms = sum(both[c]["ms_per_step"] for c in calls)
        spans[name] = {"ms": round(ms, 4), "positions_per_s": round(n / (ms * 1e-3), 1)}
    return {"sec": sec, "positions_per_s": round(n / sec, 1), "ms_per_step": round(sec * 1e3, 4),
            "kernels": kt, "single_mode_kernels": modes, "spans": spans, "roofline": roofline,
            "tuning": tuned,
            "compact_entries": int(m), "all_mode_records": int(plain.cap)}


def raw_leg(plain, steps, warmup):
    """The raw-LLR path (Plain.step_raw) on the same string or batch: step
    time, per-kernel breakdown, and whether its answers equal the compact
    path's, element by element."""
    import torch
    from paper_1501_06663_amd import lrq
    n = plain.n
    plain.step()
    torch.cuda.synchronize()
    ref = (plain.out[:n].clone(), plain.offs.clone(), plain.recs[:plain.cap].clone())
    lrq.read_errors(plain.scratch)  # clears the error word
    sec, _ = timed(plain.step_raw, steps, warmup)
    bsteps = max(3, min(steps, 10))
    _, kern = timed(plain.step_raw, bsteps, 1, record_kernels=True)
    errs = lrq.read_errors(plain.scratch)
    same = (errs == 0 and torch.equal(plain.out[:n], ref[0]) and torch.equal(plain.offs, ref[1])
            and torch.equal(plain.recs[:plain.cap], ref[2]))
    kt = kernel_table(kern, bsteps, n, plain.count.item(), plain.cap)
    # Lemma 4's alpha: the mean LLR length, the mean number of LLRs covering a
    # position, hence the mean walk
    alpha = float(plain.L[:n].double().mean().item()) if n else 0.0
    log("raw path: step %.3f ms (%s), alpha %.2f, same answers as the compact path: %s"
        % (sec * 1e3, "errors %d" % errs if errs else "no errors", alpha, same))
    return {"ms_per_step": round(sec * 1e3, 4), "positions_per_s": round(n / sec, 1),
            "alpha_mean_llr_length": round(alpha, 3),
            "compact_entries_per_position": round(plain.count.item() / max(n, 1), 4),
            "kernels_us": {k: v["avg_us"] for k, v in kt.items()},
            "same_answers_as_compact": bool(same), "error_bits": int(errs)}


def other_configs(args, dev):
    """The step on the other single-string workloads: the 2^16 uniform string,
    the 2^22 Fibonacci word (longest LCPs), the 2^26 Markov text (arrays well
    beyond the 256 MiB last-level cache)."""
    import torch
    from paper_1501_06663_amd import lrq, workloads
    legs = {}
    for name, desc, make in (
            ("uniform_64k", "i.i.d. uniform ACGT, n=65,536, seed 0", workloads.config1),
            ("fibonacci_4m", "Fibonacci word, n=2^22", workloads.config3a),
            ("markov_64m", "order-2 Markov text over 96 symbols, Zipf(1.1), n=2^26, seed 0",
             workloads.config3b)):
        t0 = time.perf_counter()
        text = make()
        sa = lrq.build_sa_host(text)
        log("%s: n %d, generate + host SA %.2f s" % (name, len(text), time.perf_counter() - t0))
        plain = Plain(text, sa, None, dev)
        meas = measure(plain, max(3, args.steps // 2), args.warmup, not args.no_tune)
        del meas["sec"]
        if name != "fibonacci_4m":  # its LLRs are ~10^6 long: the raw walks do not apply
            meas["raw_path"] = raw_leg(plain, max(3, args.steps // 2), args.warmup)
        meas["workload"] = desc
        legs[name] = meas
        del plain, text, sa
        torch.cuda.empty_cache()
    return legs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="override the string length (testing)")
    ap.add_argument("--workload", choices=("dna16m", "markov64m"), default="dna16m",
                    help="the headline string: DNA-like 2^24 (default) or Markov text 2^26")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU time the oracle baseline repeats its span for")
    ap.add_argument("--plain-only", action="store_true", help="only the plain step (profiling runs)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the uniform / Fibonacci / Markov single-string legs")
    ap.add_argument("--no-tune", action="store_true", help="keep the default kernel shapes")
    ap.add_argument("--serving-strings", type=int, default=96)
    ap.add_argument("--serving-rates", type=str, default="25,50,100",
                    help="Poisson arrival rates (strings/s) of the serving leg")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of known "
                         "traffic, to calibrate profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (--gpus %d "
              "is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1501_06663_amd import lrq, workloads
    dev = torch.device("cuda:0")

    if args.copy_mib:
        # one launch of the probe library's streaming copy_kernel: a kernel whose
        # HBM traffic is known exactly (copy_mib MiB read, copy_mib MiB written)
        import ctypes as C
        from paper_1501_06663_amd import build as B
        plib = C.CDLL(B.PROBE_LIB)
        plib.probe_copy.restype = C.c_int
        plib.probe_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        src = torch.ones(args.copy_mib << 18, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        rc = plib.probe_copy(src.data_ptr(), dst.data_ptr(), (args.copy_mib << 20) // 16,
                             torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        if rc != 0:
            raise SystemExit("probe_copy failed: %d" % rc)
        log("calibration copy_kernel: %d MiB read + %d MiB written" % (args.copy_mib, args.copy_mib))
        del src, dst

    if args.workload == "markov64m":
        n = args.n or workloads.C3B_N
        log("generating Markov text n=%d" % n)
        text = workloads.markov_text(n, 0)
        wdesc = ("plain order-2 Markov text over 96 printable symbols with Zipf(1.1) marginals, "
                 "n=%d, seed 0" % n)
    else:
        n = args.n or workloads.C2_N
        log("generating DNA-like n=%d" % n)
        text = workloads.dna_like(n, 0)
        wdesc = ("plain DNA-like string, n=%d, P(ACGT)=.3/.2/.2/.3, %d planted mutated copies "
                 "(log-uniform 50-5000), seed 0" % (n, int(round(2000 * n / 2 ** 24))))
    t0 = time.perf_counter()
    sa = lrq.build_sa_host(text)
    sa_s = time.perf_counter() - t0
    log("host SA %.2f s" % sa_s)
    plain = Plain(text, sa, None, dev)
    meas = measure(plain, args.steps, args.warmup, not args.no_tune)
    sec, kt, m = meas["sec"], meas["kernels"], meas["compact_entries"]
    value = n / sec
    # end to end: host SA, pageable host-to-device copies of text and SA, one step
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain.text.copy_(torch.from_numpy(text))
    plain.sa.copy_(torch.from_numpy(sa))
    torch.cuda.synchronize()
    h2d_s = time.perf_counter() - t0
    e2e_s = sa_s + h2d_s + sec
    # end to end with the suffix array built on the device: text copy, SA, one step
    sa_work = torch.empty(lrq.sa_work_bytes(n, 1), dtype=torch.uint8, device=dev)
    dsa = []
    for rep in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain.text.copy_(torch.from_numpy(text))
        t1 = time.perf_counter()
        lrq.build_sa(plain.text, n, None, 1, plain.sa, sa_work)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        plain.step()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if rep:  # the first repetition warms up
            dsa.append((t1 - t0, t2 - t1, t3 - t2, t3 - t0))
    if lrq.read_errors(plain.scratch):
        raise SystemExit("device error bits after the device-SA runs")
    if not np.array_equal(plain.sa.cpu().numpy(), sa):
        raise SystemExit("device SA differs from the host SA")
    del sa_work
    best = min(dsa, key=lambda x: x[3])
    log("device SA %.2f ms; end to end %.2f ms" % (best[1] * 1e3, best[3] * 1e3))
    raw = raw_leg(plain, args.steps, args.warmup)
    roofline = dict(meas["roofline"])
    roofline["traffic"] = pmc_traffic(roofline["kernel"], args.workload)
    for k, row in list(kt.items()) + list(meas["single_mode_kernels"].items()):
        row["traffic"] = pmc_traffic(k, args.workload)  # HBM-side bytes per launch, profiled
    spans = meas["spans"]
    tuned = meas["tuning"]

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "positions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wdesc,
                   "span": "rank scatter + text-order LCP + LLR filter + one scan giving the leftmost "
                           "LR and all LRs of every position; text and SA resident in HBM",
                   "compact_entries": int(m), "all_mode_records": int(meas["all_mode_records"])},
        "roofline": roofline,
        "kernels": kt,
        "single_mode_kernels": meas["single_mode_kernels"],
        "spans": spans,
        "host_sa_s": round(sa_s, 3),
        "e2e": {"host_sa_s": round(sa_s, 3), "h2d_ms": round(h2d_s * 1e3, 3),
                "step_ms": round(sec * 1e3, 4), "positions_per_s": round(n / e2e_s, 1)},
        "e2e_device_sa": {"text_h2d_ms": round(best[0] * 1e3, 3), "device_sa_ms": round(best[1] * 1e3, 3),
                          "step_ms": round(best[2] * 1e3, 3), "total_ms": round(best[3] * 1e3, 3),
                          "positions_per_s": round(n / best[3], 1)},
        "tuning": tuned,
        "raw_path": raw,
    }
    del plain
    torch.cuda.empty_cache()
    if not args.plain_only and not args.no_configs:
        result["other_configs"] = other_configs(args, dev)
    if not args.plain_only:
        result["ceilings"] = ceilings(dev)
        log("ceilings %s" % result["ceilings"])
        # the random-access kernels against the probes of their own access
        # pattern: one random 8-byte write per position in the rank scatter
        rs = kt.get("rank_scatter_kernel")
        probe = result["ceilings"].get("scatter8_128MiB_Gaccess_per_s")
        if rs and probe:
            rate = n / (rs["avg_us"] * 1e-6) / 1e9
            result["random_access"] = {"rank_scatter_kernel": {
                "random_8B_writes_G_per_s": round(rate, 2),
                "scatter_probe_128MiB_G_per_s": probe,
                "frac_of_probe": round(rate / probe, 3)}}

    if not args.no_batched and not args.plain_only:
        text4, off4 = workloads.config4()
        t0 = time.perf_counter()
        sa4 = lrq.build_sa_host_batch(text4, off4)
        log("batch: %d strings, %d chars, host SA %.2f s" % (len(off4) - 1, len(text4), time.perf_counter() - t0))
        bat = Plain(text4, sa4, off4, dev)
        btuned = None
        if not args.no_tune:
            from paper_1501_06663_amd import autotune
            btuned = autotune.tune(bat.step, key=autotune.size_key(len(text4), len(off4) - 1), reps=2,
                                   use_cache=False)
            log("batched tuning %s" % btuned["tuning"])
        bsec, _ = timed(bat.step, max(2, args.steps // 2), 1)
        # the same step captured once in a HIP graph and replayed
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            bat.step()
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            bat.step()
        gsec, _ = timed(graph.replay, max(2, args.steps // 2), 1)
        del graph, bat
        torch.cuda.empty_cache()
        singles = [Plain(text4[off4[b]:off4[b + 1]].copy(), sa4[off4[b]:off4[b + 1]].copy(), None, dev)
                   for b in range(len(off4) - 1)]

        def one_per_launch():
            for p in singles:
                p.step()
        ssec, _ = timed(one_per_launch, 2, 1)
        del singles
        torch.cuda.empty_cache()
        tot4 = int(off4[-1])
        result["batched"] = {
            "workload": "512 DNA-like strings, lengths log-uniform in [2^10, 2^20], %d chars total, seed 0" % tot4,
            "batched_positions_per_s": round(tot4 / bsec, 1), "batched_ms": round(bsec * 1e3, 3),
            "batched_graph_positions_per_s": round(tot4 / gsec, 1),
            "batched_graph_ms": round(gsec * 1e3, 3),
            "one_string_per_launch_positions_per_s": round(tot4 / ssec, 1),
            "one_string_per_launch_ms": round(ssec * 1e3, 3),
            "speedup": round(ssec / bsec, 3),
            "tuning": None if btuned is None else btuned["tuning"]}
        log("batched %.3f ms vs one-per-launch %.3f ms" % (bsec * 1e3, ssec * 1e3))

    if not args.no_serving and not args.plain_only:
        from paper_1501_06663_amd import serving
        ex = serving.GpuExecutor(sa_threads=min(os.cpu_count() or 1, 16))
        legs = []
        for rate in [float(x) for x in args.serving_rates.split(",") if x]:
            trace = list(workloads.serving_trace(rate, args.serving_strings, seed=0))
            log("serving: %d strings at %.0f/s (%d chars, %d query batches)" % (
                len(trace), rate, sum(len(r.text) for r in trace), sum(len(r.batches) for r in trace)))
            rep = serving.Server(ex, budget_bytes=32 << 30).run(trace, keep_results=False)
            summ = rep.summary()
            summ["arrival_rate_strings_per_s"] = rate
            legs.append(summ)
            log("  p50 %.2f ms p99 %.2f ms, %.3e positions/s" % (
                summ["latency_p50_ms"], summ["latency_p99_ms"], summ["positions_per_s"]))
        if ex.errors():
            raise SystemExit("serving: device error bits")
        result["served"] = {
            "workload": "Poisson arrivals of DNA-like or protein-like strings, lengths log-uniform "
                        "in [1e4, 4e6]; 1-64 query batches each of 1e3-1e5 uniform positions, "
                        "exponential gaps of mean 2 ms; leftmost mode; 32 GiB budget; seed 0",
            "legs": legs}

    if not args.no_cpu and not args.plain_only:
        log("cpu baseline (oracle) on the %d-char string, >= %.0f s" % (n, args.cpu_seconds))
        result["cpu_baseline"] = cpu_baseline(text, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
