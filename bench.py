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
        # size the all-mode output once; every step then runs the one-pass kernel
        self.build()
        self.cap = lrq.lr_all_count(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.scratch)
        self.recs = torch.empty((max(self.cap, 1), 2), dtype=torch.int32, device=dev)

    def build(self):
        l = self.lrq
        l.rank_scatter(self.sa, self.n, self.seg, self.nseg, self.work, None, self.scratch)
        l.plcp(self.text, self.n, self.seg, self.nseg, self.work, self.scratch)
        l.llr_filter(self.work, self.n, self.seg, self.nseg, self.llrc, self.count, self.blocks, None,
                     self.scratch)

    def step(self):
        l = self.lrq
        self.build()
        l.lr_leftmost(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.out, self.scratch)
        l.lr_all(self.llrc, self.blocks, self.n, self.seg, self.nseg, self.offs, self.recs, self.cap,
                 self.scratch, want_total=False)


def timed(fn, steps, warmup, record_kernels=False):
    import torch
    from paper_1501_06663_amd import lrq
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if record_kernels:
        lrq.timing_start(1 << 20)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = lrq.timing_collect() if record_kernels else []
    return (t1 - t0) / steps, kern


def algorithmic_bytes(name, n, m, recs):
    """Bytes per launch each kernel must move, from the data it reads and writes
    (int32 positions; see the design doc for the derivation)."""
    rho = m / n
    table = {
        "rank_scatter_kernel": 12.0 * n,                     # SA 4 in, neighbour pair 8 out
        "plcp_chunks_kernel": 19.0 * n,                      # pairs 8 in + 8 out, text 1, two compared chars
        "llr_filter_kernel": 8.0 * n + 8.0 * m,              # LCP pairs in, compact array out
        "lr_leftmost_kernel": 8.0 * m + 8.0 * n,             # compact array in, one record per position
        "lr_all_kernel": 8.0 * m + 8.0 * n + 8.0 * recs,     # compact array in, CSR out
    }
    del rho
    return table.get(name)


def kernel_table(kern, steps, n, m, recs):
    agg = {}
    for name, ms in kern:
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


def cpu_baseline(n_sample):
    import oracle
    from paper_1501_06663_amd import workloads
    threads = oracle.set_threads(min(os.cpu_count() or 1, 16))
    s = workloads.dna_like(n_sample, 0)
    t0 = time.perf_counter()
    sa = oracle.suffix_array(s)
    t1 = time.perf_counter()
    rk = oracle.rank(sa)
    lc = oracle.lcp(s, sa, rk)
    L = oracle.llr_lengths(rk, lc)
    oracle.compact(L)
    oracle.lr_leftmost_raw(L)
    oracle.lr_all_raw(L)
    t2 = time.perf_counter()
    return {"value": round(n_sample / (t2 - t1), 1), "unit": "positions/s", "cores": threads,
            "kind": "oracle",
            "sample": ("DNA-like string of %d characters from the same generator (planted-copy density "
                       "of the 2^24 workload); timed span = Rank, Kasai LCP, Lemma-1 lengths, compaction, "
                       "Algorithm 1 and Algorithm 3 walks (the GPU step's span, from a resident SA); "
                       "%.2f s; the oracle's own suffix sort took a further %.2f s, untimed"
                       % (n_sample, t2 - t1, t1 - t0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="override the string length (testing)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 22)
    ap.add_argument("--plain-only", action="store_true", help="only the plain step (profiling runs)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of known "
                         "traffic, to calibrate profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (--gpus %d "
              "is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1501_06663_amd import lrq, workloads
    dev = torch.device("cuda:0")

    if args.copy_mib:
        src = torch.ones(args.copy_mib << 18, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read + %d MiB written" % (args.copy_mib, args.copy_mib))
        del src, dst

    n = args.n or workloads.C2_N
    log("generating DNA-like n=%d" % n)
    text = workloads.dna_like(n, 0)
    t0 = time.perf_counter()
    sa = lrq.build_sa_host(text)
    sa_s = time.perf_counter() - t0
    log("host SA %.2f s" % sa_s)
    plain = Plain(text, sa, None, dev)
    m = plain.count.item()
    log("compact entries %d, all-mode records %d" % (m, plain.cap))
    sec, kern = timed(plain.step, args.steps, args.warmup, record_kernels=True)
    errs = lrq.read_errors(plain.scratch)
    if errs:
        raise SystemExit("device error bits %d" % errs)
    value = n / sec
    log("plain step %.3f ms  -> %.3e positions/s" % (sec * 1e3, value))
    kt = kernel_table(kern, args.steps, n, m, plain.cap)
    dom = max((r for r in kt.items() if "alg_bytes" in r[1]), key=lambda kv: kv[1]["ms_per_step"])
    dname, drow = dom
    roofline = {"bound": "hbm", "kernel": dname, "achieved": drow["achieved_GBps"],
                "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": drow["frac_of_hbm_peak"],
                "traffic": None}

    # Spans: Q = filter + scans from resident LCP pairs; build = rank+plcp+filter.
    spans = {}
    for name, calls in (("leftmost_Q", ("llr_filter_kernel", "lr_leftmost_kernel")),
                        ("all_Q", ("llr_filter_kernel", "lr_all_kernel"))):
        ms = sum(kt[c]["ms_per_step"] for c in calls if c in kt)
        spans[name] = {"ms": round(ms, 4), "positions_per_s": round(n / (ms * 1e-3), 1)}

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "positions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "plain DNA-like string, n=%d, P(ACGT)=.3/.2/.2/.3, %d planted mutated "
                               "copies (log-uniform 50-5000), seed 0" % (n, int(round(2000 * n / 2 ** 24))),
                   "span": "rank scatter + text-order LCP + LLR filter + leftmost LR + all LRs "
                           "(one pass); text and SA resident in HBM",
                   "compact_entries": int(m), "all_mode_records": int(plain.cap)},
        "roofline": roofline,
        "kernels": kt,
        "spans": spans,
        "host_sa_s": round(sa_s, 3),
    }
    del plain
    torch.cuda.empty_cache()

    if not args.no_batched and not args.plain_only:
        text4, off4 = workloads.config4()
        t0 = time.perf_counter()
        sa4 = lrq.build_sa_host_batch(text4, off4)
        log("batch: %d strings, %d chars, host SA %.2f s" % (len(off4) - 1, len(text4), time.perf_counter() - t0))
        bat = Plain(text4, sa4, off4, dev)
        bsec, _ = timed(bat.step, max(2, args.steps // 2), 1)
        del bat
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
            "one_string_per_launch_positions_per_s": round(tot4 / ssec, 1),
            "one_string_per_launch_ms": round(ssec * 1e3, 3),
            "speedup": round(ssec / bsec, 3)}
        log("batched %.3f ms vs one-per-launch %.3f ms" % (bsec * 1e3, ssec * 1e3))

    if not args.no_cpu and not args.plain_only:
        log("cpu baseline (oracle) on %d chars" % args.cpu_sample)
        result["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
