"""The raw-LLR path (lrq_llr_lengths, lrq_lr_leftmost_raw, lrq_lr_all_raw:
Algorithms 1 and 3 over the raw LLR array of Section 4.1) against the
oracle's Algorithms 1 and 3, element by element, and at full size against the
oracle's digests.

The GPU side runs rank scatter -> PLCP -> Lemma-1 lengths -> raw walks
through the C ABI; the oracle runs its own suffix sort, Kasai LCP, Lemma 1 and
walks.  The two share only the input bytes."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from gpu_common import say
from paper_1501_06663_amd import workloads

pytestmark = pytest.mark.gpu


def gpu_raw(text_np, seg_off_np=None, max_walk=0, capacity=None):
    """Leftmost records, CSR offsets and records, and the device error word."""
    import torch
    from paper_1501_06663_amd import lrq
    dev = torch.device("cuda:0")
    text_np = np.ascontiguousarray(text_np, dtype=np.uint8)
    total = len(text_np)
    if seg_off_np is None:
        sa_np = lrq.build_sa_host(text_np) if total else np.zeros(0, np.int32)
        seg, nseg = None, 1
    else:
        seg_off_np = np.ascontiguousarray(seg_off_np, dtype=np.int64)
        sa_np = lrq.build_sa_host_batch(text_np, seg_off_np)
        seg = torch.from_numpy(seg_off_np).to(dev)
        nseg = len(seg_off_np) - 1
    t = max(total, 1)
    text = torch.from_numpy(np.concatenate([text_np, np.zeros(8, np.uint8)])).to(dev)
    sa = torch.from_numpy(np.concatenate([sa_np, np.zeros(1, np.int32)])).to(dev)
    scratch = torch.zeros(lrq.scratch_bytes(total, nseg), dtype=torch.uint8, device=dev)
    work = torch.full((2 * t + 4,), -7, dtype=torch.int32, device=dev)
    L = torch.full((t + 2,), -7, dtype=torch.int32, device=dev)
    out = torch.full((t, 2), -7, dtype=torch.int32, device=dev)
    out_both = torch.full((t, 2), -7, dtype=torch.int32, device=dev)
    offsets = torch.full((t + 1,), -7, dtype=torch.int64, device=dev)
    if total:
        lrq.rank_scatter(sa, total, seg, nseg, work, None, scratch)
        lrq.plcp(text, total, seg, nseg, work, scratch)
    lrq.llr_lengths(work, total, L)
    lrq.lr_leftmost_raw(L, total, seg, nseg, out, scratch, max_walk=max_walk)
    cap = capacity if capacity is not None else 4 * t + 16
    recs = torch.full((max(cap, 1), 2), -7, dtype=torch.int32, device=dev)
    try:
        n_rec = lrq.lr_all_raw(L, total, seg, nseg, offsets, recs, cap, scratch, max_walk=max_walk,
                               out=out_both)
    except lrq.LrqError as e:
        if e.status != -3:  # LRQ_ENOSPC
            raise
        n_rec = None
    errs = lrq.read_errors(scratch)
    torch.cuda.synchronize()
    res = {"L": L[:total].cpu().numpy(), "leftmost": out[:total].cpu().numpy(),
           "leftmost_both": out_both[:total].cpu().numpy(),
           "offsets": offsets[: total + 1].cpu().numpy(), "errors": errs, "n_rec": n_rec}
    if n_rec is not None:
        res["recs"] = recs[:n_rec].cpu().numpy()
    return res


def check(tag, text_np, seg_off_np=None):
    say("case: raw", tag, "n=%d" % len(text_np))
    got = gpu_raw(text_np, seg_off_np)
    if seg_off_np is None:
        want = oracle.pipeline(text_np, sa_method="doubling")
    else:
        want = oracle.pipeline_batch(text_np, seg_off_np, sa_method="doubling")
    assert got["errors"] == 0, tag
    np.testing.assert_array_equal(got["L"], want["L"], err_msg=tag + ": Lemma-1 lengths")
    np.testing.assert_array_equal(got["leftmost"], want["leftmost"], err_msg=tag + ": leftmost")
    np.testing.assert_array_equal(got["leftmost_both"], want["leftmost"],
                                  err_msg=tag + ": leftmost from the all-mode walks")
    np.testing.assert_array_equal(got["offsets"], want["all_offsets"], err_msg=tag + ": offsets")
    np.testing.assert_array_equal(got["recs"], want["all_recs"], err_msg=tag + ": records")


def test_empty_and_tiny():
    got = gpu_raw(np.zeros(0, np.uint8))
    assert got["n_rec"] == 0 and got["offsets"].tolist() == [0]
    check("one character", np.frombuffer(b"a", np.uint8).copy())
    check("mississippi", np.frombuffer(b"mississippi", np.uint8).copy())


@pytest.mark.parametrize("n", [255, 256, 257, 5000])
@pytest.mark.parametrize("sigma", [2, 4, 20])
def test_random(n, sigma):
    rng = np.random.default_rng(11 * n + sigma)
    check("random n=%d sigma=%d" % (n, sigma), (rng.integers(0, sigma, n) + 97).astype(np.uint8))


def test_dna_like():
    check("dna-like 2^18", workloads.dna_like(1 << 18, 5))


def test_batch():
    rng = np.random.default_rng(4)
    lens = rng.integers(0, 700, 60)
    lens[5] = 0
    lens[17] = 1
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    text = (rng.integers(0, 3, int(off[-1])) + 97).astype(np.uint8)
    check("batch of 60", text, off)


def test_walk_bound():
    # a unary string: the LLRs covering the last positions number ~n, so the
    # walks pass any small bound, set LRQ_ERR_WALK and stop
    from paper_1501_06663_amd import lrq
    text = np.full(3000, ord("a"), np.uint8)
    got = gpu_raw(text, max_walk=100)
    assert got["errors"] & lrq.ERR_WALK
    # with a bound above the longest walk the answers are exact
    got = gpu_raw(text, max_walk=4000)
    want = oracle.pipeline(text, sa_method="doubling")
    assert got["errors"] == 0
    np.testing.assert_array_equal(got["leftmost"], want["leftmost"])
    np.testing.assert_array_equal(got["offsets"], want["all_offsets"])
    np.testing.assert_array_equal(got["recs"], want["all_recs"])


def test_capacity():
    rng = np.random.default_rng(9)
    text = (rng.integers(0, 2, 3000) + 97).astype(np.uint8)
    full = gpu_raw(text)
    assert full["n_rec"] > 10
    small = gpu_raw(text, capacity=10)
    assert small["n_rec"] is None  # LRQ_ENOSPC, with the offsets complete
    np.testing.assert_array_equal(small["offsets"], full["offsets"])


GOLD = os.path.join(os.path.dirname(__file__), "golden", "full_digests.json")
with open(GOLD) as f:
    DIGESTS = json.load(f)

INPUTS = {
    "c1": lambda: (workloads.config1(), None),
    "c2": lambda: (workloads.config2(), None),
    "c3b": lambda: (workloads.config3b(), None),
    "c4": lambda: workloads.config4(),
}


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.parametrize("name", sorted(INPUTS))
def test_full_size_raw_digests(name):
    """The full-size workloads whose repeats are short (the Fibonacci word's
    are not: see test_fibonacci_walk_bound)."""
    import torch
    from paper_1501_06663_amd import lrq
    want = DIGESTS[name]
    text_np, seg_np = INPUTS[name]()
    say("case: raw full-size", name, "n=%d" % len(text_np))
    assert sha(text_np) == want["text"]
    dev = torch.device("cuda:0")
    sa_np = lrq.build_sa_host(text_np) if seg_np is None else lrq.build_sa_host_batch(text_np, seg_np)
    seg = None if seg_np is None else torch.from_numpy(seg_np).to(dev)
    idx = lrq.Index(torch.from_numpy(text_np).to(dev), torch.from_numpy(sa_np).to(dev), seg,
                    keep_L=True)
    n = idx.total
    out = torch.empty((n, 2), dtype=torch.int32, device=dev)
    lrq.lr_leftmost_raw(idx.L, n, idx.seg_off, idx.nseg, out, idx.scratch)
    assert sha(out.cpu().numpy()) == want["leftmost"], "leftmost records"
    offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
    recs = torch.empty((want["all_total"], 2), dtype=torch.int32, device=dev)
    tot = lrq.lr_all_raw(idx.L, n, idx.seg_off, idx.nseg, offsets, recs, want["all_total"],
                         idx.scratch)
    assert tot == want["all_total"]
    assert sha(offsets.cpu().numpy()) == want["all_offsets"], "all-mode offsets"
    assert sha(recs.cpu().numpy()) == want["all_recs"], "all-mode records"
    assert idx.errors() == 0


def test_fibonacci_walk_bound():
    """The Fibonacci word's LLRs are about a million characters long: the raw
    walks hit their bound and say so, instead of running for hours."""
    import torch
    from paper_1501_06663_amd import lrq
    text_np = workloads.config3a()
    say("case: raw fibonacci bound", "n=%d" % len(text_np))
    dev = torch.device("cuda:0")
    idx = lrq.Index(torch.from_numpy(text_np).to(dev),
                    torch.from_numpy(lrq.build_sa_host(text_np)).to(dev), None, keep_L=True)
    out = torch.empty((idx.total, 2), dtype=torch.int32, device=dev)
    lrq.lr_leftmost_raw(idx.L, idx.total, None, 1, out, idx.scratch)
    assert idx.errors() & lrq.ERR_WALK


def test_llr_past_its_string_is_reported():
    """An L value that runs past its string sets LRQ_ERR_SA; the walk stops
    there and nothing is read or written out of bounds."""
    import torch
    from paper_1501_06663_amd import lrq
    dev = torch.device("cuda:0")
    n = 1000
    L = torch.zeros(n + 2, dtype=torch.int32, device=dev)
    L[n - 2] = 100
    out = torch.full((n, 2), -7, dtype=torch.int32, device=dev)
    scratch = torch.zeros(lrq.scratch_bytes(n, 1), dtype=torch.uint8, device=dev)
    lrq.lr_leftmost_raw(L, n, None, 1, out, scratch)
    assert lrq.read_errors(scratch) & lrq.ERR_SA
    o = out.cpu().numpy()
    assert (o[: n - 2] == np.array([-1, 0])).all()  # untouched by the bad entry
