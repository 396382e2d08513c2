"""The batched hot path captured once in a HIP graph and replayed.

Every replay must equal the eager run.  Replays are interleaved with eager
work on the same buffers and with synchronisations, as graph-replay bugs
(stale counters, memset nodes) show up only on replays after the first."""
import numpy as np
import pytest

from gpu_common import say
from paper_1501_06663_amd import workloads

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager():
    import torch
    from paper_1501_06663_amd import lrq
    say("case: graph capture of the batched step (24 strings)")
    dev = torch.device("cuda:0")
    text_np, off_np = workloads.config4(seed=21, nseg=24, min_log2=8, max_log2=16)
    sa_np = lrq.build_sa_host_batch(text_np, off_np)
    n, nseg = len(text_np), len(off_np) - 1
    text = torch.from_numpy(text_np).to(dev)
    sa = torch.from_numpy(sa_np).to(dev)
    seg = torch.from_numpy(off_np).to(dev)
    work = torch.empty(2 * n, dtype=torch.int32, device=dev)
    llrc = torch.empty((n, 2), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    blocks = torch.zeros(lrq.block_entries(n), dtype=torch.int64, device=dev)
    out = torch.empty((n, 2), dtype=torch.int32, device=dev)
    offs = torch.empty(n + 1, dtype=torch.int64, device=dev)
    scratch = torch.zeros(lrq.scratch_bytes(n, nseg), dtype=torch.uint8, device=dev)

    def step(cap):
        lrq.index_build(text, sa, n, seg, nseg, work, llrc, count, blocks, None, scratch)
        lrq.lr_leftmost(llrc, blocks, n, seg, nseg, out, scratch)
        lrq.lr_all(llrc, blocks, n, seg, nseg, offs, recs, cap, scratch, want_total=False)

    lrq.index_build(text, sa, n, seg, nseg, work, llrc, count, blocks, None, scratch)
    cap = lrq.lr_all_count(llrc, blocks, n, seg, nseg, scratch)
    recs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
    step(cap)
    torch.cuda.synchronize()
    want = [t.clone() for t in (llrc[: int(count.item())], blocks, out, offs, recs)]

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step(cap)                      # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(cap)
    for rep in range(4):
        for t in (llrc, out, offs, recs):
            t.fill_(-5)                # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (llrc[: int(count.item())], blocks, out, offs, recs)
        for a, b in zip(got, want):
            assert torch.equal(a, b), "replay %d differs" % rep
    assert lrq.read_errors(scratch) == 0
