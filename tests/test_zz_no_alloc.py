"""lrq_query_multi_noalloc, the point-query call that takes no scratch buffer
(its error word and scan sums live in the library's own device array),
against lrq_query_multi on the same inputs, bit for bit, in both modes: two
calls in a row, the second with a smaller input, so that the array's leftover
contents from the first call cannot leak into the second."""
import numpy as np
import pytest

from gpu_common import say
from paper_1501_06663_amd import workloads

pytestmark = pytest.mark.gpu


def _index(dev, lrq, texts):
    import torch
    off = np.zeros(len(texts) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(t) for t in texts])
    text = np.concatenate(texts)
    idx = lrq.Index(torch.from_numpy(text).to(dev),
                    torch.from_numpy(lrq.build_sa_host_batch(text, off)).to(dev),
                    torch.from_numpy(off).to(dev))
    refs = [(idx.llrc.data_ptr(), idx.blocks.data_ptr(), int(off[-1]), int(off[b]),
             int(off[b + 1] - off[b])) for b in range(len(texts))]
    return idx, refs


def _queries(rng, lens, m, bad_at=None):
    sid = rng.integers(0, len(lens), m).astype(np.int32)
    pos = np.array([rng.integers(0, lens[s]) for s in sid], dtype=np.int32)
    if bad_at is not None:
        pos[bad_at] = -3                      # outside its string: (-1, 0) + LRQ_ERR_QUERY
    return sid, pos


def test_noalloc_equals_query_multi_twice():
    import torch
    from paper_1501_06663_amd import lrq
    dev = torch.device("cuda:0")
    texts = [workloads.dna_like(60000, 71), workloads.protein_like(40000, 72),
             workloads.markov_text(30000, 73), workloads.staircase_repeats(60, 300, 4000)]
    idx, refs = _index(dev, lrq, texts)
    refs_t = torch.tensor(refs, dtype=torch.int64, device=dev)
    lens = [len(t) for t in texts]
    rng = np.random.default_rng(5)
    for call, m in enumerate((50000, 7000)):            # the second call is smaller
        say("case: noalloc call %d, m=%d, both modes" % (call + 1, m))
        sid, pos = _queries(rng, lens, m, bad_at=17 if call == 0 else None)
        st, pt = torch.from_numpy(sid).to(dev), torch.from_numpy(pos).to(dev)
        scratch = torch.zeros(lrq.scratch_bytes(m), dtype=torch.uint8, device=dev)
        # leftmost
        want = torch.empty((m, 2), dtype=torch.int32, device=dev)
        lrq.query_multi(refs_t, len(refs), st, pt, m, want, scratch)
        want_err = lrq.read_errors(scratch)
        got = torch.full((m, 2), -7, dtype=torch.int32, device=dev)
        _, err = lrq.query_multi_noalloc(refs_t, len(refs), st, pt, m, got)
        assert torch.equal(got, want), "leftmost records, call %d" % (call + 1)
        assert err == want_err == (lrq.ERR_QUERY if call == 0 else 0)
        # all mode, with the leftmost records too
        woffs = torch.empty(m + 1, dtype=torch.int64, device=dev)
        wrecs = torch.empty((4 * m, 2), dtype=torch.int32, device=dev)
        wleft = torch.empty((m, 2), dtype=torch.int32, device=dev)
        wtot = lrq.query_multi(refs_t, len(refs), st, pt, m, wleft, scratch, mode=lrq.ALL,
                               offsets=woffs, recs=wrecs, capacity=4 * m)
        lrq.read_errors(scratch)
        goffs = torch.full((m + 1,), -7, dtype=torch.int64, device=dev)
        grecs = torch.full((4 * m, 2), -7, dtype=torch.int32, device=dev)
        gleft = torch.full((m, 2), -7, dtype=torch.int32, device=dev)
        gtot, err = lrq.query_multi_noalloc(refs_t, len(refs), st, pt, m, gleft, mode=lrq.ALL,
                                            offsets=goffs, recs=grecs, capacity=4 * m)
        assert gtot == wtot
        assert torch.equal(goffs, woffs), "offsets, call %d" % (call + 1)
        assert torch.equal(grecs[:gtot], wrecs[:wtot]), "records, call %d" % (call + 1)
        assert torch.equal(gleft, wleft), "all-mode leftmost records, call %d" % (call + 1)
        assert err == (lrq.ERR_QUERY if call == 0 else 0)
    # a record buffer that is too short: LRQ_ENOSPC with the total, nothing
    # written past the capacity, and the capacity bit in this call's errors
    cap = wtot // 2
    grecs = torch.full((cap + 4, 2), -7, dtype=torch.int32, device=dev)
    with pytest.raises(lrq.LrqError) as e:
        lrq.query_multi_noalloc(refs_t, len(refs), st, pt, m, None, mode=lrq.ALL, offsets=goffs,
                                recs=grecs, capacity=cap)
    assert e.value.status == -3
    assert torch.equal(goffs, woffs)
    assert torch.equal(grecs[:cap], wrecs[:cap]) and bool((grecs[cap:] == -7).all())
    _, err = lrq.query_multi_noalloc(refs_t, len(refs), st, pt, m, gleft)
    assert err == 0, "each call starts with a clear error word"
    assert idx.errors() == 0
