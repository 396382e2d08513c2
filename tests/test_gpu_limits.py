"""The edges of the 32-bit calls' range, on the GPU.

  * One string of LRQ_MAX_TOTAL = 2^31 - 2 characters, a^n, through the
    32-bit calls: the largest input they accept.  Its answers have the closed
    form that the oracle's pins tie to brute force (tests/test_oracle_pins.py):
    with SA[r] = n-1-r, L[i] = max(n-1-i, n-i), the compact array is
    (0, n-1), (1, n-1), the leftmost LR of k is (0, n-1) for k < n-1 and
    (1, n-1) at k = n-1, and all mode gives 2n - 2 records, more than 2^31.
    Outputs are checked at sampled positions, including the last ones, where
    an int32 sum of a position and a length would overflow.
  * A batch of 60,000 strings of 0 to 12 characters over two letters, plus a
    few longer ones, compared element by element with the oracle at every
    stage (many segment boundaries inside every tile and LCP block)."""
import numpy as np
import pytest

from gpu_common import compare, gpu_stages, oracle_view, say
from paper_1501_06663_amd import workloads

pytestmark = pytest.mark.gpu


def test_int32_at_the_size_limit():
    import torch
    from paper_1501_06663_amd import lrq
    n = lrq.MAX_TOTAL
    say("case: a^n with n = %d (the 32-bit limit) on the 32-bit path" % n)
    dev = torch.device("cuda:0")
    text = torch.full((n,), 97, dtype=torch.uint8, device=dev)
    sa = torch.arange(n - 1, -1, -1, dtype=torch.int32, device=dev)  # shorter suffix first
    idx = lrq.Index(text, sa, build=False)
    assert not idx.wide
    del sa
    idx.build()
    torch.cuda.synchronize()
    say("  built; checking")
    samples = np.unique(np.concatenate([
        [0, 1, 2, 3, n // 2, n - 4, n - 3, n - 2, n - 1],
        np.random.default_rng(1).integers(0, n, 4000)])).astype(np.int64)
    st = torch.from_numpy(samples).to(dev)
    # the build hands Lemma 1's L = max(PLCP, NLCP) to its filter through the
    # first half of the work buffer: n - i for i >= 1, n - 1 at 0
    L = idx.work[:n][st].cpu().numpy().astype(np.int64)
    assert np.array_equal(L, np.where(samples >= 1, n - samples, n - 1)), "L"
    assert idx.count == 2
    assert idx.compact().cpu().tolist() == [[0, n - 1], [1, n - 1]]
    left = idx.leftmost()
    got = left[st].cpu().numpy()
    want = np.stack([np.where(samples < n - 1, 0, 1), np.full(len(samples), n - 1)], axis=1)
    assert np.array_equal(got, want), "leftmost"
    del left
    torch.cuda.empty_cache()
    assert idx.all_count() == 2 * n - 2
    lq, offs, recs = idx.query(st.to(torch.int32), mode=lrq.ALL)
    assert np.array_equal(lq.cpu().numpy(), want)
    offs, recs = offs.cpu().numpy(), recs.cpu().numpy()
    for q, k in enumerate(samples):
        lst = recs[offs[q]:offs[q + 1]].tolist()
        want_k = [[0, n - 1]] if k == 0 else ([[1, n - 1]] if k == n - 1 else [[0, n - 1], [1, n - 1]])
        assert lst == want_k, (k, lst)
    assert idx.errors() == 0


def test_many_tiny_strings():
    rng = np.random.default_rng(31)
    lens = rng.integers(0, 13, 60000)
    lens[rng.integers(0, len(lens), 5)] = [3000, 5000, 700, 4096, 4097]
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    text = (rng.integers(0, 2, int(off[-1])) + 97).astype(np.uint8)
    say("case: batch of %d strings of 0-12 characters (plus 5 longer), %d characters"
        % (len(lens), len(text)))
    compare(gpu_stages(text, off), oracle_view(text, off), tag="tiny strings")
