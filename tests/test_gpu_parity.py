"""Parity of the HIP path with the CPU oracle, element by element, at sizes
the oracle finishes in seconds.  Every stage is compared: Rank, the suffix
neighbours, text-order LCP pairs, Lemma-1 lengths, the compact LLR array,
leftmost LRs and the all-LR CSR lists.  Integer work: the bar is equality.

Cases span several tiles of every kernel and ragged tails (sizes around the
LLR tile of 4096, the PLCP block span of 4096 and the LR tile of 2048),
alphabets from 1 to 256 symbols, the long-repeat extremes (unary strings,
Fibonacci words) that exercise the seeded head levels of the LCP kernel, and
batches with empty, one-character and identical segments."""
import numpy as np
import pytest

from gpu_common import compare, gpu_stages, oracle_view, say
from paper_1501_06663_amd import workloads

pytestmark = pytest.mark.gpu


def run_case(tag, text, seg_off=None, walks="raw", sa_method="naive", modes=("leftmost", "all")):
    say("case:", tag, "n=%d" % len(text), "segments=%s" % (None if seg_off is None else len(seg_off) - 1))
    g = gpu_stages(text, seg_off, modes=modes)
    o = oracle_view(text, seg_off, walks=walks, sa_method=sa_method)
    compare(g, o, tag=tag)
    return g, o


@pytest.mark.parametrize("s", [b"a", b"ab", b"aa", b"mississippi", b"abcabcddbca", b"ababab",
                               b"abcaabcb", b"xyz", b"\x00\x00\xff\x00\xff"])
def test_paper_examples_and_tiny(s):
    run_case("tiny %r" % s, np.frombuffer(s, np.uint8))


@pytest.mark.parametrize("n", [2, 3, 15, 16, 17, 63, 64, 65, 255, 256, 257, 2047, 2048, 2049,
                               4095, 4096, 4097, 8191, 12289, 20000])
@pytest.mark.parametrize("sigma", [2, 4, 12, 96])
def test_sizes_around_tiles(n, sigma):
    rng = np.random.default_rng(n * 7 + sigma)
    run_case("random n=%d sigma=%d" % (n, sigma), (rng.integers(0, sigma, n) + 33).astype(np.uint8))


@pytest.mark.parametrize("sigma", [1, 256])
def test_alphabet_extremes(sigma):
    rng = np.random.default_rng(sigma)
    n = 9000
    text = rng.integers(0, sigma, n).astype(np.uint8) + (7 if sigma == 1 else 0)
    run_case("sigma=%d" % sigma, text, sa_method="doubling" if sigma == 1 else "naive",
             walks="window" if sigma == 1 else "raw")


@pytest.mark.parametrize("sigma", [3, 5, 16, 17])
def test_code_widths(sigma):
    """The LCP kernels read texts of at most 2, 4 or 16 distinct characters
    packed to 1, 2 or 4 bits; the boundaries of each width, with byte values
    spread over 0..255."""
    rng = np.random.default_rng(100 + sigma)
    values = np.sort(rng.choice(256, sigma, replace=False)).astype(np.uint8)
    base = values[rng.integers(0, sigma, 30000)]
    # a few long planted repeats, so that compares run past one word
    for q in range(5):
        a, b, m = rng.integers(0, 20000), rng.integers(0, 20000), 3000
        base[b:b + m] = base[a:a + m].copy()
    run_case("sigma=%d" % sigma, base)


def test_config1_full():
    run_case("config1 uniform n=65536", workloads.config1())


def test_dna_like_1m():
    run_case("dna-like n=2^20", workloads.dna_like(1 << 20, 0))


def test_markov_1m():
    run_case("markov n=2^20", workloads.markov_text(1 << 20, 0))


def test_protein_like_512k():
    run_case("protein-like n=2^19", workloads.protein_like(1 << 19, 1))


@pytest.mark.parametrize("n", [1 << 16, (1 << 18) + 5])
def test_fibonacci(n):
    run_case("fibonacci n=%d" % n, workloads.fibonacci_word(n), walks="window", sa_method="doubling")


@pytest.mark.parametrize("n", [5000, 70000])
def test_unary(n):
    run_case("unary n=%d" % n, np.full(n, 65, np.uint8), walks="window", sa_method="doubling")


def test_periodic_with_defects():
    base = np.frombuffer(b"acgtacgatt", np.uint8)
    text = np.tile(base, 6000).copy()
    text[::9973] = ord("n")
    run_case("periodic", text, walks="window")


@pytest.mark.parametrize("lr_tile", [1024, 2048, 4096])
def test_wide_windows(lr_tile):
    """Positions covered by more than 64 compact entries (the scan's tie mask
    holds 64) and tile starts covered by more than the 64 staged margin
    entries (the window is then read from global memory)."""
    from paper_1501_06663_amd import lrq
    text = workloads.staircase_repeats(150, 3996, 8192)
    lrq.set_tuning(lr_tile=lr_tile)
    try:
        run_case("staircase lr_tile=%d" % lr_tile, text)
        seg = workloads.staircase_repeats(120, 2000, 4500, seed=1)
        both = np.concatenate([seg, text, seg[:77]])
        off = np.array([0, len(seg), len(seg) + len(text), len(both)], np.int64)
        run_case("staircase batch lr_tile=%d" % lr_tile, both, off)
    finally:
        lrq.set_tuning()


def test_batch_mixed_segments():
    text, off = workloads.config4(seed=5, nseg=40, min_log2=0, max_log2=14)
    # append an empty segment, a 1-char one, and two identical segments
    twin = workloads.dna_like(3000, 99, 3)
    text = np.concatenate([text, np.array([71], np.uint8), twin, twin])
    off = np.concatenate([off, [off[-1], off[-1] + 1, off[-1] + 1 + 3000, off[-1] + 1 + 6000]])
    g, o = run_case("batch 44 segments", text, off)
    # the two identical segments give identical local answers
    a = slice(int(off[-3]), int(off[-2]))
    b = slice(int(off[-2]), int(off[-1]))
    assert np.array_equal(g["leftmost"][a], g["leftmost"][b])


def test_batch_segments_on_block_boundaries():
    # strings that start exactly at multiples of 4096 (the LCP walk's block, whose
    # keep summary then says "starts a string"), empty strings there too, and a
    # string that repeats its predecessor so that L at a block's first position
    # is large while the previous block ends inside another string
    a = workloads.dna_like(4096, 11)
    b = workloads.dna_like(4096, 12)
    text = np.concatenate([a, a, b, b[:100], workloads.dna_like(8192 - 100, 13), a])
    off = np.array([0, 4096, 8192, 8192, 12288, 12388, 20480, 20480, 24576], np.int64)
    assert off[-1] == len(text)
    run_case("batch on block boundaries", text, off)


def test_batch_tiny_segments():
    rng = np.random.default_rng(3)
    lens = rng.integers(0, 40, 300)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    text = (rng.integers(0, 3, int(off[-1])) + 97).astype(np.uint8)
    run_case("batch 300 tiny segments", text, off)


def test_empty_string():
    import torch
    from paper_1501_06663_amd import lrq
    say("case: empty string")
    dev = torch.device("cuda:0")
    text = torch.zeros(8, dtype=torch.uint8, device=dev)
    sa = torch.zeros(8, dtype=torch.int32, device=dev)
    idx = lrq.Index(text[:0], sa[:0])
    assert idx.count == 0
    off, recs = idx.all()
    assert off.cpu().tolist() == [0] and recs.shape[0] == 0
    assert idx.leftmost().shape[0] == 0
    assert idx.errors() == 0


def test_point_queries_match_all_positions():
    import torch
    from paper_1501_06663_amd import lrq
    say("case: point queries dna-like n=200000")
    text_np = workloads.dna_like(200000, 4)
    dev = torch.device("cuda:0")
    idx = lrq.Index(torch.from_numpy(text_np).to(dev),
                    torch.from_numpy(lrq.build_sa_host(text_np)).to(dev))
    full = idx.leftmost().cpu().numpy()
    rng = np.random.default_rng(1)
    pos = rng.integers(0, len(text_np), 50000).astype(np.int32)
    got = idx.query(torch.from_numpy(pos).to(dev)).cpu().numpy()
    assert np.array_equal(got, full[pos])
    assert idx.errors() == 0
    # out-of-range positions answer (-1, 0) and raise the query error bit
    bad = torch.tensor([-1, len(text_np), 5], dtype=torch.int32, device=dev)
    got = idx.query(bad).cpu().numpy()
    assert got[:2].tolist() == [[-1, 0], [-1, 0]] and got[2].tolist() == full[5].tolist()
    assert idx.errors() == lrq.ERR_QUERY


def test_paper_input_rank_lcp():
    """The filter from the paper's own device input (Rank + SA-order LCP).
    Rank and LCP are the GPU path's own (from its rank scatter and text-order
    LCP, permuted to SA order on the host); the expected values are the
    oracle's."""
    import torch
    from paper_1501_06663_amd import lrq
    text_np = workloads.dna_like(100000, 8)
    say("case: rank+lcp input n=100000")
    g = gpu_stages(text_np, modes=())
    n = len(text_np)
    lcp = np.zeros(n + 1, np.int32)
    lcp[g["rank"]] = g["pn"][:, 0]
    dev = torch.device("cuda:0")
    rank = torch.from_numpy(g["rank"]).to(dev)
    lcp_t = torch.from_numpy(lcp).to(dev)
    work = torch.empty(2 * n, dtype=torch.int32, device=dev)
    llrc = torch.empty((n, 2), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    blocks = torch.zeros(lrq.block_entries(n), dtype=torch.int64, device=dev)
    L = torch.empty(n, dtype=torch.int32, device=dev)
    scratch = torch.zeros(lrq.scratch_bytes(n), dtype=torch.uint8, device=dev)
    lrq.llr_from_rank_lcp(rank, lcp_t, n, work, llrc, count, blocks, L, scratch)
    o = oracle_view(text_np)
    assert np.array_equal(L.cpu().numpy(), o["L"])
    assert np.array_equal(llrc[: int(count.item())].cpu().numpy(), o["llrc_global"])
    assert np.array_equal(blocks.cpu().numpy(), o["blocks"])
    assert lrq.read_errors(scratch) == 0


def test_capacity_overflow_is_reported_not_written():
    import torch
    from paper_1501_06663_amd import lrq
    say("case: all-mode capacity too small")
    text_np = workloads.dna_like(30000, 2)
    dev = torch.device("cuda:0")
    idx = lrq.Index(torch.from_numpy(text_np).to(dev),
                    torch.from_numpy(lrq.build_sa_host(text_np)).to(dev))
    total = idx.all_count()
    cap = total // 2
    recs = torch.full((total, 2), -9, dtype=torch.int32, device=dev)
    offs = torch.empty(idx.total + 1, dtype=torch.int64, device=dev)
    with pytest.raises(lrq.LrqError) as e:
        lrq.lr_all(idx.llrc, idx.blocks, idx.total, None, 1, offs, recs, cap, idx.scratch)
    assert e.value.status == -3                       # LRQ_ENOSPC
    assert idx.errors() == lrq.ERR_CAPACITY
    r = recs.cpu().numpy()
    assert np.all(r[cap:] == -9)            # nothing written past the capacity
    assert int(offs[-1].item()) == total
    # the caller retries with the reported size and gets the full answer
    got = lrq.lr_all(idx.llrc, idx.blocks, idx.total, None, 1, offs, recs, total, idx.scratch)
    assert got == total and idx.errors() == 0


def test_bad_suffix_array_sets_error_bits():
    """An SA that is not a permutation is caught by the kernels' bounds checks
    (error bits), with no write outside the buffers."""
    import torch
    from paper_1501_06663_amd import lrq
    say("case: corrupt SA")
    n = 5000
    dev = torch.device("cuda:0")
    text = torch.from_numpy(workloads.uniform_dna(n, 1)).to(dev)
    sa = torch.from_numpy(lrq.build_sa_host(text.cpu().numpy())).to(dev)
    sa[17] = n + 100
    sa[18] = -3
    idx = lrq.Index(text, sa)
    assert idx.errors() & lrq.ERR_SA
