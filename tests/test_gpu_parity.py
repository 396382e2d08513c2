"""Parity of the HIP path with the CPU oracle, element by element, at sizes
the oracle finishes in seconds.  Every stage is compared: Rank, the suffix
neighbours, text-order LCP pairs, Lemma-1 lengths, the compact LLR array,
leftmost LRs and the all-LR CSR lists, through the 32-bit calls and through
the 64-bit (lrq64_) calls.  Integer work: the bar is equality.

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
    """Every stage of the 32-bit calls and of the 64-bit (lrq64_) calls on the
    same input, each compared with the oracle."""
    say("case:", tag, "n=%d" % len(text), "segments=%s" % (None if seg_off is None else len(seg_off) - 1))
    o = oracle_view(text, seg_off, walks=walks, sa_method=sa_method)
    g = gpu_stages(text, seg_off, modes=modes)
    compare(g, o, tag=tag)
    say("  and with 64-bit positions")
    g64 = gpu_stages(text, seg_off, modes=modes, wide=True)
    compare(g64, o, tag=tag + " (64-bit)")
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


@pytest.mark.parametrize("nseg", [63, 64, 65, 4096, 4097])
def test_batch_segment_counts(nseg):
    # segment counts around the rounds of the kernels' segment search: up to
    # 64 strings take one round of 64 probes (and 512-thread rank-scatter
    # blocks), more take two; with 64 or 4,096 strings the last round's range
    # is 64 starts wide, so a position in its last string needs the start one
    # past the range, loaded separately
    rng = np.random.default_rng(nseg)
    lens = rng.integers(1, 48, nseg)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    text = (rng.integers(0, 4, int(off[-1])) + 97).astype(np.uint8)
    run_case("batch %d segments" % nseg, text, off)


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


def _oracle_all_at(o, pos):
    off, rec = o["all_offsets"], o["all_recs"]
    pos = np.asarray(pos, dtype=np.int64)
    outo = np.zeros(len(pos) + 1, dtype=np.int64)
    outo[1:] = np.cumsum(off[pos + 1] - off[pos])
    parts = [rec[off[k]:off[k + 1]] for k in pos]
    return outo, (np.concatenate(parts) if parts else np.zeros((0, 2), np.int32)).reshape(-1, 2)


@pytest.mark.parametrize("kind", ["dna", "protein", "staircase"])
def test_point_queries_match_the_oracle(kind):
    """lrq_query_positions in both modes against the oracle's answers at the
    queried positions (Algorithm 2 / Algorithm 4 per position); queries
    repeat positions and cover both ends of the string."""
    import torch
    from paper_1501_06663_amd import lrq
    text_np = {"dna": lambda: workloads.dna_like(200000, 4),
               "protein": lambda: workloads.protein_like(120000, 5),
               "staircase": lambda: workloads.staircase_repeats(111, 300, 6000)}[kind]()
    n = len(text_np)
    say("case: point queries", kind, "n=%d" % n)
    dev = torch.device("cuda:0")
    idx = lrq.Index(torch.from_numpy(text_np).to(dev),
                    torch.from_numpy(lrq.build_sa_host(text_np)).to(dev))
    o = oracle_view(text_np)
    rng = np.random.default_rng(1)
    pos = np.concatenate([rng.integers(0, n, 30000), [0, n - 1, 0, n // 2, n // 2]]).astype(np.int32)
    pt = torch.from_numpy(pos).to(dev)
    got = idx.query(pt).cpu().numpy()
    assert np.array_equal(got, o["leftmost"][pos])
    left, off, recs = idx.query(pt, mode=lrq.ALL, capacity=100)   # too small: enlarged once
    woff, wrec = _oracle_all_at(o, pos)
    assert np.array_equal(left.cpu().numpy(), o["leftmost"][pos])
    assert np.array_equal(off.cpu().numpy(), woff)
    assert np.array_equal(recs.cpu().numpy(), wrec)
    assert idx.errors() == 0
    # out-of-range positions: (-1, 0) / empty lists and the query error bit
    bad = torch.tensor([-1, n, 5], dtype=torch.int32, device=dev)
    got = idx.query(bad).cpu().numpy()
    assert got[:2].tolist() == [[-1, 0], [-1, 0]] and got[2].tolist() == o["leftmost"][5].tolist()
    assert idx.errors() == lrq.ERR_QUERY
    # all mode: records past capacity are never written
    m = len(pos)
    offs = torch.full((m + 1,), -7, dtype=torch.int64, device=dev)
    cap = int(woff[-1]) // 2
    recs = torch.full((cap + 4, 2), -7, dtype=torch.int32, device=dev)
    with pytest.raises(lrq.LrqError) as e:
        lrq.query_positions(idx.llrc, idx.blocks, n, pt, m, None, idx.scratch, mode=lrq.ALL,
                            offsets=offs, recs=recs, capacity=cap)
    assert e.value.status == -3
    assert np.array_equal(offs.cpu().numpy(), woff)
    r = recs.cpu().numpy()
    assert np.array_equal(r[:cap], wrec[:cap]) and (r[cap:] == -7).all()
    assert idx.errors() == lrq.ERR_CAPACITY


def test_query_multi_both_modes():
    """lrq_query_multi over strings living in two indexes (a 3-string batch
    and a single string), both modes, with an unknown string id, against the
    oracle per string."""
    import torch
    from paper_1501_06663_amd import lrq
    say("case: query_multi over two indexes, both modes")
    dev = torch.device("cuda:0")
    strings = [workloads.dna_like(30000, 41), workloads.protein_like(20000, 42),
               workloads.markov_text(25000, 43), workloads.dna_like(50000, 44)]
    off = np.array([0, 30000, 50000, 75000], dtype=np.int64)
    btext = np.concatenate(strings[:3])
    bidx = lrq.Index(torch.from_numpy(btext).to(dev),
                     torch.from_numpy(lrq.build_sa_host_batch(btext, off)).to(dev),
                     torch.from_numpy(off).to(dev))
    sidx = lrq.Index(torch.from_numpy(strings[3]).to(dev),
                     torch.from_numpy(lrq.build_sa_host(strings[3])).to(dev))
    refs = [(bidx.llrc.data_ptr(), bidx.blocks.data_ptr(), 75000, int(off[b]), int(off[b + 1] - off[b]))
            for b in range(3)] + [(sidx.llrc.data_ptr(), sidx.blocks.data_ptr(), 50000, 0, 50000)]
    refs_t = torch.tensor(refs, dtype=torch.int64, device=dev)
    rng = np.random.default_rng(7)
    sid = rng.integers(0, 4, 20000).astype(np.int32)
    sid[17] = 4                                           # no such string
    pos = np.array([rng.integers(0, len(strings[s])) if s < 4 else 0 for s in sid], np.int32)
    wants = [oracle_view(s) for s in strings]
    m = len(sid)
    scratch = torch.zeros(lrq.scratch_bytes(m), dtype=torch.uint8, device=dev)
    st, pt = torch.from_numpy(sid).to(dev), torch.from_numpy(pos).to(dev)
    out = torch.empty((m, 2), dtype=torch.int32, device=dev)
    lrq.query_multi(refs_t, 4, st, pt, m, out, scratch)
    offs = torch.empty(m + 1, dtype=torch.int64, device=dev)
    recs = torch.empty((4 * m, 2), dtype=torch.int32, device=dev)
    out2 = torch.empty((m, 2), dtype=torch.int32, device=dev)
    tot = lrq.query_multi(refs_t, 4, st, pt, m, out2, scratch, mode=lrq.ALL, offsets=offs,
                          recs=recs, capacity=4 * m)
    got_l, got_l2 = out.cpu().numpy(), out2.cpu().numpy()
    got_o, got_r = offs.cpu().numpy(), recs[:tot].cpu().numpy()
    assert lrq.read_errors(scratch) == lrq.ERR_QUERY        # the unknown string id only
    for q in range(m):
        if sid[q] == 4:
            assert got_l[q].tolist() == [-1, 0] and got_o[q + 1] == got_o[q]
            continue
        w = wants[sid[q]]
        k = int(pos[q])
        assert got_l[q].tolist() == w["leftmost"][k].tolist(), q
        assert got_l2[q].tolist() == w["leftmost"][k].tolist(), q
        lst = w["all_recs"][w["all_offsets"][k]:w["all_offsets"][k + 1]]
        assert np.array_equal(got_r[got_o[q]:got_o[q + 1]], lst), q


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
