"""Pins of the CPU oracle to the paper and to mathematics (no GPU).

Each test ties an oracle function to something other than itself: values the
paper prints (fixtures under tests/golden/, each with its citation), brute
force over all tiny strings, closed forms, textbook identities and
invariants that the paper proves.  A plausible slip anywhere in the oracle
(an off-by-one in the LCP sentinels, a strict/non-strict tie test, a wrong
stop test, a transposed max) fails at least one of them; the last tests
plant such slips in copies of the oracle's rules and check that the pins
catch them.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from paper_1501_06663_amd import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def as_sets(off, rec):
    return [set(map(tuple, rec[off[k]:off[k + 1]].tolist())) for k in range(len(off) - 1)]


def leftmost_from_sets(sets):
    out = []
    for st in sets:
        out.append(min(st) if st else (-1, 0))
    return np.array(out, dtype=np.int32).reshape(-1, 2)


def full(s, **kw):
    return oracle.pipeline(s, **kw)


# ------------------------------------------------------------ paper's values

def test_mississippi_table1():
    g = gold("mississippi.json")
    for method in ("naive", "doubling"):
        sa = oracle.suffix_array(g["text"].encode(), method)
        assert (sa + 1).tolist() == g["sa_1based"]
        lc = oracle.lcp(g["text"].encode(), sa, oracle.rank(sa))
        assert lc.tolist() == g["lcp"]


def test_abcabcddbca_lr2():
    g = gold("abcabcddbca.json")
    r = full(g["text"].encode())
    k = g["k_1based"] - 1
    got = as_sets(r["all_offsets"], r["all_recs"])[k]
    want = {(a - 1, b - a + 1) for a, b in g["lr_set_1based_start_end"]}
    assert got == want
    assert tuple(r["leftmost"][k]) == min(want)


def test_ababab_llr():
    g = gold("ababab.json")
    r = full(g["text"].encode())
    for k1, (a, b) in g["llr_1based"].items():
        i = int(k1) - 1
        assert r["L"][i] == b - a + 1
    starts = set(r["llrc"][:, 0].tolist())
    for k1 in g["useless_1based"]:
        assert k1 - 1 not in starts


def test_fig3_compaction():
    g = gold("fig3_compaction.json")
    L = np.array(g["llrr"], dtype=np.int32)
    c = oracle.compact(L)
    assert [(s + 1, ln) for s, ln in c.tolist()] == [tuple(x) for x in g["llrc_1based"]]
    flag = np.zeros(len(L), dtype=np.int64)
    flag[c[:, 0]] = 1
    assert flag.tolist() == g["flag"]
    assert np.cumsum(flag).tolist() == g["prefix_sum"]


def test_fig3_realised_by_a_string():
    # A text whose Lemma-1 lengths are exactly Figure 3's raw LLR array.
    g = gold("fig3_compaction.json")
    assert full(b"abcaabcb")["L"].tolist() == g["llrr"]


# --------------------------------------------------------------- brute force

def _check_against_brute(s):
    off_b, rec_b = oracle.lr_brute(s)
    sets = as_sets(off_b, rec_b)
    r = full(s)
    assert as_sets(r["all_offsets"], r["all_recs"]) == sets, s
    assert r["leftmost"].tolist() == leftmost_from_sets(sets).tolist(), s
    n = len(s)
    assert oracle.lr_leftmost_compact(r["llrc"], n).tolist() == r["leftmost"].tolist()
    off_c, rec_c = oracle.lr_all_compact(r["llrc"], n)
    assert np.array_equal(off_c, r["all_offsets"]) and np.array_equal(rec_c, r["all_recs"])
    assert oracle.lr_window(r["L"], "leftmost").tolist() == r["leftmost"].tolist()
    off_w, rec_w = oracle.lr_window(r["L"], "all")
    assert np.array_equal(off_w, r["all_offsets"]) and np.array_equal(rec_w, r["all_recs"])


@pytest.mark.parametrize("sigma,nmax", [(2, 11), (3, 8)])
def test_exhaustive_small_strings(sigma, nmax):
    """Every string over a sigma-letter alphabet up to length nmax."""
    alpha = b"abc"[:sigma]
    for n in range(1, nmax + 1):
        for tup in itertools.product(alpha, repeat=n):
            _check_against_brute(bytes(tup))


@pytest.mark.parametrize("sigma", [1, 2, 4, 20, 96])
def test_random_strings_vs_brute(sigma):
    rng = np.random.default_rng(1000 + sigma)
    for _ in range(12):
        n = int(rng.integers(1, 41))
        s = rng.integers(0, sigma, n).astype(np.uint8) + 32
        _check_against_brute(s.tobytes())


@pytest.mark.parametrize("sigma", [1, 2, 4, 20, 96])
def test_walk_forms_agree_mid_size(sigma):
    """Algorithms 1/3 (raw), 2/4 (compact) and the sliding window agree."""
    rng = np.random.default_rng(2000 + sigma)
    for _ in range(6):
        n = int(rng.integers(1, 301))
        s = (rng.integers(0, sigma, n).astype(np.uint8) + 32).tobytes()
        r = full(s)
        assert oracle.lr_leftmost_compact(r["llrc"], n).tolist() == r["leftmost"].tolist()
        oc, rc = oracle.lr_all_compact(r["llrc"], n)
        assert np.array_equal(oc, r["all_offsets"]) and np.array_equal(rc, r["all_recs"])
        assert oracle.lr_window(r["L"]).tolist() == r["leftmost"].tolist()


# ------------------------------------------------------- SA / LCP definitions

def _direct_lcp(s, i, j):
    h = 0
    while i + h < len(s) and j + h < len(s) and s[i + h] == s[j + h]:
        h += 1
    return h


@pytest.mark.parametrize("kind", ["dna", "fib", "markov", "unary"])
def test_sa_and_lcp_by_definition(kind):
    n = 3000
    s = {"dna": lambda: workloads.dna_like(n, 7, 6), "fib": lambda: workloads.fibonacci_word(n),
         "markov": lambda: workloads.markov_text(n, 3), "unary": lambda: np.full(n, 65, np.uint8)}[kind]()
    b = s.tobytes()
    sa = oracle.suffix_array(s)
    assert sorted(sa.tolist()) == list(range(n))
    for r in range(1, n):
        assert b[sa[r - 1]:] < b[sa[r]:]
    lc = oracle.lcp(s, sa, oracle.rank(sa))
    assert lc[0] == 0 and lc[n] == 0
    rng = np.random.default_rng(5)
    for r in rng.integers(1, n, 300):
        assert lc[r] == _direct_lcp(b, int(sa[r - 1]), int(sa[r]))


@pytest.mark.parametrize("n", [1, 2, 17, 1 << 12, (1 << 14) + 3])
def test_naive_sort_equals_prefix_doubling(n):
    for s in (workloads.fibonacci_word(n), workloads.dna_like(n, 11, 3),
              workloads.markov_text(n, 4), np.full(n, 7, np.uint8)):
        assert np.array_equal(oracle.suffix_array(s, "naive"), oracle.suffix_array(s, "doubling"))


def test_llr_direct_matches_lemma1():
    for s in (workloads.dna_like(2000, 3, 5), workloads.fibonacci_word(1500),
              workloads.markov_text(2000, 9)):
        L = full(s)["L"]
        idx = np.arange(len(s))
        assert np.array_equal(oracle.llr_direct(s, idx), L)


# ---------------------------------------------------- closed forms / lemmas

@pytest.mark.parametrize("n", [1, 2, 3, 8, 50])
def test_unary_string_closed_form(n):
    """S = a^n: 1-based leftmost <1,n-1> for k<n and <2,n-1> for k=n."""
    r = full(b"a" * n)
    if n == 1:
        assert r["leftmost"].tolist() == [[-1, 0]]
        return
    want = [[0, n - 1]] * (n - 1) + [[1, n - 1]]
    assert r["leftmost"].tolist() == want
    sets = as_sets(r["all_offsets"], r["all_recs"])
    assert sets[0] == {(0, n - 1)} and sets[-1] == {(1, n - 1)}
    for k in range(1, n - 1):
        assert sets[k] == {(0, n - 1), (1, n - 1)}


def test_singletons_have_no_lr():
    s = b"xaybzacb"
    r = full(s)
    counts = {c: s.count(c) for c in set(s)}
    for k, c in enumerate(s):
        if counts[c] == 1:
            assert tuple(r["leftmost"][k]) == (-1, 0)
            assert r["all_offsets"][k + 1] == r["all_offsets"][k]
        else:
            assert r["leftmost"][k][1] >= 1


@pytest.mark.parametrize("seed", range(4))
def test_longest_lr_is_longest_repeated_substring(seed):
    s = workloads.dna_like(5000, seed, 4)
    r = full(s)
    assert r["leftmost"][:, 1].max() == r["lcp"].max()


@pytest.mark.parametrize("seed", range(3))
def test_lemma2_and_compaction_invariants(seed):
    s = workloads.markov_text(4000, seed)
    r = full(s)
    L = r["L"].astype(np.int64)
    assert np.all(L[:-1] <= L[1:] + 1)            # Lemma 2
    assert L[-1] <= 1
    c = r["llrc"].astype(np.int64)
    assert np.all(np.diff(c[:, 0]) > 0)           # starts strictly increase
    assert np.all(np.diff(c[:, 0] + c[:, 1]) > 0)  # ends strictly increase


def test_alphabet_relabelling_invariance():
    s = workloads.dna_like(3000, 2, 3)
    perm = np.arange(256, dtype=np.uint8)
    perm[[65, 67, 71, 84]] = [84, 65, 67, 71]
    r1, r2 = full(s), full(perm[s])
    assert np.array_equal(r1["L"], r2["L"])
    assert np.array_equal(r1["leftmost"], r2["leftmost"])
    assert np.array_equal(r1["all_recs"], r2["all_recs"])


def test_records_are_repeats_that_cover_k():
    s = workloads.protein_like(1500, 4, 3)
    b = s.tobytes()
    r = full(s)
    off, rec = r["all_offsets"], r["all_recs"]
    for k in range(0, len(s), 7):
        for st, ln in rec[off[k]:off[k + 1]].tolist():
            assert st <= k <= st + ln - 1
            sub = b[st:st + ln]
            assert b.find(sub) != st or b.find(sub, st + 1) >= 0   # occurs at some j != st


def _occurs_elsewhere(b, i, ln):
    """Does b[i:i+ln] also start at some j != i?  (bytes.find checks every
    start, so overlapping occurrences count, as Section 2's definition of a
    unique substring requires.)"""
    sub = b[i:i + ln]
    return b.find(sub) != i or b.find(sub, i + 1) >= 0


def _definition_violations(b, left, off, rec, ks):
    """Positions among ks where (left, off, rec) break Definition 1, checked
    with plain substring search and none of the oracle's code: for M_k the
    reported LR length at k,
      * no substring of length M_k + 1 that covers k may occur twice (so no
        longer covering repeat exists: any longer one would contain such a
        substring, occurring at both of its places);
      * the all-mode list of k must be exactly the starts of the length-M_k
        substrings that cover k and occur twice, and the leftmost record its
        smallest start."""
    n = len(b)
    bad = []
    for k in ks:
        m = int(left[k][1])
        ok = all(not _occurs_elsewhere(b, i, m + 1)
                 for i in range(max(0, k - m), min(k, n - m - 1) + 1))
        got = rec[off[k]:off[k + 1]].tolist()
        if m == 0:
            ok = ok and got == [] and tuple(left[k]) == (-1, 0)
        else:
            want = [i for i in range(max(0, k - m + 1), min(k, n - m) + 1)
                    if _occurs_elsewhere(b, i, m)]
            ok = (ok and [st for st, _ in got] == want and all(ln == m for _, ln in got)
                  and bool(want) and tuple(left[k]) == (want[0], m))
        if not ok:
            bad.append(k)
    return bad


def _sample_positions(M, n, seed=31):
    # random positions, plus the ones with the longest LRs (inside planted
    # copies, where the covering windows are widest)
    rng = np.random.default_rng(seed)
    return sorted(set(rng.integers(0, n, 100).tolist())
                  | set(np.argsort(-M, kind="stable")[:20].tolist()))


@pytest.mark.parametrize("kind", ["dna_planted", "markov", "protein_planted"])
def test_no_longer_covering_repeat_exists(kind):
    """Definition 1 on sampled positions of mid-size strings (see
    _definition_violations)."""
    n = {"dna_planted": 12000, "markov": 20000, "protein_planted": 10000}[kind]
    s = {"dna_planted": lambda: workloads.dna_like(n, 21, 6),
         "markov": lambda: workloads.markov_text(n, 22),
         "protein_planted": lambda: workloads.protein_like(n, 23, 5)}[kind]()
    r = full(s)
    M = r["leftmost"][:, 1].astype(np.int64)
    assert M.max() >= (40 if kind != "markov" else 5)
    ks = _sample_positions(M, n)
    assert _definition_violations(s.tobytes(), r["leftmost"], r["all_offsets"], r["all_recs"],
                                  ks) == []


def test_planted_cover_slip_fails_the_definition_check():
    """A walk whose cover test is strict (i + L_i - 1 > k instead of >= k)
    drops the LLRs that end exactly at k; the Definition-1 check above finds
    the positions where that changes the answer."""
    s = workloads.dna_like(6000, 24, 4)
    r = full(s)
    L = r["L"].astype(np.int64)
    n = len(s)
    left, offs, recs = [], [0], []
    for k in range(n):
        # the covering LLRs, walking left from k until one ends before k, with
        # the planted slip: one that ends exactly at k is not counted
        cov = []
        for i in range(k, -1, -1):
            if i + L[i] - 1 < k:
                break
            if i + L[i] - 1 > k:
                cov.append(i)
        m = max((int(L[i]) for i in cov), default=0)
        lst = sorted(i for i in cov if L[i] == m) if m else []
        left.append((lst[0], m) if lst else (-1, 0))
        recs.extend((i, m) for i in lst)
        offs.append(len(recs))
    left = np.array(left, np.int64)
    offs = np.array(offs, np.int64)
    recs = np.array(recs, np.int64).reshape(-1, 2)
    M = r["leftmost"][:, 1].astype(np.int64)
    ks = _sample_positions(M, n)
    assert _definition_violations(s.tobytes(), r["leftmost"], r["all_offsets"], r["all_recs"], ks) == []
    assert len(_definition_violations(s.tobytes(), left, offs, recs, ks)) > 0


def test_empty_string():
    r = full(b"")
    assert r["leftmost"].shape == (0, 2) and r["all_offsets"].tolist() == [0]


# ------------------------------------------------ readings of the paper text

def _compact_walk_literal(c, k):
    """Algorithm 2 with the stop test exactly as printed (end < k)."""
    best = (-1, 0)
    ends = c[:, 0] + c[:, 1] - 1
    t0 = int(np.searchsorted(ends, k))
    if t0 >= len(c) or c[t0, 0] > k:
        return best
    for t in range(t0, len(c)):
        if ends[t] < k:
            break
        if c[t, 1] > best[1]:
            best = (int(c[t, 0]), int(c[t, 1]))
    return best


def test_printed_compact_stop_test_is_a_misprint():
    """Taken literally, the printed stop test keeps walking past entries that
    start right of k and reports them; the reading 'stop at start > k' agrees
    with the definition (brute force).  Finds a witness among short ternary
    strings."""
    witness = None
    for n in range(2, 8):
        for tup in itertools.product(b"abc", repeat=n):
            s = bytes(tup)
            r = full(s)
            for k in range(n):
                if _compact_walk_literal(r["llrc"], k) != tuple(r["leftmost"][k]):
                    witness = (s, k)
                    break
            if witness:
                break
        if witness:
            break
    assert witness is not None
    s, k = witness
    off, rec = oracle.lr_brute(s)
    assert tuple(leftmost_from_sets(as_sets(off, rec))[k]) == tuple(full(s)["leftmost"][k])


# ------------------------------------------ planted slips are caught (CPU)

def _leftmost_walk_variant(L, strict):
    out = []
    for k in range(len(L)):
        best = (-1, 0)
        for i in range(k, -1, -1):
            if i + L[i] - 1 < k:
                break
            if (L[i] > best[1]) if strict else (L[i] >= best[1]):
                best = (i, int(L[i]))
        out.append(best)
    return out


def test_planted_tie_slip_is_caught():
    """Walking left with '>' keeps the rightmost of equal LLRs: the abcabcddbca
    pin (leftmost LR_2 = abc) catches it."""
    L = full(b"abcabcddbca")["L"]
    assert _leftmost_walk_variant(L, strict=False)[1] == (0, 3)
    assert _leftmost_walk_variant(L, strict=True)[1] != (0, 3)


def test_planted_lcp_sentinel_slip_is_caught():
    """Dropping the trailing LCP sentinel (reading LCP[Rank[i]+1] for the last
    suffix as garbage instead of 0) changes mississippi's Lemma-1 lengths."""
    s = b"mississippi"
    sa = oracle.suffix_array(s)
    rk = oracle.rank(sa)
    lc = oracle.lcp(s, sa, rk)
    good = oracle.llr_lengths(rk, lc)
    bad_lc = lc.copy()
    bad_lc[-1] = 9
    assert oracle.llr_lengths(rk, bad_lc).tolist() != good.tolist()
    assert good.tolist() == [0, 4, 3, 2, 4, 3, 2, 1, 1, 1, 1]
