"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the oracle-side tests and the GPU path.  It draws
strings and request traces only; it holds none of the longest-repeat
arithmetic.  Every generator uses ``numpy.random.default_rng(seed)`` (PCG64)
and draws in the fixed order documented in each function, so a (config,
size, seed) triple always yields the same bytes.

The paper's experiments use the Pizza&Chili DNA, English and Protein texts
(Section 6, "Experiment Environment Setup"); those files are not available
here, so these generators stand in for them:

* uniform DNA                      -- i.i.d. over ACGT (small plain case)
* DNA-like with planted copies     -- skewed ACGT background plus mutated
                                      copies of log-uniform length, which give
                                      the long, nested repeats of genomic text
* Fibonacci word                   -- the classic extreme of long repeats
* order-2 Markov text              -- a stand-in for natural-language text
* protein-like                     -- 20 residues with Zipf(1.0) frequencies
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Iterator, List, Optional, Tuple

import numpy as np

DNA = np.frombuffer(b"ACGT", dtype=np.uint8)
PROTEIN = np.frombuffer(b"ACDEFGHIKLMNPQRSTVWY", dtype=np.uint8)
# 95 printable ASCII symbols 0x20..0x7E plus newline.
TEXT96 = np.concatenate([np.arange(0x20, 0x7F, dtype=np.uint8),
                         np.array([0x0A], dtype=np.uint8)])

# Full-size configurations of the measured workloads.
C1_N = 65_536
C2_N = 16_777_216
C2_COPIES = 2_000
C3A_N = 1 << 22
C3B_N = 67_108_864
C4_SEGMENTS = 512
C4_MIN_LOG2, C4_MAX_LOG2 = 10, 20


def _zipf_probs(k: int, s: float) -> np.ndarray:
    w = 1.0 / np.arange(1, k + 1, dtype=np.float64) ** s
    return w / w.sum()


def uniform_dna(n: int, seed: int = 0) -> np.ndarray:
    """n i.i.d. uniform characters over ACGT.  Draws: one integers(0,4,n)."""
    rng = np.random.default_rng(seed)
    return DNA[rng.integers(0, 4, n)]


def plant_copies(s: np.ndarray, n_copies: int, rng: np.random.Generator,
                 alphabet: np.ndarray, min_len: int = 50, max_len: int = 5000,
                 mutate: float = 0.01) -> np.ndarray:
    """Apply ``n_copies`` mutated copy operations to ``s`` in place.

    Copy c, in order: length m = floor(exp(U(ln min_len, ln max_len))),
    capped at len(s)//4; source and destination offsets uniform in
    [0, len(s)-m); each copied character is, with probability ``mutate``,
    replaced by a uniformly chosen *different* symbol of ``alphabet``.
    Copies are applied to the evolving string.  Per copy the draws are:
    random() for m, integers() for src, integers() for dst, random(m) for the
    mutation mask, integers(1, |alphabet|, k) for the k replacements.
    """
    n = len(s)
    if n < 8 or n_copies <= 0:
        return s
    sigma = len(alphabet)
    lut = np.full(256, 0, dtype=np.int64)
    lut[alphabet] = np.arange(sigma)
    lo, hi = math.log(min_len), math.log(max_len)
    cap = max(1, n // 4)
    for _ in range(n_copies):
        m = int(math.exp(lo + (hi - lo) * rng.random()))
        m = max(1, min(m, cap))
        src = int(rng.integers(0, n - m))
        dst = int(rng.integers(0, n - m))
        seg = s[src:src + m].copy()
        mask = rng.random(m) < mutate
        k = int(mask.sum())
        if k:
            old = lut[seg[mask]]
            seg[mask] = alphabet[(old + rng.integers(1, sigma, k)) % sigma]
        s[dst:dst + m] = seg
    return s


def dna_like(n: int, seed: int = 0, n_copies: Optional[int] = None) -> np.ndarray:
    """DNA-like string: background P(A,C,G,T) = (.3,.2,.2,.3) plus planted copies.

    ``n_copies`` defaults to the full-size density, 2000 copies per 2^24
    characters, rounded.  Draws: choice(4, n, p) for the background, then the
    copy draws of :func:`plant_copies`.
    """
    rng = np.random.default_rng(seed)
    s = DNA[rng.choice(4, size=n, p=[0.3, 0.2, 0.2, 0.3])]
    if n_copies is None:
        n_copies = int(round(C2_COPIES * n / float(C2_N)))
    return plant_copies(s, n_copies, rng, DNA)


def protein_like(n: int, seed: int = 0, n_copies: Optional[int] = None) -> np.ndarray:
    """20-letter protein-like string, residue ranks Zipf(1.0), plus planted copies.

    The residue of rank r (1-based) is the r-th letter of ACDEFGHIKLMNPQRSTVWY.
    Planted copies use the DNA-like density (2000 per 2^24 characters), since
    real protein collections also repeat whole domains.
    """
    rng = np.random.default_rng(seed)
    s = PROTEIN[rng.choice(20, size=n, p=_zipf_probs(20, 1.0))]
    if n_copies is None:
        n_copies = int(round(C2_COPIES * n / float(C2_N)))
    return plant_copies(s, n_copies, rng, PROTEIN)


def fibonacci_word(n: int) -> np.ndarray:
    """First n characters of the fixed point of a -> ab, b -> a (over {a,b})."""
    a, b = b"a", b"ab"
    while len(b) < n:
        a, b = b, b + a
    return np.frombuffer(b[:n], dtype=np.uint8).copy()


def markov_text(n: int, seed: int = 0, chains: Optional[int] = None,
                s: float = 1.1) -> np.ndarray:
    """Order-2 Markov text over 96 printable symbols with Zipf(s) marginals.

    P(next | a, b) = 1/2 Zipf(s) over a global symbol order + 1/2 Zipf(s) over
    a per-context order, so the unigram marginal is close to Zipf(s).  The
    text is ``chains`` independent chains of equal length laid end to end
    (the chain context restarts at each junction), which lets the sampling
    run vectorised across chains; by default every chain is 4096 symbols
    long (16384 chains at n = 2^26).  Draws, in order: permutation(96) for the
    global order; 96*96 permutations(96) for the contexts; two initial
    symbols per chain; then, per block of steps, the Zipf ranks and the
    mixture coins.
    """
    rng = np.random.default_rng(seed)
    k = len(TEXT96)
    glob = rng.permutation(k)
    ctx_perm = np.argsort(rng.random((k * k, k)), axis=1).astype(np.int16)
    cum = np.cumsum(_zipf_probs(k, s))
    cum[-1] = 1.0
    if chains is None:
        chains = max(1, n // 4096)
    chains = max(1, min(chains, n))
    steps = -(-n // chains)
    out = np.empty((chains, steps), dtype=np.int16)
    a = glob[np.searchsorted(cum, rng.random(chains), side="right")]
    b = glob[np.searchsorted(cum, rng.random(chains), side="right")]
    block = 1024
    for t0 in range(0, steps, block):
        t1 = min(steps, t0 + block)
        r = np.searchsorted(cum, rng.random((chains, t1 - t0)), side="right")
        coin = rng.random((chains, t1 - t0)) < 0.5
        for t in range(t1 - t0):
            rt = r[:, t]
            nxt = np.where(coin[:, t], glob[rt], ctx_perm[a * k + b, rt])
            out[:, t0 + t] = nxt
            a, b = b, nxt
    return TEXT96[out.reshape(-1)[:n]]


def staircase_repeats(steps: int, anchor: int, background: int, base_len: int = 200,
                      seed: int = 0) -> np.ndarray:
    """A string whose repeats overlap as much as the keep rule allows: an
    i.i.d. ACGT background of ``background`` characters, followed, for
    i = 0..steps-1, by 8 random separator characters and a copy of
    ``s[anchor + i : anchor + i + base_len + i]``.  Position anchor + i then
    has a repeat of length about base_len + i, so the compact LLR array keeps
    a run of ``steps`` consecutive entries and positions inside the run are
    covered by up to ``steps`` of them -- far wider windows than the measured
    workloads produce.  Draws: the background, then all separators at once."""
    if anchor + 2 * steps + base_len > background:
        raise ValueError("the copied spans must lie inside the background")
    rng = np.random.default_rng(seed)
    bg = DNA[rng.integers(0, 4, background)]
    seps = DNA[rng.integers(0, 4, (steps, 8))]
    parts = [bg]
    for i in range(steps):
        parts.append(seps[i])
        parts.append(bg[anchor + i: anchor + i + base_len + i])
    return np.ascontiguousarray(np.concatenate(parts))


def log_uniform_lengths(rng: np.random.Generator, count: int, lo: float, hi: float) -> np.ndarray:
    """floor(exp(U(ln lo, ln hi))) for ``count`` draws (one random(count))."""
    u = rng.random(count)
    return np.floor(np.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * u)).astype(np.int64)


# ---------------------------------------------------------------- configs --

def config1(seed: int = 0, n: int = C1_N) -> np.ndarray:
    """Plain single string: i.i.d. uniform ACGT."""
    return uniform_dna(n, seed)


def config2(seed: int = 0, n: int = C2_N) -> np.ndarray:
    """Plain DNA-like string with planted mutated copies (2000 per 2^24 chars)."""
    return dna_like(n, seed)


def config3a(n: int = C3A_N) -> np.ndarray:
    """Fibonacci word prefix."""
    return fibonacci_word(n)


def config3b(seed: int = 0, n: int = C3B_N) -> np.ndarray:
    """Order-2 Markov text over 96 printable symbols, Zipf(1.1) marginals."""
    return markov_text(n, seed)


def config4(seed: int = 0, nseg: int = C4_SEGMENTS, min_log2: int = C4_MIN_LOG2,
            max_log2: int = C4_MAX_LOG2) -> Tuple[np.ndarray, np.ndarray]:
    """Batch of independent DNA-like strings with log-uniform lengths.

    Returns (concatenated text, int64 segment offsets of length nseg+1).
    Draws: the nseg lengths from one generator seeded ``seed``; string b is
    then :func:`dna_like` with seed ``seed*100003 + b + 1`` and
    Poisson(2000*m/2^24) planted copies drawn from the lengths generator.
    """
    rng = np.random.default_rng(seed)
    lens = log_uniform_lengths(rng, nseg, 2.0 ** min_log2, 2.0 ** max_log2)
    copies = rng.poisson(C2_COPIES * lens / float(C2_N))
    parts = [dna_like(int(m), seed * 100003 + b + 1, int(c))
             for b, (m, c) in enumerate(zip(lens, copies))]
    off = np.zeros(nseg + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    text = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    return text, off


@dataclass
class Request:
    """One serving request: a string that arrives, then query batches on it."""
    rid: int
    arrival: float                 # seconds from trace start
    kind: str                      # "dna" or "protein"
    text: np.ndarray
    batch_times: List[float] = field(default_factory=list)   # absolute seconds
    batches: List[np.ndarray] = field(default_factory=list)  # int32 positions
    mode: str = "leftmost"         # "leftmost": one record per position; "all": every LR


def serving_trace(rate: float, count: int, seed: int = 0, min_len: float = 1e4,
                  max_len: float = 4e6, mean_gap: float = 2e-3,
                  max_batches: int = 64, min_q: float = 1e3,
                  max_q: float = 1e5, all_fraction: float = 0.0) -> Iterator[Request]:
    """Poisson arrivals (``rate`` strings/s) of DNA-like or protein-like strings.

    Each string: length floor(exp(U(ln min_len, ln max_len))); kind 50/50;
    U{1..max_batches} query batches of floor(exp(U(ln min_q, ln max_q)))
    positions uniform in [0, n), separated by exponential gaps of mean
    ``mean_gap`` seconds after the arrival.  Strings are generated lazily.
    A request asks for all LRs of its positions with probability
    ``all_fraction`` (drawn from a second generator seeded seed + 7919, so the
    other draws do not depend on it), otherwise for the leftmost one.
    """
    rng = np.random.default_rng(seed)
    mode_rng = np.random.default_rng(seed + 7919)
    t = 0.0
    for rid in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(log_uniform_lengths(rng, 1, min_len, max_len)[0])
        kind = "dna" if rng.random() < 0.5 else "protein"
        sub = int(rng.integers(0, 2 ** 31 - 1))
        copies = int(rng.poisson(C2_COPIES * n / float(C2_N)))
        text = (dna_like if kind == "dna" else protein_like)(n, sub, copies)
        req = Request(rid, t, kind, text,
                      mode="all" if mode_rng.random() < all_fraction else "leftmost")
        nb = int(rng.integers(1, max_batches + 1))
        qt = t
        for _ in range(nb):
            qt += float(rng.exponential(mean_gap))
            m = int(log_uniform_lengths(rng, 1, min_q, max_q)[0])
            req.batch_times.append(qt)
            req.batches.append(rng.integers(0, n, m).astype(np.int32))
        yield req


def retime(trace: List[Request], factor: float, gap_factor: float = 1.0) -> List[Request]:
    """The same strings and query batches with every arrival time multiplied
    by ``factor`` (a factor of r0 / r turns a trace drawn at rate r0 into one
    at rate r) and each batch's delay after its string's arrival multiplied by
    ``gap_factor``.  The texts and position arrays are shared with the input
    trace."""
    out = []
    for r in trace:
        a = r.arrival * factor
        out.append(Request(r.rid, a, r.kind, r.text,
                           [a + (bt - r.arrival) * gap_factor for bt in r.batch_times],
                           r.batches, r.mode))
    return out
