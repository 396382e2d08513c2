"""The seeded generators: determinism, and that the stress inputs have the
structure their tests rely on (checked with the oracle)."""
import numpy as np

import oracle
from paper_1501_06663_amd import workloads


def covering_counts(text):
    sa = oracle.suffix_array(text, method="doubling")
    rk = oracle.rank(sa)
    L = oracle.llr_lengths(rk, oracle.lcp(text, sa, rk))
    c = oracle.compact(L)
    starts = c[:, 0].astype(np.int64)
    ends = starts + c[:, 1].astype(np.int64) - 1
    k = np.arange(len(text))
    # entries with start <= k minus entries with end < k
    return np.searchsorted(starts, k, side="right") - np.searchsorted(ends, k, side="left")


def test_generators_are_deterministic():
    assert np.array_equal(workloads.dna_like(5000, 3), workloads.dna_like(5000, 3))
    assert np.array_equal(workloads.markov_text(5000, 3), workloads.markov_text(5000, 3))
    assert np.array_equal(workloads.staircase_repeats(40, 100, 1000), workloads.staircase_repeats(40, 100, 1000))
    assert not np.array_equal(workloads.dna_like(5000, 3), workloads.dna_like(5000, 4))


def test_staircase_has_wide_windows():
    text = workloads.staircase_repeats(150, 3996, 8192)
    cov = covering_counts(text)
    assert cov.max() > 64            # wider than the all-mode tie mask
    assert cov[4096] > 64            # a tile start covered by more than the staged margin
    seg = workloads.staircase_repeats(120, 2000, 4500, seed=1)
    assert covering_counts(seg).max() > 64
