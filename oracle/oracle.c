/*
 * oracle.c -- plain, slow CPU reference for longest-repeat (LR) queries.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the GPU path.
 *
 * Source: Y. Tian and B. Xu, "On Longest Repeat Queries Using GPU"
 * (arXiv 1501.06663).  The paper is 1-based; everything here is 0-based:
 * position k of the paper is k-1 here, and "does not exist" is the paper's
 * own <-1,0> sentinel.
 *
 *   suffix order, repeat, singleton ....... Section 2 (problem formulation)
 *   SA, Rank, LCP with zero sentinels ..... Section 3, Table 1 (mississippi)
 *   L_i = max(LCP[Rank[i]], LCP[Rank[i]+1]) Section 3, Lemma 1
 *   LRs from the raw LLR array ............ Definition 1, Lemmas 2-3 (the
 *                                           results of Algorithms 1 and 3)
 *   compaction of the LLR array ........... Section 4.2 (useless = contained
 *                                           in another LLR), Lemma 2
 *   compact-walk leftmost / all LRs ....... Section 4.2, Algorithms 2 and 4
 *
 * Readings of the paper that this file takes:
 *   - tuples are <start, length> as the prose says, not <start, end>;
 *   - the compact walk stops at the first entry whose start lies right of k
 *     (the printed stop test compares the entry's end with k, which never
 *     fires because ends increase along the array);
 *   - ties go to the smallest start; all-mode lists are in ascending start;
 *   - an empty LCP neighbour counts as 0 (LCP[1] = LCP[n+1] = 0).
 *
 * Pins that tie this file to the paper and to mathematics rather than to
 * itself live in tests/test_oracle_pins.py.  Not thread-safe (the suffix
 * sorts use file-scope state for qsort's comparator).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ misc */

int oracle_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
    return omp_get_max_threads();
#else
    (void)t;
    return 1;
#endif
}

/* -------------------------------------------- Section 2-3: suffix array */

static const uint8_t *g_s;   /* text of the sort in progress */
static int64_t g_n;          /* its length */

/* Section 2's order: compare byte by byte; a proper prefix is smaller. */
static int cmp_suffix(const void *pa, const void *pb)
{
    int64_t i = *(const int32_t *)pa, j = *(const int32_t *)pb;
    int64_t li = g_n - i, lj = g_n - j;
    int c = memcmp(g_s + i, g_s + j, (size_t)(li < lj ? li : lj));
    if (c) return c;
    return li < lj ? -1 : (li > lj ? 1 : 0);
}

/* SA by sorting all suffixes directly (Section 3's definition). */
int oracle_sa_naive(const uint8_t *s, int64_t n, int32_t *sa)
{
    if (n < 0 || (n > 0 && (!s || !sa))) return -1;
    for (int64_t i = 0; i < n; i++) sa[i] = (int32_t)i;
    g_s = s; g_n = n;
    qsort(sa, (size_t)n, sizeof(int32_t), cmp_suffix);
    return 0;
}

static const int32_t *g_rank;
static int64_t g_h;

static int cmp_pair(const void *pa, const void *pb)
{
    int64_t i = *(const int32_t *)pa, j = *(const int32_t *)pb;
    if (g_rank[i] != g_rank[j]) return g_rank[i] < g_rank[j] ? -1 : 1;
    int64_t ri = i + g_h < g_n ? g_rank[i + g_h] : -1;
    int64_t rj = j + g_h < g_n ? g_rank[j + g_h] : -1;
    return ri < rj ? -1 : (ri > rj ? 1 : 0);
}

/*
 * SA by prefix doubling (Manber-Myers): after the round with step h every
 * suffix is ranked by its first 2h characters, by sorting the pairs
 * (rank[i], rank[i+h]) with a missing second half ranked lowest.  Used where
 * the direct sort is too slow (very long repeats); tests check that both
 * sorts agree.
 */
int oracle_sa_doubling(const uint8_t *s, int64_t n, int32_t *sa)
{
    if (n < 0 || (n > 0 && (!s || !sa))) return -1;
    if (n == 0) return 0;
    int32_t *rank = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *tmp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!rank || !tmp) { free(rank); free(tmp); return -2; }
    for (int64_t i = 0; i < n; i++) { sa[i] = (int32_t)i; rank[i] = s[i]; }
    g_n = n; g_rank = rank;
    for (int64_t h = 1;; h <<= 1) {
        g_h = h;
        qsort(sa, (size_t)n, sizeof(int32_t), cmp_pair);
        tmp[sa[0]] = 0;
        for (int64_t r = 1; r < n; r++)
            tmp[sa[r]] = tmp[sa[r - 1]] + (cmp_pair(&sa[r - 1], &sa[r]) != 0);
        memcpy(rank, tmp, (size_t)n * sizeof(int32_t));
        if (rank[sa[n - 1]] == n - 1 || h >= n) break;
    }
    free(rank); free(tmp);
    return 0;
}

/* Rank is the inverse of SA (Section 3). */
int oracle_rank(const int32_t *sa, int64_t n, int32_t *rank)
{
    for (int64_t r = 0; r < n; r++) rank[sa[r]] = (int32_t)r;
    return 0;
}

/*
 * LCP[0..n] (n+1 entries): LCP[r] = lcp(suffix SA[r-1], suffix SA[r]) for
 * 1 <= r <= n-1 and LCP[0] = LCP[n] = 0 (Section 3; the paper's LCP[1] and
 * LCP[n+1]).  Computed with Kasai et al.'s method, which the paper cites for
 * the LCP step (Theorem 1): walking positions in text order, the lcp with the
 * preceding suffix drops by at most one from i to i+1.
 */
int oracle_lcp_kasai(const uint8_t *s, int64_t n, const int32_t *sa,
                     const int32_t *rank, int32_t *lcp)
{
    lcp[0] = 0;
    lcp[n] = 0;
    int64_t h = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t r = rank[i];
        if (r == 0) { h = 0; continue; }
        int64_t j = sa[r - 1];
        while (i + h < n && j + h < n && s[i + h] == s[j + h]) h++;
        lcp[r] = (int32_t)h;
        if (h > 0) h--;
    }
    return 0;
}

/* Lemma 1: |LLR_i| = max(LCP[Rank[i]], LCP[Rank[i]+1]); 0 means no LLR_i. */
int oracle_llr_lengths(const int32_t *rank, const int32_t *lcp, int64_t n, int32_t *L)
{
    for (int64_t i = 0; i < n; i++) {
        int32_t a = lcp[rank[i]], b = lcp[rank[i] + 1];
        L[i] = a > b ? a : b;
    }
    return 0;
}

/*
 * |LLR_i| straight from its meaning in Lemma 1's proof: the longest common
 * prefix of suffix i with any other suffix, found by comparing suffix i with
 * every other suffix.  O(n * lcp) per position; used for sampled checks on
 * strings too long for the full pipeline above.
 */
int oracle_llr_direct(const uint8_t *s, int64_t n, const int64_t *idx, int64_t m, int32_t *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < m; q++) {
        int64_t i = idx[q], best = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            int64_t h = 0;
            while (i + h < n && j + h < n && s[i + h] == s[j + h]) h++;
            if (h > best) best = h;
        }
        out[q] = (int32_t)best;
    }
    return 0;
}

/* ------------------------------- Section 4.1: LRs from the raw LLR array */

/* Right end of LLR_i; an empty LLR_i (L_i = 0) "ends" at i - 1. */
static int64_t llr_end(const int32_t *L, int64_t i)
{
    return i + (int64_t)L[i] - 1;
}

/*
 * The LLRs that cover k.  Every LR is an LLR (Lemma 3), so LR_k is a longest
 * LLR covering k (Definition 1), and LLR_i covers k iff i <= k <= end_i.  By
 * Lemma 2 (L_i <= L_{i+1} + 1) the right ends never decrease in i, so the
 * covering LLRs are exactly the indices [lo, k] with lo the first i whose end
 * reaches k: found here by binary search.  Empty (lo = k + 1) iff L_k = 0.
 */
static int64_t covering_lo(const int32_t *L, int64_t k)
{
    int64_t lo = 0, hi = k + 1;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (llr_end(L, mid) >= k) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/*
 * Leftmost LR of every position from the raw LLR array (the result of
 * Algorithm 1): the longest covering LLR, the smallest start on ties (the
 * first maximum of a left-to-right scan of [lo, k]).
 */
int oracle_lr_leftmost_raw(const int32_t *L, int64_t n, int32_t *out /* 2n */)
{
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t k = 0; k < n; k++) {
        int32_t bs = -1, bl = 0;
        for (int64_t i = covering_lo(L, k); i <= k; i++)
            if (L[i] > bl) { bs = (int32_t)i; bl = L[i]; }
        out[2 * k] = bs;
        out[2 * k + 1] = bl;
    }
    return 0;
}

/*
 * All LRs of every position from the raw LLR array (the result of
 * Algorithm 3): every covering LLR of the maximal covering length, in
 * ascending start.  offsets has n+1 entries; rec holds (start, length)
 * pairs.  Returns the total record count; rec is written only when
 * cap >= total.
 */
int64_t oracle_lr_all_raw(const int32_t *L, int64_t n, int64_t *offsets,
                          int32_t *rec, int64_t cap)
{
    offsets[0] = 0;
    int32_t *len = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t *from = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t k = 0; k < n; k++) {
        int64_t lo = covering_lo(L, k);
        int32_t m = 0;
        for (int64_t i = lo; i <= k; i++)
            if (L[i] > m) m = L[i];
        int64_t c = 0;
        for (int64_t i = lo; i <= k; i++)
            c += (m > 0 && L[i] == m);
        len[k] = m;
        from[k] = lo;
        offsets[k + 1] = c;
    }
    for (int64_t k = 0; k < n; k++) offsets[k + 1] += offsets[k];
    int64_t total = offsets[n];
    if (rec && cap >= total) {
#pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t k = 0; k < n; k++) {
            int64_t w = offsets[k];
            for (int64_t i = from[k]; i <= k && len[k] > 0; i++)
                if (L[i] == len[k]) { rec[2 * w] = (int32_t)i; rec[2 * w + 1] = len[k]; w++; }
        }
    }
    free(len); free(from);
    return total;
}

/*
 * The same answers in O(n + output) for strings whose LLRs are very long
 * (where the walks above cost O(alpha n) with huge alpha).  By Lemma 2 the
 * right ends i + L_i - 1 never decrease, so the LLRs covering k are exactly
 * the indices [lo(k), k] with lo(k) non-decreasing in k (empty if L_k = 0):
 * a sliding window.  A monotone deque of indices with non-increasing L
 * (equal values kept, so the front is the leftmost maximum and all maxima
 * form the leading run) gives the textbook sliding-window maximum.
 * Leftmost mode if offsets is NULL (out gets 2n ints); otherwise all mode in
 * CSR as in oracle_lr_all_raw.
 */
int64_t oracle_lr_window(const int32_t *L, int64_t n, int32_t *out,
                         int64_t *offsets, int32_t *rec, int64_t cap)
{
    int64_t *dq = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t head = 0, tail = 0, lo = 0, total = 0;
    if (offsets) offsets[0] = 0;
    for (int64_t k = 0; k < n; k++) {
        while (tail > head && L[dq[tail - 1]] < L[k]) tail--;
        dq[tail++] = k;
        while (lo <= k && lo + (int64_t)L[lo] - 1 < k) lo++;
        while (tail > head && dq[head] < lo) head++;
        int empty = (lo > k);
        if (!offsets) {
            out[2 * k] = empty ? -1 : (int32_t)dq[head];
            out[2 * k + 1] = empty ? 0 : L[dq[head]];
        } else {
            if (!empty) {
                int32_t mx = L[dq[head]];
                for (int64_t q = head; q < tail && L[dq[q]] == mx; q++) {
                    if (rec && total < cap) { rec[2 * total] = (int32_t)dq[q]; rec[2 * total + 1] = mx; }
                    total++;
                }
            }
            offsets[k + 1] = total;
        }
    }
    free(dq);
    return total;
}

/* ----------------------------------------- Section 4.2: compact LLR array */

/*
 * The compact LLR array (Section 4.2): the useful LLRs, those that are not a
 * substring of another LLR, as (start, length) pairs in increasing start.  A
 * later LLR_j (j > i) starts after LLR_i and cannot contain it; an earlier
 * one ends at or before end_{i-1} (Lemma 2: right ends never decrease), so
 * LLR_i is contained in some other LLR iff it is contained in LLR_{i-1}, i.e.
 * iff end_i <= end_{i-1}.  Keep i iff L_i > 0 and (i = 0 or end_i > end_{i-1}).
 * Returns the number of entries.
 */
int64_t oracle_compact(const int32_t *L, int64_t n, int32_t *rec)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++) {
        int useful = L[i] > 0 && (i == 0 || llr_end(L, i) > llr_end(L, i - 1));
        if (useful) { rec[2 * m] = (int32_t)i; rec[2 * m + 1] = L[i]; m++; }
    }
    return m;
}

/*
 * BinarySearch(LLRc, k) of Algorithm 2: the smallest index of an entry that
 * covers k, or -1.  Ends strictly increase, so this is the first entry with
 * end >= k, provided its start is <= k.
 */
static int64_t first_covering(const int32_t *c, int64_t m, int64_t k)
{
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if ((int64_t)c[2 * mid] + c[2 * mid + 1] - 1 >= k) hi = mid; else lo = mid + 1;
    }
    if (lo < m && c[2 * lo] <= k) return lo;
    return -1;
}

/* Algorithm 2 (leftmost): binary search, then walk right while start <= k. */
int oracle_lr_leftmost_compact(const int32_t *c, int64_t m, int64_t n, int32_t *out)
{
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t k = 0; k < n; k++) {
        int32_t bs = -1, bl = 0;
        int64_t t0 = first_covering(c, m, k);
        if (t0 >= 0)
            for (int64_t t = t0; t < m; t++) {
                if (c[2 * t] > k) break;
                if (c[2 * t + 1] > bl) { bs = c[2 * t]; bl = c[2 * t + 1]; }
            }
        out[2 * k] = bs;
        out[2 * k + 1] = bl;
    }
    return 0;
}

/* Algorithm 4 (all): two walks from the binary-search result; CSR output. */
int64_t oracle_lr_all_compact(const int32_t *c, int64_t m, int64_t n,
                              int64_t *offsets, int32_t *rec, int64_t cap)
{
    offsets[0] = 0;
    for (int64_t k = 0; k < n; k++) {
        int64_t t0 = first_covering(c, m, k), cnt = 0;
        if (t0 >= 0) {
            int32_t length = 0;
            for (int64_t t = t0; t < m && c[2 * t] <= k; t++)
                if (c[2 * t + 1] > length) length = c[2 * t + 1];
            for (int64_t t = t0; t < m && c[2 * t] <= k; t++)
                if (c[2 * t + 1] == length) {
                    int64_t w = offsets[k] + cnt;
                    if (rec && w < cap) { rec[2 * w] = c[2 * t]; rec[2 * w + 1] = length; }
                    cnt++;
                }
        }
        offsets[k + 1] = offsets[k] + cnt;
    }
    return offsets[n];
}

/* -------------------------------------- Definition 1, by brute force */

/* Is S[i..i+len) a repeat, i.e. does it also start at some i' != i? */
static int is_repeat(const uint8_t *s, int64_t n, int64_t i, int64_t len)
{
    for (int64_t j = 0; j + len <= n; j++)
        if (j != i && memcmp(s + i, s + j, (size_t)len) == 0) return 1;
    return 0;
}

/*
 * Definition 1 and the problem statement of Section 2, by enumeration: for
 * each k try lengths from n-1 down and report every start of a repeat of
 * that length covering k.  Overlapping occurrences count.  Tiny n only.
 * CSR output as in oracle_lr_all_raw; (-1, 0) is not written (an empty list
 * means LR_k does not exist).
 */
int64_t oracle_lr_brute(const uint8_t *s, int64_t n, int64_t *offsets,
                        int32_t *rec, int64_t cap)
{
    int64_t total = 0;
    offsets[0] = 0;
    for (int64_t k = 0; k < n; k++) {
        for (int64_t len = n - 1; len >= 1; len--) {
            int64_t found = 0;
            int64_t i0 = k - len + 1 > 0 ? k - len + 1 : 0;
            for (int64_t i = i0; i <= k && i + len <= n; i++)
                if (is_repeat(s, n, i, len)) {
                    if (rec && total < cap) { rec[2 * total] = (int32_t)i; rec[2 * total + 1] = (int32_t)len; }
                    total++;
                    found++;
                }
            if (found) break;
        }
        offsets[k + 1] = total;
    }
    return total;
}
