// lrq_host.cpp -- host-side parts of liblrq: error reporting, scratch sizing,
// and the suffix-array builder that feeds the GPU path.
//
// The paper builds SA, Rank and LCP on the host and excludes them from its
// timings (Section 5 opening; Section 6, "Measurements"); its cited linear-time
// construction is not specified further.  This file builds SA by induced
// sorting (SA-IS: Nong, Zhang and Chan, "Two efficient algorithms for linear
// time suffix array construction", IEEE Trans. Computers 2011), written from
// that paper's description.  Rank and LCP are then computed on the GPU.

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lrq.h"
#include "lrq_internal.h"

namespace lrq {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

// Per calling thread: threads that drive the library concurrently (a build
// thread beside a query thread) never see each other's setting.
Tuning &tuning() {
    static thread_local Tuning t;
    return t;
}

bool tuning_valid(const Tuning &t) {
    return (t.plcp_chunk == 8 || t.plcp_chunk == 16 || t.plcp_chunk == 32) &&
           (t.llr_waves == 4 || t.llr_waves == 8) &&
           (t.lr_tile == 1024 || t.lr_tile == 2048 || t.lr_tile == 4096) &&
           (t.fuse_filter == 0 || t.fuse_filter == 1);
}

namespace {

// ---- SA-IS ------------------------------------------------------------------
//
// Suffix i is S-type if it is smaller than suffix i+1, L-type otherwise; the
// last suffix is L-type because the (virtual) end-of-string marker after it is
// the smallest symbol.  An LMS position is an S-type position preceded by an
// L-type one.  Sorting the LMS suffixes fixes the order of every other suffix by
// two induction passes over the buckets (first character classes): L-type
// suffixes fill bucket heads left to right, S-type suffixes fill bucket tails
// right to left.  The LMS suffixes themselves are sorted by naming the sorted
// LMS substrings and, when names repeat, recursing on the string of names.

template <class Ch>
void sais(const Ch *s, int32_t *sa, int64_t n, int64_t K) {
    if (n <= 0) return;
    if (n == 1) { sa[0] = 0; return; }
    std::vector<uint8_t> stype(n);
    stype[n - 1] = 0;
    for (int64_t i = n - 2; i >= 0; --i)
        stype[i] = (s[i] < s[i + 1]) || (s[i] == s[i + 1] && stype[i + 1]);
    auto is_lms = [&](int64_t i) { return i > 0 && stype[i] && !stype[i - 1]; };

    std::vector<int64_t> bucket(K + 1, 0);
    for (int64_t i = 0; i < n; ++i) bucket[int64_t(s[i]) + 1]++;
    for (int64_t c = 0; c < K; ++c) bucket[c + 1] += bucket[c];
    std::vector<int64_t> ptr(K);
    auto heads = [&] { for (int64_t c = 0; c < K; ++c) ptr[c] = bucket[c]; };
    auto tails = [&] { for (int64_t c = 0; c < K; ++c) ptr[c] = bucket[c + 1]; };

    auto induce = [&] {
        heads();
        sa[ptr[s[n - 1]]++] = int32_t(n - 1);  // induced by the end marker
        for (int64_t r = 0; r < n; ++r) {
            const int64_t j = int64_t(sa[r]) - 1;
            if (sa[r] > 0 && !stype[j]) sa[ptr[s[j]]++] = int32_t(j);
        }
        tails();
        for (int64_t r = n - 1; r >= 0; --r) {
            const int64_t j = int64_t(sa[r]) - 1;
            if (sa[r] > 0 && stype[j]) sa[--ptr[s[j]]] = int32_t(j);
        }
    };

    // Stage 1: LMS positions at their bucket tails (any order), then induce:
    // this sorts the LMS substrings.
    std::fill(sa, sa + n, -1);
    tails();
    std::vector<int32_t> lms;
    for (int64_t i = 1; i < n; ++i)
        if (is_lms(i)) lms.push_back(int32_t(i));
    for (int64_t q = int64_t(lms.size()) - 1; q >= 0; --q) sa[--ptr[s[lms[q]]]] = lms[q];
    induce();
    const int64_t m = int64_t(lms.size());
    if (m == 0) return;  // no LMS suffix: the induction already sorted everything

    // Stage 2: name the LMS substrings in sorted order.
    std::vector<int32_t> sorted;
    sorted.reserve(m);
    for (int64_t r = 0; r < n; ++r)
        if (is_lms(sa[r])) sorted.push_back(sa[r]);
    auto same_substring = [&](int64_t a, int64_t b) {
        for (int64_t d = 0;; ++d) {
            if (a + d == n || b + d == n) return false;  // the end marker is unique
            if (s[a + d] != s[b + d] || stype[a + d] != stype[b + d]) return false;
            if (d > 0 && (is_lms(a + d) || is_lms(b + d))) return is_lms(a + d) && is_lms(b + d);
        }
    };
    std::vector<int32_t> name(n, -1);
    int64_t names = 0;
    for (int64_t q = 0; q < m; ++q) {
        if (q == 0 || !same_substring(sorted[q - 1], sorted[q])) ++names;
        name[sorted[q]] = int32_t(names - 1);
    }

    // Stage 3: order of the LMS suffixes, by recursion when names repeat.
    std::vector<int32_t> reduced(m), order(m);
    for (int64_t q = 0; q < m; ++q) reduced[q] = name[lms[q]];
    if (names < m) {
        sais(reduced.data(), order.data(), m, names);
    } else {
        for (int64_t q = 0; q < m; ++q) order[reduced[q]] = int32_t(q);
    }

    // Stage 4: sorted LMS suffixes at their bucket tails, then induce.
    std::fill(sa, sa + n, -1);
    tails();
    for (int64_t q = m - 1; q >= 0; --q) {
        const int32_t p = lms[order[q]];
        sa[--ptr[s[p]]] = p;
    }
    induce();
}

}  // namespace
}  // namespace lrq

using namespace lrq;

extern "C" {

int lrq_version(void) { return LRQ_API_VERSION; }

const char *lrq_status_str(int status) {
    switch (status) {
        case LRQ_OK: return "ok";
        case LRQ_EINVAL: return "invalid argument";
        case LRQ_ERANGE: return "size out of range";
        case LRQ_ENOSPC: return "buffer too small for the result";
        case LRQ_ENOMEM: return "scratch buffer too small";
        case LRQ_EDEVICE: return "HIP device error";
        case LRQ_EDATA: return "device-side input check failed";
        default: return "unknown status";
    }
}

const char *lrq_last_error(void) { return g_err.c_str(); }

int lrq_scratch_bytes(int64_t total, int32_t nseg, size_t *bytes) {
    clear_error();
    if (!bytes) { set_error("bytes is NULL"); return LRQ_EINVAL; }
    if (total < 0 || nseg < 1) { set_error("total < 0 or nseg < 1"); return LRQ_EINVAL; }
    if (total > LRQ_MAX_TOTAL) { set_error("total > LRQ_MAX_TOTAL"); return LRQ_ERANGE; }
    *bytes = scratch_bytes_any(total, nseg);
    return LRQ_OK;
}

int lrq64_scratch_bytes(int64_t total, int32_t nseg, size_t *bytes) {
    clear_error();
    if (!bytes) { set_error("bytes is NULL"); return LRQ_EINVAL; }
    if (total < 0 || nseg < 1) { set_error("total < 0 or nseg < 1"); return LRQ_EINVAL; }
    if (total > LRQ64_MAX_TOTAL) { set_error("total > LRQ64_MAX_TOTAL"); return LRQ_ERANGE; }
    *bytes = scratch_bytes_any(total, nseg);
    return LRQ_OK;
}

int lrq_set_tuning(const lrq_tuning *t) {
    clear_error();
    Tuning tu;
    if (t) {
        tu.plcp_chunk = t->plcp_chunk;
        tu.llr_waves = t->llr_waves;
        tu.lr_tile = t->lr_tile;
        tu.fuse_filter = t->fuse_filter;
    }
    if (!tuning_valid(tu)) {
        set_error("unsupported tuning (plcp_chunk %d, llr_waves %d, lr_tile %d, fuse_filter %d)",
                  tu.plcp_chunk, tu.llr_waves, tu.lr_tile, tu.fuse_filter);
        return LRQ_EINVAL;
    }
    tuning() = tu;
    return LRQ_OK;
}

int lrq_get_tuning(lrq_tuning *t) {
    clear_error();
    if (!t) { set_error("NULL argument"); return LRQ_EINVAL; }
    t->plcp_chunk = tuning().plcp_chunk;
    t->llr_waves = tuning().llr_waves;
    t->lr_tile = tuning().lr_tile;
    t->fuse_filter = tuning().fuse_filter;
    return LRQ_OK;
}

int lrq_build_sa_host(const uint8_t *h_text, int64_t n, int32_t *h_sa) {
    clear_error();
    if (n < 0) { set_error("n < 0"); return LRQ_EINVAL; }
    if (n > LRQ_MAX_TOTAL) { set_error("n > LRQ_MAX_TOTAL"); return LRQ_ERANGE; }
    if (n == 0) return LRQ_OK;
    if (!h_text || !h_sa) { set_error("NULL argument"); return LRQ_EINVAL; }
    try {
        sais(h_text, h_sa, n, 256);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed in SA construction");
        return LRQ_ENOMEM;
    }
    return LRQ_OK;
}

int lrq_build_sa_host_batch(const uint8_t *h_text, const int64_t *h_seg_off, int32_t nseg,
                            int32_t *h_sa) {
    clear_error();
    if (nseg < 1 || !h_seg_off) { set_error("nseg < 1 or h_seg_off NULL"); return LRQ_EINVAL; }
    if (h_seg_off[0] != 0) { set_error("h_seg_off[0] != 0"); return LRQ_EINVAL; }
    for (int32_t b = 0; b < nseg; ++b)
        if (h_seg_off[b + 1] < h_seg_off[b]) { set_error("h_seg_off decreases at %d", b); return LRQ_EINVAL; }
    const int64_t total = h_seg_off[nseg];
    if (total > LRQ_MAX_TOTAL) { set_error("total > LRQ_MAX_TOTAL"); return LRQ_ERANGE; }
    if (total > 0 && (!h_text || !h_sa)) { set_error("NULL argument"); return LRQ_EINVAL; }
    int failed = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : failed)
    for (int32_t b = 0; b < nseg; ++b) {
        try {
            sais(h_text + h_seg_off[b], h_sa + h_seg_off[b], h_seg_off[b + 1] - h_seg_off[b], 256);
        } catch (const std::bad_alloc &) {
            failed |= 1;
        }
    }
    if (failed) { set_error("host allocation failed in SA construction"); return LRQ_ENOMEM; }
    return LRQ_OK;
}

}  // extern "C"
